#!/usr/bin/env python3
"""Benchmark of the MGAR topology-optimisation hot path on one MI355X.

A step is one optimisation cycle of the 128^3 trilinear-hex heat-conduction
problem: density filter, SIMP conductivity, the solve (MGAR reanalysis with
MGCG fallback, or plain MGCG for the reference loop) to relative residual
1e-8, compliance and sensitivities, and the OC update. All inputs live in HBM
before the timed region. Warmup steps run the first cycles of the loop (the
cycles below N_on use MGCG in both loops); the timed steps continue it.

Prints one JSON line:
  value          DOF-solves/s of the MGAR loop (free DOFs x solves / second)
  ms_per_step    MGAR loop, milliseconds per optimisation cycle
  mgcg           the same figures for the plain-MGCG loop on the same GPU
  batched        48 2D + 8 3D designs of uneven sizes solved together (FP64),
                 with the block size of its launches from the batch tuner
                 (tuned_block, block_us), against the same solves one design
                 at a time; batched.mixed
                 the same in the mixed-precision form (FP32 multigrid over
                 BF16 densities, FP32 inner PCG runs with FP64 residual
                 replacement, same 1e-8 FP64 residual test)
  learned_mixed  the mixed-precision MGAR loop with the learned initial guess
                 (the 4-level 16/32/64/64-channel U-Net on the element grid,
                 trained by the library's kernels with 40 Adam steps over the
                 pairs of cycles 2..20, in the background on its own stream
                 during cycles 21..45, evaluated from 46 and used
                 when its true residual beats the previous temperature's;
                 after a losing cycle the guess is left out for 1, 2, 4 ..
                 16 cycles, a win resets the gap); training time is inside
                 the timed cycles, which are always N_on..maxit (10..80 at
                 128^3) whatever --steps says
  seed_network   that U-Net alone at the workload's size: inference and one
                 training step (events), convolution rate against the dense
                 BF16 matrix-core peak (2.5 PFLOP/s)
  mgar_mixed     the MGAR loop in the mixed-precision form (one FP32 PCG run,
                 FP32 multigrid over BF16 densities, its residual replaced by
                 the FP64 one every 1e-3 of reduction, same 1e-8 FP64 residual
                 test); reported beside value, which stays the all-FP64 loop
  paper_setting  the MGAR and plain-MGCG loops again in the paper's solver
                 settings (reconstruction criterion eps1 = 0.5, MGCG accuracy
                 eps2 = 1e-6), same workload and cycles: s/opt-iter, paths,
                 efficiency improvement 1 - t_MGAR / t_MGCG (the paper's
                 measure) and the relative difference of the final objectives;
                 always over cycles N_on..maxit (10..80 at 128^3)
  roofline       the finest-grid stencil kernel named there: algorithmic bytes
                 per launch / average launch time from HIP events recorded at
                 the start and end of each launch in the timed cycles, against
                 8 TB/s; stream_ref gives, for scale, the GB/s of plain torch
                 element-wise kernels at the node-vector size and at 64 Mi
                 elements (beyond the Infinity Cache); effective gives the
                 GB/s of one whole V-cycle and one whole PCG iteration with the
                 bytes of their unfused definitions
  paper_tables   (with --paper-tables) the paper's Table 2 and 3 experiments
                 in its own solver settings with continuous filtering: MGCG
                 evaluations, CG iterations, efficiency improvement and
                 objective differences beside the paper's figures
  oversize_control  (with --oversize N) FP64 MGCG solves on an N^3 grid whose
                 vectors exceed the Infinity Cache: the same kernel's rate,
                 time per PCG iteration, DOF-solves/s
  cpu_baseline   the CPU oracle (NumPy/SciPy, FP64) timed on one full MGCG
                 solve of the same grid
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# finest-grid stencil kernel reported in the roofline object (mode bit of mgar_profile)
ROOF_MODE = 1          # apply + dot: q = K p, p.q  (one launch per CG iteration, finest grid only)
# kernel that runs a launch shape {kind, kz, zd, ntx} (kind 0: node-parallel,
# 1: z-marching, 2: two-row z-marching)
SHAPE_KERNEL = {0: "k_stencil_b", 1: "k_stencil_z", 2: "k_stencil_z2"}


def roof_kernel(shape):
    if shape[0] == 2:   # two-row shapes run the CG direction update inside the apply
        return (f"k_stencil_z2<SM_PAPPLY_DOT> shape {shape} "
                "(finest grid: p = z + beta p_old stored, q = K p, p.q)")
    return (f"{SHAPE_KERNEL.get(shape[0], '?')}<SM_APPLY_DOT> shape {shape} "
            "(finest grid, q = K p with p.q)")


COUNTERS = os.path.join(ROOT, "profiles", "stencil_apply_dot_128cube.md")
STENCIL_SRC = os.path.join(ROOT, "paper_2210_00947_amd", "csrc", "stencil.hip")


ZBUF_SRC = os.path.join(ROOT, "paper_2210_00947_amd", "csrc", "zbuf.h")


def _definition(text, head):
    """Source text of the definition that starts with `head`, up to the first
    closing brace at the start of a line."""
    i = text.index(head)
    return text[i:text.index("\n}\n", i) + 3]


def roof_kernel_source_sha():
    """SHA-256 over the source the roofline kernel is compiled from: the
    definition of k_stencil_z2, the node formula apply27g and the buffer-load
    helpers (zbuf.h). Edits elsewhere in the stencil file leave it unchanged."""
    import hashlib
    text = open(STENCIL_SRC).read()
    parts = [_definition(text, "template <int MODE, int ZD, typename T, typename CL>\n__global__ __launch_bounds__(ZT) "
                               "void k_stencil_z2("),
             _definition(text, "template <typename T, bool NEEDX, typename FA, typename FB, typename FC, typename GA, "
                               "typename GB>\n__device__ inline T apply27g("),
             open(ZBUF_SRC).read()]
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()


def committed_traffic(shape):
    """HBM traffic per launch of the roofline kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, or None when the kernel's source
    (roof_kernel_source_sha) has changed since they were taken, when they were
    taken on another launch shape, or when they are missing."""
    try:
        src = roof_kernel_source_sha()
        for line in open(COUNTERS):
            line = line.strip()
            if not line.startswith("counters:"):
                continue
            kv = dict(f.split("=", 1) for f in line.split()[1:])
            if kv.get("source_sha256") != src or kv.get("shape") != ",".join(map(str, shape)):
                return None
            return (float(kv["fetch_kib"]) + float(kv["write_kib"])) * 1024.0 * float(kv.get("scale", 1.0))
    except (OSError, ValueError, KeyError):
        return None
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_loop(prob, use_mgar, warmup, steps, W, TopOpt, torch, precision=0, seed=None, roof_cycles=0,
             eps_accept=None):
    """Warm-up cycles, then `steps` timed cycles. The roofline kernel is timed
    with HIP events recorded at the start and end of each of its launches:
    over the timed cycles (roof_cycles = 0, the default; kernels are launched
    eagerly, the library's default), or on roof_cycles further cycles (for
    runs that replay captured PCG iterations, where kernel timing cannot run)."""
    opt = TopOpt(prob, W.element_source(prob), use_mgar=use_mgar, precision=precision, seed=seed,
                 eps_accept=eps_accept)
    for _ in range(warmup):
        opt.step()
    if roof_cycles == 0:
        opt.h.mgar_profile(1 << ROOF_MODE)
        opt.h.mgar_profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [opt.step() for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n, ms, by = 0, 0.0, 0.0
    if roof_cycles == 0:
        n, ms, by = opt.h.mgar_profile_read()
        opt.h.mgar_profile(0)
    else:
        opt.h.mgar_profile(1 << ROOF_MODE)
        opt.h.mgar_profile_read()
        for _ in range(roof_cycles):
            opt.step()
        torch.cuda.synchronize()
        n, ms, by = opt.h.mgar_profile_read()
        opt.h.mgar_profile(0)
    el = t1 - t0
    roof_shape = opt.h.mgar_tune_get(0, 0, ROOF_MODE)
    paths = {"mgcg": 0, "accept": 0, "fallback": 0}
    for r in recs:
        paths[["mgcg", "accept", "fallback"][r.path]] += 1
    out = {
        "tuned_shapes": opt.tune_source,
        "elapsed_s": el,
        "s_per_opt_iter": el / steps,
        "cg_iters_mean": sum(r.cg_iters for r in recs) / steps,
        "refinements_mean": sum(r.refinements for r in recs) / steps,
        "seed_used_cycles": sum(r.seed_used for r in recs),
        "seed_evaluated_cycles": sum(r.res_seed == r.res_seed for r in recs),
        "paths": paths,
        "final_compliance": recs[-1].compliance,
        "kernel_launches": n,
        "kernel_ms_total": ms,
        "kernel_bytes_total": by,
        "roof_shape": roof_shape,
    }
    opt.h.close()
    return out


def run_batched(W, M, torch, nsolves=5, precision=None):
    """The batched workload (48 2D + 8 3D designs of uneven sizes): `nsolves`
    batched MGCG solves from T0 = 0 on reseeded densities, then the same
    solves one design at a time through single-design handles on the same
    GPU, and one batched reanalysis step (MGCG at x, MGAR at a perturbed x).
    precision: M.PREC_FP64 (default) or M.PREC_MIXED, for the batch and the
    single-design handles alike."""
    import numpy as np
    prec = M.PREC_FP64 if precision is None else precision
    probs = W.batched_designs()
    b = M.Batch([M.params_for(p, precision=prec) for p in probs])
    free = 0
    for p in probs:
        nfix = 1
        for a in range(p.dim):
            nfix *= p.fix_hi[a] - p.fix_lo[a] + 1
        free += p.nnodes - nfix

    def cat(arrs, off):
        out = np.zeros(off[-1])
        for i, a in enumerate(arrs):
            out[off[i]:off[i + 1]] = a
        return torch.as_tensor(out, dtype=torch.float64, device="cuda")

    q = torch.empty(b.N, dtype=torch.float64, device="cuda")
    b.mgar_batch_load_vector(cat([W.element_source(p) for p in probs], b.elem_off), q)
    xs = [cat([W.reseeded_density(p, 31 * r + i) for i, p in enumerate(probs)], b.elem_off)
          for r in range(nsolves)]
    # block size of the batched launches from the tuner (timed on a density
    # set of its own, not one of the timed solves)
    xtune = cat([W.reseeded_density(p, 1000 + i) for i, p in enumerate(probs)], b.elem_off)
    block, block_us = b.mgar_batch_autotune(xtune, q, 1e-8, reps=3)
    T = torch.empty(b.N, dtype=torch.float64, device="cuda")
    b.mgcg_batch_solve(xs[0], q, None, 1e-8, T)       # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, refs = [], []
    for x in xs:
        st = b.mgcg_batch_solve(x, q, None, 1e-8, T)
        its.append(max(s["cg_iters"] for s in st))
        refs.append(max(s["refinements"] for s in st))
    torch.cuda.synchronize()
    bt = (time.perf_counter() - t0) / nsolves
    # MGAR step at a perturbed design (exact mode: every design falls back)
    x1 = cat([np.clip(W.reseeded_density(p, i) + 0.01 * W.random_vector(p.nelem, 77 + i), 0, 1)
              for i, p in enumerate(probs)], b.elem_off)
    T1 = torch.empty_like(T)
    b.mgcg_batch_solve(xs[0], q, None, 1e-8, T)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sa = b.mgar_batch_solve(x1, q, T, 1e-8, T1)
    torch.cuda.synchronize()
    at = time.perf_counter() - t1
    b.close()
    # the same MGCG solves, one design after another through single handles
    hs = [M.Handle(M.params_for(p, precision=prec)) for p in probs]
    qs, ts = [], []
    for p, h in zip(probs, hs):
        qi = torch.empty(p.nnodes, dtype=torch.float64, device="cuda")
        h.mgar_load_vector(torch.as_tensor(W.element_source(p), device="cuda"), qi)
        qs.append(qi)
        ts.append(torch.empty_like(qi))
    xsd = [[torch.as_tensor(W.reseeded_density(p, 31 * r + i), device="cuda") for i, p in enumerate(probs)]
           for r in range(nsolves)]
    for h, qi, ti, x in zip(hs, qs, ts, xsd[0]):
        h.mgcg_solve(x, qi, None, 1e-8, ti)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for r in range(nsolves):
        for h, qi, ti, x in zip(hs, qs, ts, xsd[r]):
            h.mgcg_solve(x, qi, None, 1e-8, ti)
    torch.cuda.synchronize()
    stime = (time.perf_counter() - t2) / nsolves
    for h in hs:
        h.close()
    return {
        "designs": len(probs), "free_dofs": free,
        "batched_mgcg_s_per_solve": bt, "batched_dof_solves_per_s": free / bt,
        "precision": "mixed" if prec == M.PREC_MIXED else "fp64",
        "max_cg_iters": its, "max_refinements": refs,
        "batched_mgar_s": at, "batched_mgar_paths": {"accept": sum(s["path"] == 1 for s in sa),
                                                     "fallback": sum(s["path"] == 2 for s in sa)},
        "one_by_one_mgcg_s_per_solve": stime, "one_by_one_dof_solves_per_s": free / stime,
        "speedup": stime / bt,
        "tuned_block": block, "block_us": {str(k): v for k, v in block_us.items()},
    }


# The paper's Table 2 (uniform source, volume fraction 0.5; PAPER sizes 360,
# 720, 1560, 2040 elements per side) and Table 3 (four-quadrant source, 480
# and 960, volume fractions 0.4 and 0.6) figures, for context next to the runs.
PAPER_TABLE2 = {360: (107, 0.4165, 0.0015), 720: (115, 0.3911, 0.00037), 1560: (125, 0.3518, 0.000040),
                2040: (127, 0.3410, 0.000033)}
PAPER_TABLE3 = {(480, 0.4): (7.71, 7.38, 112, 0.4050, 0.0013), (480, 0.6): (7.69, 7.32, 102, 0.4546, 0.000050),
                (960, 0.4): (7.81, 7.51, 124, 0.3593, 0.00028), (960, 0.6): (7.47, 7.24, 109, 0.4368, 0.000015)}


def paper_levels(n, min_coarse=4):
    """Grids of the paper-mode runs (n x n, sink on the middle tenth of the left
    side): the deepest hierarchy whose coarsest grid keeps at least min_coarse
    elements per side and a Dirichlet node (a coarse node is fixed when the
    finest node under it is). The coarsest inverse is built on one CU in
    O(nodes^3): 38 ms at 23^2 nodes, 343 ms at 31^2 on MI355X, so a deep
    hierarchy keeps that build out of the cycle time."""
    import workloads as W
    lo, hi = W.sink_box_2d(n, n)
    levels = 1
    while n % (1 << levels) == 0 and n >> levels >= min_coarse:
        s = 1 << levels
        if (hi[1] // s) * s < lo[1]:      # no multiple of the coarse spacing inside the sink
            break
        levels += 1
    return levels


def paper_tables(W, TopOpt, torch, ncycles=300):
    """The paper's experiments of Tables 2 and 3 in its solver settings (eps1 =
    0.5, eps2 = 1e-6, cg_max 200, m = 2, N_on = 40 of 300 cycles, continuous
    filtering from 1.4 L / 50 down to r_min = 3 over 250 cycles, source 1e-4
    per unit volume or the four-quadrant source): an MGAR loop and a pure MGCG
    loop per case, with the deepest hierarchy of each grid (paper_levels; the
    paper uses nl = 3, whose coarsest grids of 8k-260k nodes the dense
    coarsest solve here cannot take). Sizes: Table 2's 360, 720, 1560 and
    2040 elements per side allow only shallow hierarchies (360 = 8 x 45), so
    the nearest sizes with deep ones are run instead (352, 704, 1536, 2048;
    DOFs within 5 %); Table 3's 480 and 960 are run as printed. Reported
    per case: MGCG evaluations (pure-MGCG cycles plus rejected reductions),
    accepted reductions, mean CG iterations of MGAR's and of the pure MGCG
    loop, efficiency improvement 1 - t_MGAR / t_MGCG, relative difference of
    the final objectives, and the paper's figures."""
    cases = [("table2", n, 0.5, False, PAPER_TABLE2[p]) for n, p in ((352, 360), (704, 720), (1536, 1560),
                                                                     (2048, 2040))]
    cases += [("table3", n, vf, True, PAPER_TABLE3[(n, vf)]) for n in (480, 960) for vf in (0.4, 0.6)]
    out = []
    for table, n, vf, quad, paper in cases:
        prob = W.paper_2d(n, paper_levels(n), volfrac=vf, maxit=ncycles)
        qe = W.quadrant_source(prob) if quad else W.element_source(prob)
        res = {}
        for name, use_mgar in (("mgar", True), ("mgcg", False)):
            opt = TopOpt(prob, qe, use_mgar=use_mgar, eps_accept=0.5, cg_max=200, continuous={"r_min": 3.0})
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cyc = opt.run(ncycles)
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t0, cyc)
            opt.h.close()
        (ta, ca), (tc, cc) = res["mgar"], res["mgcg"]
        row = {"table": table, "n": n, "levels": prob.levels, "dofs": prob.nnodes, "volfrac": vf,
               "source": "quadrants" if quad else "uniform",
               "mgcg_evaluations": sum(c.path != 1 for c in ca), "accepted": sum(c.path == 1 for c in ca),
               "cg_iters_mgar": sum(c.cg_iters for c in ca) / max(1, sum(c.path != 1 for c in ca)),
               "cg_iters_mgcg": sum(c.cg_iters for c in cc) / ncycles,
               "s_mgar": ta, "s_mgcg": tc, "efficiency_improvement": 1.0 - ta / tc,
               "objective_rel_diff": abs(ca[-1].compliance - cc[-1].compliance) / abs(cc[-1].compliance)}
        if table == "table2":
            row["paper"] = {"size": {352: 360, 704: 720, 1536: 1560, 2048: 2040}[n], "mgcg_evaluations": paper[0],
                            "efficiency_improvement": paper[1], "objective_rel_diff": paper[2]}
        else:
            row["paper"] = {"cg_iters_mgar": paper[0], "cg_iters_mgcg": paper[1], "mgcg_evaluations": paper[2],
                            "efficiency_improvement": paper[3], "objective_rel_diff": paper[4]}
        log(f"[bench] paper {table} {n}^2 vf {vf}: MGCG evaluations {row['mgcg_evaluations']} "
            f"(paper {row['paper']['mgcg_evaluations']}), efficiency {100 * row['efficiency_improvement']:.1f} % "
            f"(paper {100 * row['paper']['efficiency_improvement']:.1f} %), objective diff "
            f"{100 * row['objective_rel_diff']:.4f} %")
        out.append(row)
    return out


def cpu_baseline(prob, W, nsolves=3):
    """Full oracle MGCG solves on the benchmark grid (FP64, SciPy), timed with
    perf_counter; cores = process CPU time / wall time (the oracle leaves
    the thread counts of NumPy/SciPy's native libraries at their defaults;
    the record lists them, the CPUs the process may run on and the thread
    environment variables)."""
    import numpy as np
    from oracle import solvers
    s = solvers.MgarSolver(prob, solvers.MgarParams(cg_max=200))
    c0 = time.process_time()
    t0 = time.perf_counter()
    its = []
    for r in range(nsolves):
        _, st = s.mgcg(W.reseeded_density(prob, r), np.zeros(prob.nnodes), prob.tol)
        its.append(st.cg_iters)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    free = int(s.fep.free.size)
    return {
        "value": free * nsolves / wall,
        "unit": "DOF-solves/s",
        "cores": max(1, int(round(cpu / wall))),
        "kind": "oracle",
        "sample": (f"{nsolves} oracle MGCG solves (assembled CSR K, {prob.levels}-level V-cycle, dense "
                   f"coarsest Cholesky) of the {prob.nelx}^3 grid from T0 = 0 at rel. residual "
                   f"{prob.tol:g}, densities uniform(0.3, 0.5) seeds 0..{nsolves - 1}; CG iterations "
                   f"{its}, {wall:.1f} s wall incl. assembly"),
        "seconds": wall,
        "cpu_model": _cpu_model(),
        "os_cpu_count": os.cpu_count(),
        "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
        "thread_env": {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                                       "MKL_NUM_THREADS", "BLIS_NUM_THREADS")},
        "blas_threadpools": _threadpools(),
    }


def _threadpools():
    """Thread pools of the native libraries NumPy/SciPy loaded (BLAS, OpenMP):
    library, API and thread count, as threadpoolctl reports them."""
    try:
        from threadpoolctl import threadpool_info
        return [{k: d.get(k) for k in ("internal_api", "prefix", "num_threads", "version")}
                for d in threadpool_info()]
    except Exception as e:   # threadpoolctl missing or failing: say so in the record
        return [{"error": str(e)}]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def effective_bandwidth(prob, W, TopOpt, torch, reps=50):
    """Effective HBM rates of whole solver pieces at the workload's size, with
    the algorithmic bytes of their unfused definitions (N = nodes, FP64):
    one V-cycle through mgar_vcycle (masked copy of b 16N + V-cycle 112N;
    back-to-back calls, so launch gaps are included) and one PCG iteration
    (V-cycle 112N + apply 24N + x/r update 48N + p update 24N = 208N; the
    marginal device time per iteration between timed MGCG solves from T0 = 0
    to rel. residuals 1e-2 and 1e-12, three of each, so set-up cancels)."""
    n = prob.nnodes
    opt = TopOpt(prob, W.element_source(prob), use_mgar=False, timing=True)
    opt.step()                       # K0 and its hierarchy from the first design
    f64 = dict(dtype=torch.float64, device="cuda")
    x = torch.empty(n, **f64)
    for _ in range(3):
        opt.h.mgar_vcycle(opt.q, None, x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        opt.h.mgar_vcycle(opt.q, None, x)
    e1.record()
    torch.cuda.synchronize()
    vc_us = e0.elapsed_time(e1) * 1e3 / reps
    ms = {1e-2: 0.0, 1e-12: 0.0}
    its = {}
    for _ in range(3):
        for tol in ms:
            st = opt.h.mgcg_solve(opt.xphys, opt.q, None, tol, x)
            ms[tol] += st["ms"] / 3
            its[tol] = st["cg_iters"]
    it_us = (ms[1e-12] - ms[1e-2]) * 1e3 / max(its[1e-12] - its[1e-2], 1)
    out = {}
    for name, by, us in (("vcycle", 128.0 * n, vc_us), ("pcg_iteration", 208.0 * n, it_us)):
        gbs = by / us / 1e3
        out[name] = {"bytes": by, "us": us, "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS}
    out["pcg_iteration"]["cg_iters"] = [its[1e-2], its[1e-12]]
    return out


def oversize_levels(n):
    """Grids of the oversize control: halve n until 4 elements per axis are
    left (5^3 coarsest nodes, as at 128^3), or until n is odd."""
    levels = 1
    while (n >> (levels - 1)) > 4 and (n >> (levels - 1)) % 2 == 0:
        levels += 1
    return levels


def oversize_control(W, M, torch, n, nsolves=3):
    """FP64 MGCG solves (T0 = 0, rel. residual 1e-8, uniform(0.3, 0.5)
    densities) on an n^3 grid whose vectors no longer fit the 256 MB
    Infinity Cache (n = 256: 16.98 M nodes, 136 MB per FP64 vector). Reports
    the roofline kernel's rate there (HIP events at kernel start and end over
    the timed solves), the time per PCG iteration with the 208N algorithmic
    bytes of its unfused definition, and DOF-solves/s."""
    from paper_2210_00947_amd import tune
    levels = oversize_levels(n)
    prob = W.make_3d(f"3d-{n}^3", n, levels, volfrac=0.3, filter_r=2.0, maxit=80, x_init=0.3)
    h = M.Handle(M.params_for(prob))
    tune.autotune(h, h.params, tune.device_arch())
    q = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgar_load_vector(torch.as_tensor(W.element_source(prob), device="cuda"), q)
    xs = [torch.as_tensor(W.reseeded_density(prob, r), device="cuda") for r in range(nsolves + 1)]
    T = torch.empty_like(q)
    h.mgcg_solve(xs[0], q, None, 1e-8, T)
    h.mgar_profile(1 << ROOF_MODE)
    h.mgar_profile_read()
    for x in xs[1:]:
        h.mgcg_solve(x, q, None, 1e-8, T)
    launches, kms, kby = h.mgar_profile_read()
    h.mgar_profile(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for x in xs[1:]:
        its += h.mgcg_solve(x, q, None, 1e-8, T)["cg_iters"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    shape = h.mgar_tune_get(0, 0, ROOF_MODE)
    h.close()
    nfix = 1
    for a in range(3):
        nfix *= prob.fix_hi[a] - prob.fix_lo[a] + 1
    free = prob.nnodes - nfix
    it_s = el / max(its, 1)
    gbs = kby / (kms * 1e-3) / 1e9 if kms > 0 else None
    return {"grid": f"{n}^3", "levels": levels, "nodes": prob.nnodes, "solves": nsolves,
            "ms_per_solve": el / nsolves * 1e3, "cg_iters_per_solve": its / nsolves,
            "dof_solves_per_s": free * nsolves / el,
            "pcg_iteration": {"us": it_s * 1e6, "bytes": 208.0 * prob.nnodes,
                              "GB/s": 208.0 * prob.nnodes / it_s / 1e9,
                              "frac": 208.0 * prob.nnodes / it_s / 1e9 / HBM_PEAK_GBS},
            "roof_kernel": {"kernel": roof_kernel(shape), "launches": launches,
                            "avg_launch_us": kms / max(launches, 1) * 1e3,
                            "bytes_per_launch": kby / max(launches, 1),
                            "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS if gbs else None}}


def stream_reference(torch, sizes, reps=30):
    """Context for the roofline fraction: what plain element-wise torch kernels
    (FP64; events around `reps` back-to-back launches after 5 warm-up ones)
    reach on this GPU, in GB/s of bytes read + written, for vectors of each
    size in `sizes` (elements): copy (1 read, 1 write), a + b (2, 1) and
    a + b * c (3, 1)."""
    out = {}
    for n in sizes:
        a, b, c, d = (torch.rand(n, dtype=torch.float64, device="cuda") for _ in range(4))
        row = {}
        for name, fn, nvec in (("copy", lambda: d.copy_(a), 2),
                               ("add", lambda: torch.add(a, b, out=d), 3),
                               ("fma", lambda: torch.addcmul(a, b, c, out=d), 4)):
            for _ in range(5):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            row[name] = 8.0 * n * nvec / us / 1e3   # GB/s
        out[str(n)] = row
        del a, b, c, d
    return out


SEED_CHANNELS = (16, 32, 64, 64)
MFMA_BF16_PEAK_TFLOPS = 2500.0


def seed_network_timing(prob, W, M, torch, reps=10):
    """The learned guess's U-Net on the workload's element grid: inference and
    one Adam training step (forward, backward and update), timed with events
    on the network's stream, and the convolutions' rate against the dense
    BF16 matrix-core peak. FLOP counts are those of the 3x3x3 convolutions
    (2 x voxels x in x out x 27 per layer; a training step counted as three
    forward passes)."""
    C = SEED_CHANNELS
    net = M.Net(M.params_for(prob), channels=C)
    net.mgar_net_set_params(W.unet_init(C, seed=0))
    x = torch.as_tensor(W.reseeded_density(prob, 0), device="cuda")
    T = torch.as_tensor(W.random_vector(prob.nnodes, 5), device="cuda").abs()
    out = torch.empty_like(T)
    L = len(C)
    V = [prob.nelem >> (3 * l) for l in range(L)]
    mac = 0
    for l in range(L):
        mac += V[l] * 27 * ((3 if l == 0 else C[l - 1]) * C[l] + C[l] * C[l])
    for l in range(L - 2, -1, -1):
        mac += V[l] * 27 * ((C[l + 1] + C[l]) * C[l] + C[l] * C[l])
    fwd_flop = 2.0 * mac

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_inf = timed(lambda: net.mgar_net_infer(x, 1.0, out))
    t_train = timed(lambda: net.mgar_net_train_step(x, T, 1.0, 1e-3, want_loss=False))
    net.close()
    return {"channels": list(C), "grid": [prob.nelx, prob.nely, prob.nelz], "forward_gflop": fwd_flop / 1e9,
            "infer_ms": t_inf, "train_step_ms": t_train,
            "infer_tflops": fwd_flop / t_inf / 1e9, "train_tflops": 3 * fwd_flop / t_train / 1e9,
            "peak_tflops": MFMA_BF16_PEAK_TFLOPS,
            "infer_frac": fwd_flop / t_inf / 1e9 / MFMA_BF16_PEAK_TFLOPS,
            "train_frac": 3 * fwd_flop / t_train / 1e9 / MFMA_BF16_PEAK_TFLOPS}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=71, help="timed optimisation cycles")
    ap.add_argument("--warmup", type=int, default=9, help="untimed cycles before the timed ones")
    ap.add_argument("--config", default="c3", help="workload: c0, c1, c2 or c3 (default 128^3)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--roof-cycles", type=int, default=0,
                    help="0: time the roofline kernel over the timed cycles; N > 0: on N further cycles")
    ap.add_argument("--no-mgcg", action="store_true", help="skip the plain-MGCG reference loop")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched workload (48 2D + 8 3D designs solved together)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned+mixed loop (U-Net trained on the pairs of cycles 2..20, evaluated from 46)")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the MGAR and MGCG loops in the paper's solver settings (eps1 0.5, eps2 1e-6)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision MGAR loop (FP32 multigrid over BF16 densities)")
    ap.add_argument("--paper-tables", action="store_true",
                    help="also run the paper's Table 2 and Table 3 experiments in its settings (300 cycles each)")
    ap.add_argument("--net-only", action="store_true",
                    help="only time the learned guess's U-Net (inference and one training step) and exit")
    ap.add_argument("--oversize", type=int, default=0, metavar="N",
                    help="also run FP64 MGCG solves on an N^3 grid beyond the Infinity Cache (e.g. 256)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent designs would be sharded across GPUs, one process per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2210_00947_amd import mgar as M
    from paper_2210_00947_amd.topopt import TopOpt

    M.lib()
    prob = W.CONFIGS[args.config]
    if args.net_only:
        print(json.dumps({"seed_network": seed_network_timing(prob, W, M, torch)}), flush=True)
        return
    nfix = 1
    for a in range(prob.dim):
        nfix *= prob.fix_hi[a] - prob.fix_lo[a] + 1
    free = prob.nnodes - nfix
    log(f"[bench] {prob.name}: {prob.nnodes} nodes, {free} free DOFs; warmup {args.warmup}, steps {args.steps}")
    mg_ar = run_loop(prob, True, args.warmup, args.steps, W, TopOpt, torch, roof_cycles=args.roof_cycles)
    log(f"[bench] MGAR loop: {mg_ar['s_per_opt_iter']*1e3:.3f} ms/cycle, paths {mg_ar['paths']}")
    mgcg = None
    if not args.no_mgcg:
        mgcg = run_loop(prob, False, args.warmup, args.steps, W, TopOpt, torch)
        log(f"[bench] MGCG loop: {mgcg['s_per_opt_iter']*1e3:.3f} ms/cycle")
    mixed = None
    if not args.no_mixed:
        mixed = run_loop(prob, True, args.warmup, args.steps, W, TopOpt, torch, precision=M.PREC_MIXED)
        log(f"[bench] mixed-precision MGAR loop: {mixed['s_per_opt_iter']*1e3:.3f} ms/cycle")
    # The forms whose behaviour depends on the cycle (the learned guess is
    # trained on cycles 2..20 and first evaluated at 46; acceptances in the
    # paper's settings come once the design settles) run the whole loop
    # whatever --steps says: cycles 1..N_on-1 untimed, N_on..maxit timed.
    full_warm = max(M.n_on(prob.maxit) - 1, 0)
    full_steps = prob.maxit - full_warm
    full_cycles = f"{full_warm + 1}..{prob.maxit}"
    learned = None
    net = None
    if not args.no_learned and prob.dim == 3:
        seed_cfg = {"channels": SEED_CHANNELS, "train_until": 20, "steps": 40, "lr": 1e-3, "lag": 25}
        learned = run_loop(prob, True, full_warm, full_steps, W, TopOpt, torch, precision=M.PREC_MIXED,
                           seed=seed_cfg)
        learned["cycles"] = full_cycles
        learned["seed_config"] = {k: (list(v) if isinstance(v, tuple) else v) for k, v in seed_cfg.items()}
        net = seed_network_timing(prob, W, M, torch)
        log(f"[bench] seed network at {prob.nelx}^3: inference {net['infer_ms']:.2f} ms, training step "
            f"{net['train_step_ms']:.2f} ms ({net['train_tflops']:.0f} TFLOP/s)")
        log(f"[bench] learned+mixed MGAR loop, cycles {full_cycles}: {learned['s_per_opt_iter']*1e3:.3f} "
            f"ms/cycle, guess evaluated in {learned['seed_evaluated_cycles']} and used in "
            f"{learned['seed_used_cycles']} cycles")
    paper = None
    if not args.no_paper:
        # the paper's solver settings (Sec. 3.1, 4): reconstruction criterion
        # eps1 = 0.5, MGCG accuracy eps2 = 1e-6, on the same workload and cycles
        import dataclasses
        pp = dataclasses.replace(prob, tol=1e-6)
        p_ar = run_loop(pp, True, full_warm, full_steps, W, TopOpt, torch, eps_accept=0.5)
        p_cg = run_loop(pp, False, full_warm, full_steps, W, TopOpt, torch)
        paper = {"eps1": 0.5, "eps2": 1e-6, "cycles": full_cycles,
                 "mgar": {k: p_ar[k] for k in ("s_per_opt_iter", "cg_iters_mean", "paths", "final_compliance")},
                 "mgcg": {k: p_cg[k] for k in ("s_per_opt_iter", "cg_iters_mean", "paths", "final_compliance")},
                 "efficiency_improvement": 1.0 - p_ar["s_per_opt_iter"] / p_cg["s_per_opt_iter"],
                 "objective_rel_diff": abs(p_ar["final_compliance"] - p_cg["final_compliance"])
                 / abs(p_cg["final_compliance"])}
        log(f"[bench] paper setting (eps1 0.5, eps2 1e-6), cycles {full_cycles}: MGAR {p_ar['s_per_opt_iter']*1e3:.3f} ms/cycle "
            f"(paths {p_ar['paths']}), MGCG {p_cg['s_per_opt_iter']*1e3:.3f} ms/cycle, "
            f"efficiency improvement {100 * paper['efficiency_improvement']:.1f} %")
    batch = None
    if not args.no_batch:
        batch = run_batched(W, M, torch)
        log(f"[bench] batched workload: {batch['batched_mgcg_s_per_solve']*1e3:.2f} ms per batched solve "
            f"vs {batch['one_by_one_mgcg_s_per_solve']*1e3:.2f} ms one design at a time")
        batch["mixed"] = run_batched(W, M, torch, precision=M.PREC_MIXED)
        log(f"[bench] batched workload, mixed precision: "
            f"{batch['mixed']['batched_mgcg_s_per_solve']*1e3:.2f} ms per batched solve vs "
            f"{batch['mixed']['one_by_one_mgcg_s_per_solve']*1e3:.2f} ms one design at a time")
    value = free * args.steps / mg_ar["elapsed_s"]
    roof = None
    if mg_ar["kernel_launches"] > 0:
        avg_s = mg_ar["kernel_ms_total"] / mg_ar["kernel_launches"] * 1e-3
        per_launch = mg_ar["kernel_bytes_total"] / mg_ar["kernel_launches"]
        achieved = per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": committed_traffic(mg_ar["roof_shape"]) if prob.name == "3d-128^3" else None,
                "kernel": roof_kernel(mg_ar["roof_shape"]),
                "bytes_per_launch": per_launch, "avg_launch_us": avg_s * 1e6,
                "launches": mg_ar["kernel_launches"],
                "stream_ref": stream_reference(torch, [prob.nnodes, 64 << 20])}
        log(f"[bench] plain streaming reference (GB/s): {roof['stream_ref']}")
        if prob.dim == 3:
            roof["effective"] = effective_bandwidth(prob, W, TopOpt, torch)
            log(f"[bench] effective rates: {roof['effective']}")
    tables = None
    if args.paper_tables:
        tables = paper_tables(W, TopOpt, torch)
    over = None
    if args.oversize > 0:
        over = oversize_control(W, M, torch, args.oversize)
        log(f"[bench] oversize control: {over}")
    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle (one MGCG solve) ...")
        cpu = cpu_baseline(prob, W)
        log(f"[bench] oracle: {cpu['seconds']:.1f} s")
    out = {
        "metric": "s/opt-iter & DOF-solves/s at 128^3 hex, MGAR vs MGCG @rel.res 1e-8; HBM GB/s",
        "value": value,
        "unit": "DOF-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mg_ar["s_per_opt_iter"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"{prob.name}: SIMP heat-conduction topology optimisation, "
                                f"{prob.nelx}x{prob.nely}x{prob.nelz} trilinear hex, {prob.levels} MG levels, "
                                f"MGAR m=2 eps1=tol={prob.tol:g}, OC move {prob.move}, "
                                f"cycles {args.warmup + 1}..{args.warmup + args.steps}"),
                   "nodes": prob.nnodes, "free_dofs": free, "levels": prob.levels},
        "s_per_opt_iter": {"mgar": mg_ar["s_per_opt_iter"],
                           "mgcg": mgcg["s_per_opt_iter"] if mgcg else None,
                           "mgar_mixed": mixed["s_per_opt_iter"] if mixed else None,
                           "learned_mixed": learned["s_per_opt_iter"] if learned else None},
        "dof_solves_per_s": {"mgar": value,
                             "mgcg": free * args.steps / mgcg["elapsed_s"] if mgcg else None,
                             "mgar_mixed": free * args.steps / mixed["elapsed_s"] if mixed else None},
        "mgar": mg_ar,
        "mgcg": mgcg,
        "mgar_mixed": mixed,
        "learned_mixed": learned,
        "seed_network": net,
        "batched": batch,
        "paper_setting": paper,
        "roofline": roof,
        "oversize_control": over,
        "paper_tables": tables,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
