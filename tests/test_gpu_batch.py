"""Batched solves (many designs of uneven grids together) against the oracle
and against each design's own single-design solve."""
import numpy as np
import pytest

import workloads as W
from oracle import fe, solvers
from tests.gpu_util import dev, host, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

PROBS = [W.tiny_2d(40, 40, 3), W.tiny_3d(16, 16, 16, 3), W.tiny_2d(48, 32, 4), W.tiny_3d(16, 16, 24, 4),
         W.tiny_3d(32, 32, 32, 4), W.tiny_2d(64, 64, 5)]


def make_batch(probs, **kw):
    require_gpu()
    from paper_2210_00947_amd import mgar as M
    return M.Batch([M.params_for(p, **kw) for p in probs])


def concat(b, arrays, which="node"):
    import torch
    off = b.node_off if which == "node" else b.elem_off
    out = np.zeros(off[-1])
    for i, a in enumerate(arrays):
        out[off[i]:off[i + 1]] = a
    return torch.as_tensor(out, dtype=torch.float64, device="cuda")


def split(b, t):
    h = host(t)
    return [h[b.node_off[i]:b.node_off[i + 1]] for i in range(b.n)]


def loads(b, probs):
    import torch
    q = torch.empty(b.N, dtype=torch.float64, device="cuda")
    b.mgar_batch_load_vector(concat(b, [W.element_source(p) for p in probs], "elem"), q)
    return q


def test_layout_and_load_vector():
    b = make_batch(PROBS)
    assert b.node_off[0] == 0 and b.elem_off[0] == 0
    for i, p in enumerate(PROBS):
        assert b.node_off[i + 1] - b.node_off[i] == p.nnodes
        assert b.elem_off[i + 1] - b.elem_off[i] == p.nelem
    q = loads(b, PROBS)
    for p, qi in zip(PROBS, split(b, q)):
        assert np.abs(qi - fe.FEProblem(p).q).max() <= 1e-15 * np.abs(qi).max()


@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "eager"])
def test_batched_mgcg_matches_oracle(use_graph):
    import torch
    b = make_batch(PROBS)
    b.mgar_batch_set_graph(use_graph)
    q = loads(b, PROBS)
    xs = [W.random_density(p.nelem, 100 + i, 0.0, 1.0) for i, p in enumerate(PROBS)]
    T = torch.empty(b.N, dtype=torch.float64, device="cuda")
    st = b.mgcg_batch_solve(concat(b, xs, "elem"), q, None, 1e-8, T)
    for p, x, t, s in zip(PROBS, xs, split(b, T), st):
        t_or, s_or = solvers.MgarSolver(p, solvers.MgarParams(cg_max=200)).mgcg(x, np.zeros(p.nnodes), 1e-8)
        assert s["rc"] == 0 and s["path"] == 0
        assert s["cg_iters"] == s_or.cg_iters, p.name
        assert rel_l2(t, t_or) < 1e-8, p.name


def test_batched_equals_single_design_solves():
    import torch
    from paper_2210_00947_amd import mgar as M
    b = make_batch(PROBS)
    q = loads(b, PROBS)
    xs = [W.random_density(p.nelem, 200 + i, 0.0, 1.0) for i, p in enumerate(PROBS)]
    T0s = [W.random_vector(p.nnodes, 300 + i) for i, p in enumerate(PROBS)]
    T = torch.empty(b.N, dtype=torch.float64, device="cuda")
    st = b.mgcg_batch_solve(concat(b, xs, "elem"), q, concat(b, T0s), 1e-8, T)
    for p, x, t0, t, s in zip(PROBS, xs, T0s, split(b, T), st):
        h = M.Handle(M.params_for(p))
        qi = torch.empty(p.nnodes, dtype=torch.float64, device="cuda")
        h.mgar_load_vector(dev(W.element_source(p)), qi)
        Ti = torch.empty_like(qi)
        si = h.mgcg_solve(dev(x), qi, dev(t0), 1e-8, Ti)
        assert s["cg_iters"] == si["cg_iters"], p.name
        assert rel_l2(t, host(Ti)) < 1e-12, p.name


def test_graph_replays_match_eager_over_repeated_solves():
    """The captured iteration graph is replayed many times per solve and
    across solves; every solve must equal the eagerly launched one."""
    import torch
    bg = make_batch(PROBS)
    be = make_batch(PROBS)
    be.mgar_batch_set_graph(False)
    q = loads(bg, PROBS)
    for rep in range(3):
        xs = concat(bg, [W.random_density(p.nelem, 400 + 10 * rep + i, 0.0, 1.0)
                         for i, p in enumerate(PROBS)], "elem")
        Tg = torch.empty(bg.N, dtype=torch.float64, device="cuda")
        Te = torch.empty_like(Tg)
        sg = bg.mgcg_batch_solve(xs, q, None, 1e-8, Tg)
        torch.cuda.synchronize()
        se = be.mgcg_batch_solve(xs, q, None, 1e-8, Te)
        assert [s["cg_iters"] for s in sg] == [s["cg_iters"] for s in se]
        assert torch.equal(Tg, Te)


@pytest.mark.parametrize("eps", [1e-8, 0.5])
def test_batched_mgar_matches_oracle(eps):
    """Reanalysis per design; with eps = 0.5 the batch mixes accepted designs
    (uniform 1% density change) with rejected ones (random change)."""
    import torch
    b = make_batch(PROBS, eps_accept=eps)
    q = loads(b, PROBS)
    x0 = [W.random_density(p.nelem, 21, 0.2, 0.8) for p in PROBS]
    x1 = []
    for i, (p, x) in enumerate(zip(PROBS, x0)):
        if i % 2 == 0:
            x1.append(np.clip(1.01 * x, 0, 1))
        else:
            x1.append(np.clip(x + 0.02 * W.random_vector(p.nelem, 22), 0, 1))
    T0 = torch.empty(b.N, dtype=torch.float64, device="cuda")
    T1 = torch.empty_like(T0)
    b.mgcg_batch_solve(concat(b, x0, "elem"), q, None, 1e-8, T0)
    st = b.mgar_batch_solve(concat(b, x1, "elem"), q, T0, 1e-8, T1)
    paths = []
    for i, (p, a, c, t, s) in enumerate(zip(PROBS, x0, x1, split(b, T1), st)):
        sol = solvers.MgarSolver(p, solvers.MgarParams(eps_accept=eps))
        t0, _ = sol.mgcg(a, np.zeros(p.nnodes), 1e-8)
        t1, s_or = sol.mgar(c, t0, 1e-8)
        assert s["path"] == s_or.path, p.name
        assert abs(s["res_ca"] - s_or.res_ca) <= 1e-7 * s_or.res_ca, p.name
        if s["path"] == 2:
            assert s["cg_iters"] == s_or.cg_iters, p.name
        assert rel_l2(t, t1) < 1e-8, p.name
        paths.append(s["path"])
    if eps == 0.5:
        assert 1 in paths and 2 in paths
    # a second reanalysis after a mixed accept/fallback step stays consistent
    T2 = torch.empty_like(T0)
    st2 = b.mgar_batch_solve(concat(b, x1, "elem"), q, T1, 1e-8, T2)
    assert all(s["rc"] >= 0 for s in st2)


def test_full_batched_workload_residuals():
    """48 2D + 8 3D designs of uneven sizes in one batch; true residual of
    every fourth design from the oracle's assembled matrix."""
    import torch
    probs = W.batched_designs()
    b = make_batch(probs)
    q = loads(b, probs)
    xs = [W.reseeded_density(p, i) for i, p in enumerate(probs)]
    T = torch.empty(b.N, dtype=torch.float64, device="cuda")
    st = b.mgcg_batch_solve(concat(b, xs, "elem"), q, None, 1e-8, T)
    assert all(s["rc"] == 0 and s["res_final"] <= 1e-8 for s in st)
    ts = split(b, T)
    for i in range(0, len(probs), 4):
        p = probs[i]
        fep = fe.FEProblem(p)
        r = fep.to_free(fep.q) - fep.K_free(xs[i]) @ ts[i][fep.free]
        assert np.linalg.norm(r) / np.linalg.norm(fep.to_free(fep.q)) < 1.001e-8, p.name
        assert np.all(ts[i][fep.fixed] == 0)


def test_batch_rejects_bad_parameters():
    from paper_2210_00947_amd import mgar as M
    require_gpu()
    good = M.params_for(W.tiny_2d(40, 40, 3))
    other = M.params_for(W.tiny_2d(48, 32, 4), n_basis=3)
    with pytest.raises(M.MgarError):
        M.Batch([good, other])                     # n_basis must agree
    mixed = M.params_for(W.tiny_2d(40, 40, 3), precision=M.PREC_MIXED)
    with pytest.raises(M.MgarError):
        M.Batch([good, mixed])                     # one precision per batch
    p2 = M.params_for(W.tiny_2d(40, 40, 3), precision=M.PREC_MIXED)
    p2.penal = 2.0                                 # BF16 loads apply the p = 3 law
    with pytest.raises(M.MgarError):
        M.Batch([p2])
    with pytest.raises(M.MgarError):
        M.Batch([mixed, M.params_for(W.tiny_2d(48, 32, 4), precision=M.PREC_MIXED, inner_tol=1e-4)])
    k2 = M.params_for(W.tiny_2d(48, 32, 4))
    k2.kmin = 1e-4
    with pytest.raises(M.MgarError):
        M.Batch([good, k2])                        # one SIMP law per batch
    M.Batch([mixed, M.params_for(W.tiny_3d(16, 16, 16, 3), precision=M.PREC_MIXED)])
    one = M.params_for(W.tiny_2d(8, 8, 1))
    with pytest.raises(M.MgarError):
        M.Batch([one])                             # a batch design needs >= 2 grids


# ---------------------------------------------------------------- mixed precision
# FP32 multigrid over BF16 densities with FP32 inner PCG runs and FP64
# residual replacement, per design; compared with the FP64 oracle at the
# tolerances of the single-design mixed path (true FP64 residual <= tol,
# solution 1e-6 rel. L2 after a full solve, 1e-4 for an accepted reduced
# solution) and with each design's own single-design mixed solve.

def _fp64_residual(p, x, t):
    fep = fe.FEProblem(p)
    r = fep.to_free(fep.q) - fep.K_free(x) @ t[fep.free]
    return np.linalg.norm(r) / np.linalg.norm(fep.to_free(fep.q)), fep


@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "eager"])
def test_batched_mixed_mgcg_matches_oracle(use_graph):
    import torch
    from paper_2210_00947_amd import mgar as M
    b = make_batch(PROBS, precision=M.PREC_MIXED)
    b.mgar_batch_set_graph(use_graph)
    q = loads(b, PROBS)
    xs = [W.random_density(p.nelem, 100 + i, 0.0, 1.0) for i, p in enumerate(PROBS)]
    T = torch.empty(b.N, dtype=torch.float64, device="cuda")
    st = b.mgcg_batch_solve(concat(b, xs, "elem"), q, None, 1e-8, T)
    for p, x, t, s in zip(PROBS, xs, split(b, T), st):
        t_or, s_or = solvers.MgarSolver(p, solvers.MgarParams(cg_max=200)).mgcg(x, np.zeros(p.nnodes), 1e-8)
        res, fep = _fp64_residual(p, x, t)
        err = rel_l2(t, t_or)
        print(f"batched mixed MGCG {p.name}: true rel. residual {res:.2e} (reported {s['res_final']:.2e}), "
              f"T rel L2 err {err:.2e}, {s['cg_iters']} FP32 its ({s_or.cg_iters} FP64), "
              f"{s['refinements']} refinements")
        assert s["rc"] == 0 and s["path"] == 0 and s["refinements"] >= 1, p.name
        assert res <= 1.001e-8, p.name
        assert abs(res - s["res_final"]) <= 1e-3 * res + 1e-15, p.name
        assert err < 1e-6, p.name
        assert np.all(t[fep.fixed] == 0)
        # restarted inner runs: at most twice the FP64 count plus one run's worth
        assert s["cg_iters"] <= 2 * s_or.cg_iters + 10, (p.name, s["cg_iters"], s_or.cg_iters)


def test_batched_mixed_graph_equals_eager():
    import torch
    from paper_2210_00947_amd import mgar as M
    bg = make_batch(PROBS, precision=M.PREC_MIXED)
    be = make_batch(PROBS, precision=M.PREC_MIXED)
    be.mgar_batch_set_graph(False)
    q = loads(bg, PROBS)
    for rep in range(2):
        xs = concat(bg, [W.random_density(p.nelem, 500 + 10 * rep + i, 0.0, 1.0)
                         for i, p in enumerate(PROBS)], "elem")
        Tg = torch.empty(bg.N, dtype=torch.float64, device="cuda")
        Te = torch.empty_like(Tg)
        sg = bg.mgcg_batch_solve(xs, q, None, 1e-8, Tg)
        torch.cuda.synchronize()
        se = be.mgcg_batch_solve(xs, q, None, 1e-8, Te)
        assert [s["cg_iters"] for s in sg] == [s["cg_iters"] for s in se]
        assert torch.equal(Tg, Te)


def test_batched_mixed_equals_single_design_mixed_solves():
    """Each design of a mixed batch against its own single-design mixed solve:
    the two stop at the same FP64 residual bound by different refinement
    schedules, so they agree to the accuracy that bound gives (1e-6)."""
    import torch
    from paper_2210_00947_amd import mgar as M
    b = make_batch(PROBS, precision=M.PREC_MIXED)
    q = loads(b, PROBS)
    xs = [W.random_density(p.nelem, 200 + i, 0.0, 1.0) for i, p in enumerate(PROBS)]
    T0s = [W.random_vector(p.nnodes, 300 + i) for i, p in enumerate(PROBS)]
    T = torch.empty(b.N, dtype=torch.float64, device="cuda")
    st = b.mgcg_batch_solve(concat(b, xs, "elem"), q, concat(b, T0s), 1e-8, T)
    for p, x, t0, t, s in zip(PROBS, xs, T0s, split(b, T), st):
        h = M.Handle(M.params_for(p, precision=M.PREC_MIXED))
        qi = torch.empty(p.nnodes, dtype=torch.float64, device="cuda")
        h.mgar_load_vector(dev(W.element_source(p)), qi)
        Ti = torch.empty_like(qi)
        si = h.mgcg_solve(dev(x), qi, dev(t0), 1e-8, Ti)
        assert s["rc"] == 0 and si["rc"] == 0, p.name
        assert rel_l2(t, host(Ti)) < 1e-6, p.name


@pytest.mark.parametrize("eps", [1e-8, 0.5])
def test_batched_mixed_mgar_matches_oracle(eps):
    import torch
    from paper_2210_00947_amd import mgar as M
    b = make_batch(PROBS, eps_accept=eps, precision=M.PREC_MIXED)
    q = loads(b, PROBS)
    x0 = [W.random_density(p.nelem, 21, 0.2, 0.8) for p in PROBS]
    x1 = []
    for i, (p, x) in enumerate(zip(PROBS, x0)):
        if i % 2 == 0:
            x1.append(np.clip(1.01 * x, 0, 1))
        else:
            x1.append(np.clip(x + 0.02 * W.random_vector(p.nelem, 22), 0, 1))
    T0 = torch.empty(b.N, dtype=torch.float64, device="cuda")
    T1 = torch.empty_like(T0)
    b.mgcg_batch_solve(concat(b, x0, "elem"), q, None, 1e-8, T0)
    st = b.mgar_batch_solve(concat(b, x1, "elem"), q, T0, 1e-8, T1)
    paths = []
    for i, (p, a, c, t, s) in enumerate(zip(PROBS, x0, x1, split(b, T1), st)):
        sol = solvers.MgarSolver(p, solvers.MgarParams(eps_accept=eps))
        t0, _ = sol.mgcg(a, np.zeros(p.nnodes), 1e-8)
        t1, s_or = sol.mgar(c, t0, 1e-8)
        print(f"batched mixed MGAR {p.name} eps {eps}: path {s['path']} (oracle {s_or.path}), "
              f"Res {s['res_ca']:.4e} (oracle {s_or.res_ca:.4e}), T rel err {rel_l2(t, t1):.2e}")
        # Res in FP64 on a basis built by FP32 V-cycles over BF16 densities
        assert abs(s["res_ca"] - s_or.res_ca) <= 1e-2 * s_or.res_ca, p.name
        assert s["path"] == s_or.path, p.name
        if s["path"] == 2:
            assert s["rc"] == 0 and s["res_final"] <= 1e-8, p.name
        assert rel_l2(t, t1) < (1e-6 if s["path"] == 2 else 1e-4), p.name
        paths.append(s["path"])
    if eps == 0.5:
        assert 1 in paths and 2 in paths
    T2 = torch.empty_like(T0)
    st2 = b.mgar_batch_solve(concat(b, x1, "elem"), q, T1, 1e-8, T2)
    assert all(s["rc"] >= 0 for s in st2)


def test_full_batched_workload_mixed_residuals():
    """48 2D + 8 3D designs in one mixed batch: every design converges in
    FP64 residual; true residual of every fourth design from the oracle's
    assembled matrix."""
    import torch
    from paper_2210_00947_amd import mgar as M
    probs = W.batched_designs()
    b = make_batch(probs, precision=M.PREC_MIXED)
    q = loads(b, probs)
    xs = [W.reseeded_density(p, i) for i, p in enumerate(probs)]
    T = torch.empty(b.N, dtype=torch.float64, device="cuda")
    st = b.mgcg_batch_solve(concat(b, xs, "elem"), q, None, 1e-8, T)
    assert all(s["rc"] == 0 and s["res_final"] <= 1e-8 for s in st)
    ts = split(b, T)
    for i in range(0, len(probs), 4):
        res, fep = _fp64_residual(probs[i], xs[i], ts[i])
        assert res < 1.001e-8, probs[i].name
        assert np.all(ts[i][fep.fixed] == 0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_block_size_matches_the_oracle(precision):
    """The batched launches at each block size the tuner may choose (256,
    128, 64 threads): every design's temperature against the oracle, CG
    iterations (FP64) against the oracle's, and the block sizes against each
    other (they differ only in the order block partials of a dot are summed)."""
    import torch
    from paper_2210_00947_amd import mgar as M
    kw = {} if precision == "fp64" else {"precision": M.PREC_MIXED}
    b = make_batch(PROBS, **kw)
    q = loads(b, PROBS)
    xs = [W.random_density(p.nelem, 400 + i, 0.0, 1.0) for i, p in enumerate(PROBS)]
    ors = [solvers.MgarSolver(p, solvers.MgarParams(cg_max=200)).mgcg(x, np.zeros(p.nnodes), 1e-8)
           for p, x in zip(PROBS, xs)]
    sols = {}
    for bs in (256, 128, 64):
        b.mgar_batch_set_block(bs)
        assert b.mgar_batch_get_block() == bs
        T = torch.empty(b.N, dtype=torch.float64, device="cuda")
        st = b.mgcg_batch_solve(concat(b, xs, "elem"), q, None, 1e-8, T)
        sols[bs] = split(b, T)
        for p, t, s, (t_or, s_or) in zip(PROBS, sols[bs], st, ors):
            assert s["rc"] == 0, (bs, p.name)
            assert rel_l2(t, t_or) < (1e-8 if precision == "fp64" else 1e-6), (bs, p.name)
            if precision == "fp64":
                assert s["cg_iters"] == s_or.cg_iters, (bs, p.name)
    for bs in (128, 64):
        for t, t256 in zip(sols[bs], sols[256]):
            assert rel_l2(t, t256) < (1e-10 if precision == "fp64" else 1e-6)


def test_autotune_keeps_a_candidate_and_the_solution():
    """The tuner times the three block sizes on batched MGCG solves, keeps the
    fastest, and the batch then solves as before."""
    import torch
    b = make_batch(PROBS)
    q = loads(b, PROBS)
    xs = [W.random_density(p.nelem, 500 + i, 0.0, 1.0) for i, p in enumerate(PROBS)]
    x = concat(b, xs, "elem")
    bs, us = b.mgar_batch_autotune(x, q, 1e-8, reps=2)
    assert bs in (64, 128, 256) and b.mgar_batch_get_block() == bs
    assert all(v > 0 for v in us.values()) and us[bs] == min(us.values())
    T = torch.empty(b.N, dtype=torch.float64, device="cuda")
    st = b.mgcg_batch_solve(x, q, None, 1e-8, T)
    for p, xi, t, s in zip(PROBS, xs, split(b, T), st):
        t_or, s_or = solvers.MgarSolver(p, solvers.MgarParams(cg_max=200)).mgcg(xi, np.zeros(p.nnodes), 1e-8)
        assert s["cg_iters"] == s_or.cg_iters and rel_l2(t, t_or) < 1e-8, p.name
    print(f"batch tuner: block {bs}, mean solve times (us) {us}")
