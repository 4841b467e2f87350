"""Writes c3_loop12.json: the first 12 cycles of the 128^3 optimisation loop
run by the CPU oracle only (oracle.topopt.run_loop; N_on = 10 of 80 cycles, so
cycles 10-12 are reanalysis calls). Stored: per-cycle path, CG iterations,
Eq 28 residual and compliance; the final design and temperature at 2048
seeded sample positions each, and their sums and squared norms over the whole
grid. The oracle takes ~20 s per cycle at this size, too long to run beside the
GPU tests.

Usage: python tests/golden/make_c3_loop.py   (from the repository root)
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import topopt  # noqa: E402

CYCLES = 12
NSAMPLE = 2048


def sample_indices(n, seed):
    return np.sort(np.random.default_rng(seed).choice(n, NSAMPLE, replace=False))


def main():
    prob = W.C3
    x, xphys, t, recs = topopt.run_loop(prob, maxit=CYCLES)
    ie = sample_indices(prob.nelem, 12001)
    inn = sample_indices(prob.nnodes, 12002)
    out = {
        "workload": prob.name, "cycles": CYCLES, "n_on": topopt.n_on(prob.maxit),
        "records": [{"cycle": r.cycle, "path": r.path, "cg_iters": r.cg_iters, "compliance": r.compliance,
                     "res_ca": None if r.res_ca != r.res_ca else float(r.res_ca)} for r in recs],
        "x_index": ie.tolist(), "x_sample": x[ie].tolist(),
        "x_sum": float(x.sum()), "x_sq": float((x * x).sum()),
        "t_index": inn.tolist(), "t_sample": t[inn].tolist(),
        "t_sum": float(t.sum()), "t_sq": float((t * t).sum()),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_loop12.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
