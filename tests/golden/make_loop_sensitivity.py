"""Writes loop_sensitivity.json: how much the oracle's own optimisation loop
moves when its initial design is perturbed at the level of round-off. For
each workload the oracle loop runs twice, from x_init and from x_init * (1 +
1e-13 g) with g a seeded standard-normal vector; stored are the max-abs
differences of the filtered designs after every cycle and of the final
designs, and the relative differences of every cycle's compliance and Eq 28
residual. Two correct FP64 implementations that sum in different orders differ
by round-off in every solve, so this is the scale against which the GPU loop's
design differences are judged. Calls the oracle only.

Usage: python tests/golden/make_loop_sensitivity.py   (from the repository root; ~10 min)
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import topopt  # noqa: E402

EPS = 1e-13


def _rel(a, b):
    if a != a or b != b:     # NaN: no reduced solve in that cycle
        return 0.0
    return abs(a - b) / abs(b) if b != 0 else abs(a - b)


def sensitivity(prob, maxit=None, **loop):
    runs = []
    for pert in (False, True):
        x0 = np.full(prob.nelem, prob.x_init)
        if pert:
            x0 = x0 * (1.0 + EPS * W.random_vector(prob.nelem, 5))
        xph = []
        x, _, _, recs = topopt.run_loop(prob, maxit=maxit, x_init=x0,
                                        on_cycle=lambda k, xp, t: xph.append(np.array(xp)), **loop)
        runs.append((x, xph, recs))
    (xa, pa, ra), (xb, pb, rb) = runs
    return {
        "cycles": len(ra),
        "xphys_maxabs": [float(np.abs(a - b).max()) for a, b in zip(pa, pb)],
        "x_final_maxabs": float(np.abs(xa - xb).max()),
        "compliance_rel": [_rel(a.compliance, b.compliance) for a, b in zip(ra, rb)],
        "res_ca_rel": [_rel(a.res_ca, b.res_ca) for a, b in zip(ra, rb)],
        "same_paths": all(a.path == b.path for a, b in zip(ra, rb)),
        "same_cg_iters": all(a.cg_iters == b.cg_iters for a, b in zip(ra, rb)),
    }


def main():
    from oracle.solvers import MgarParams
    out = {"perturbation": EPS}
    for key in ("c0", "c1", "c2"):
        out[key] = sensitivity(W.CONFIGS[key])
        print(key, out[key]["x_final_maxabs"], flush=True)
    # the paper-setting loops of the GPU tests (eps1 = 0.5, eps2 = 1e-6)
    paper = MgarParams(eps_accept=0.5, cg_max=200)
    p96 = W.paper_2d(96, 3)
    out["paper96"] = sensitivity(p96, params=paper, continuous={"r_min": 3.0})
    print("paper96", out["paper96"]["x_final_maxabs"], flush=True)
    p160 = W.paper_2d(160, 4, volfrac=0.4)
    out["paper160"] = sensitivity(p160, maxit=120, params=paper, qelem=W.quadrant_source(p160),
                                  continuous={"r_min": 3.0})
    print("paper160", out["paper160"]["x_final_maxabs"], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "loop_sensitivity.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
