"""Captured PCG iterations (HIP graphs) against eager launches: every solve,
over repeated replays with eager work and synchronisation in between, must
equal the eagerly launched solve bit for bit."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import dev, host, require_gpu

pytestmark = pytest.mark.gpu

PROBS = [W.tiny_2d(40, 40, 3), W.tiny_3d(32, 32, 32, 4), W.tiny_3d(48, 32, 16, 3)]
IDS = [p.name for p in PROBS]


def pair(prob, precision, graphs):
    import torch
    from paper_2210_00947_amd import mgar as M
    require_gpu()
    h = M.Handle(M.params_for(prob, precision=precision))
    h.mgar_set_graphs(graphs)
    q = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgar_load_vector(dev(W.element_source(prob)), q)
    return h, q


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("prob", PROBS, ids=IDS)
def test_graph_replays_equal_eager(prob, precision):
    import torch
    hg, q = pair(prob, precision, True)
    he, _ = pair(prob, precision, False)
    T0g = torch.zeros(prob.nnodes, dtype=torch.float64, device="cuda")
    T0e = torch.zeros_like(T0g)
    for rep in range(4):
        x = dev(W.random_density(prob.nelem, 900 + rep, 0.05, 1.0))
        Tg = torch.empty_like(T0g)
        Te = torch.empty_like(T0g)
        if rep == 0:
            sg = hg.mgcg_solve(x, q, None, 1e-8, Tg)
            se = he.mgcg_solve(x, q, None, 1e-8, Te)
        else:
            sg = hg.mgar_solve(x, q, T0g, 1e-8, Tg)
            se = he.mgar_solve(x, q, T0e, 1e-8, Te)
        torch.cuda.synchronize()
        assert sg["cg_iters"] == se["cg_iters"] and sg["path"] == se["path"]
        assert sg["refinements"] == se["refinements"]
        assert torch.equal(Tg, Te), rep
        # eager work on the handle's stream between replays
        y = torch.empty_like(Tg)
        hg.mgar_op_apply(0, dev(W.random_density(prob.nelem, 5, 1e-3, 1.0)), Tg, y)
        T0g, T0e = Tg, Te
