"""The allocation-free residual entry point (mgar_residual_noalloc, static
device scratch) against mgar_residual on the same inputs, on two calls in a
row (the second on a smaller grid, so the scratch holds the first call's
partials when the second starts), plus its size and argument checks."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import dev, require_gpu

pytestmark = pytest.mark.gpu


def _case(prob, seed):
    import torch
    from paper_2210_00947_amd import mgar as M
    p = M.params_for(prob)
    h = M.Handle(p)
    q = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgar_load_vector(dev(W.element_source(prob)), q)
    x = dev(W.random_density(prob.nelem, seed, 0.0, 1.0))
    T = dev(W.random_vector(prob.nnodes, seed + 1))       # nonzero on Dirichlet nodes: read as 0
    want = h.mgar_residual(x, q, T)
    h.close()
    return p, x, q, T, want


@pytest.mark.parametrize("first,second", [
    (W.tiny_3d(48, 32, 16, 3), W.tiny_3d(16, 16, 16, 3)),
    (W.C3, W.C0),
    (W.C1, W.tiny_2d(48, 32, 4)),
])
def test_noalloc_residual_equals_handle_residual(first, second):
    require_gpu()
    import torch
    from paper_2210_00947_amd import mgar as M
    out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
    cases = [_case(first, 3), _case(second, 5)]
    for i, (p, x, q, T, _) in enumerate(cases):
        M.mgar_residual_noalloc(p, x, q, T, out[i:i + 1])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for g, (_, _, _, _, want) in zip(got, cases):
        assert want > 0.0
        assert abs(g - want) <= 1e-12 * want, (g, want)
    # the same call again after the smaller one: the scratch holds no state
    p, x, q, T, want = cases[0]
    M.mgar_residual_noalloc(p, x, q, T, out[:1])
    torch.cuda.synchronize()
    assert abs(float(out[0]) - want) <= 1e-12 * want


def test_noalloc_residual_zero_source_and_arguments():
    require_gpu()
    import torch
    from paper_2210_00947_amd import mgar as M
    prob = W.tiny_2d(16, 16, 2)
    p = M.params_for(prob)
    x = dev(W.random_density(prob.nelem, 1))
    z = torch.zeros(prob.nnodes, dtype=torch.float64, device="cuda")
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    M.mgar_residual_noalloc(p, x, z, z, out)
    torch.cuda.synchronize()
    assert float(out[0]) == 0.0
    big = M.params_for(prob)
    big.dim, big.nelx, big.nely, big.nelz = 3, 2048, 2048, 1024   # 4.3e9 nodes: beyond the maximum
    rc = M.lib().mgar_residual_noalloc(big, M._ptr(x), M._ptr(z), M._ptr(z), M._ptr(out), None)
    assert rc == M.MGAR_E_ARG
    rc = M.lib().mgar_residual_noalloc(p, None, M._ptr(z), M._ptr(z), M._ptr(out), None)
    assert rc == M.MGAR_E_ARG
