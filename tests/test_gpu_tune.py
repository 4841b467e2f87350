"""Launch shapes on the GPU: every valid shape gives bit-identical stencil
outputs, invalid ones are refused, and solves after the tuner still match the
oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import fe, solvers
from tests.gpu_util import dev, host, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

SHAPES = [[0, 0, 0, 0], [1, 4, 1, 1], [1, 6, 2, 2], [1, 12, 1, 1], [1, 24, 2, 2], [1, 5, 1, 3], [1, 5, 3, 2], [1, 8, 4, 1],
          [1, 7, 2, 1], [1, 64, 1, 1],
          # two rows per thread: one tile across x (ragged last row pair), two and
          # three tiles, one z-chunk, queue depths 1 and 2
          [2, 4, 1, 1], [2, 6, 2, 1], [2, 5, 1, 2], [2, 7, 2, 3], [2, 64, 1, 1], [2, 3, 2, 4]]


def handle(prob, **kw):
    require_gpu()
    from paper_2210_00947_amd import mgar as M
    return M.Handle(M.params_for(prob, **kw))


@pytest.mark.parametrize("prob", [W.tiny_3d(32, 32, 32, 4), W.tiny_3d(48, 32, 16, 3)],
                         ids=["32x32x32", "48x32x16"])
def test_apply_and_jacobi_bit_identical_across_shapes(prob):
    import torch
    h = handle(prob)
    g = fe.Grid(3, prob.nelx, prob.nely, prob.nelz)
    fixed = fe.fixed_mask_from_box(g, prob.fix_lo, prob.fix_hi)
    k = W.random_density(g.nelem, 81, 1e-3, 1.0)
    x = W.random_vector(g.nnodes, 82)
    b = W.random_vector(g.nnodes, 83)
    x[fixed] = 0.0
    b[fixed] = 0.0
    ref_y = ref_j = None
    for s in SHAPES:
        h.mgar_tune_set(0, 0, 0, s)
        h.mgar_tune_set(0, 0, 3, s)
        assert h.mgar_tune_get(0, 0, 0) == s
        y = torch.empty(g.nnodes, dtype=torch.float64, device="cuda")
        j = torch.empty_like(y)
        h.mgar_op_apply(0, dev(k), dev(x), y)
        h.mgar_op_jacobi(0, dev(k), dev(b), dev(x), j)
        y, j = host(y), host(j)
        if ref_y is None:
            ref_y, ref_j = y, j
            K = fe.assemble(g, k)
            want = K @ x
            want[fixed] = 0.0
            assert np.abs(y - want).max() <= 1e-13 * np.abs(want).max()
        assert np.array_equal(y, ref_y), s
        assert np.array_equal(j, ref_j), s


def test_invalid_shapes_refused():
    from paper_2210_00947_amd import mgar as M
    prob = W.tiny_3d(32, 32, 32, 4)
    h = handle(prob)
    before = h.mgar_tune_get(0, 0, 1)
    for bad in ([1, 0, 1, 1], [1, 4, 5, 1], [3, 4, 1, 1], [1, 4, 1, 0], [1, 4, 1, 34], [1, 65, 1, 1],
                [2, 4, 3, 1], [2, 4, 1, 0], [2, 0, 1, 1]):
        with pytest.raises(M.MgarError):
            h.mgar_tune_set(0, 0, 1, bad)
    assert h.mgar_tune_get(0, 0, 1) == before
    p2 = W.tiny_2d(40, 40, 3)
    h2 = handle(p2)
    with pytest.raises(M.MgarError):
        h2.mgar_tune_set(0, 0, 1, [1, 8, 1, 1])     # z-marching needs 3D
    with pytest.raises(M.MgarError):
        h2.mgar_tune_set(0, 0, 1, [2, 8, 1, 1])
    with pytest.raises(M.MgarError):
        h.mgar_tune_set(0, 9, 1, [0, 0, 0, 0])      # no such level


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_solves_after_autotune_match_oracle(precision):
    import torch
    prob = W.tiny_3d(32, 32, 32, 4)
    h = handle(prob, precision=precision)
    best = h.mgar_autotune(3)
    assert best[0][0][1] > 0.0                      # finest apply + dot was timed
    if precision == 1:
        assert best[1][0][1] > 0.0
    q = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgar_load_vector(dev(W.element_source(prob)), q)
    xphys = W.random_density(prob.nelem, 11, 0.0, 1.0)
    s = solvers.MgarSolver(prob, solvers.MgarParams(cg_max=200))
    t_or, st_or = s.mgcg(xphys, np.zeros(prob.nnodes), 1e-8)
    T = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    st = h.mgcg_solve(dev(xphys), q, None, 1e-8, T)
    assert st["rc"] == 0
    if precision == 0:
        assert st["cg_iters"] == st_or.cg_iters
        assert rel_l2(host(T), t_or) < 1e-8
    else:
        assert rel_l2(host(T), t_or) < 1e-6


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_solves_with_two_row_shapes_match_oracle(precision):
    """Every stencil mode of the two finest grids on two-row shapes (FP64 class,
    and the FP32 class in mixed precision): MGCG and MGAR still match the oracle."""
    import torch
    prob = W.tiny_3d(32, 32, 32, 4)
    h = handle(prob, precision=precision)
    for cls in range(precision + 1):
        for mode in range(7):
            h.mgar_tune_set(cls, 0, mode, [2, 6, 2, 1])
            h.mgar_tune_set(cls, 1, mode, [2, 5, 1, 1])
    q = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgar_load_vector(dev(W.element_source(prob)), q)
    s = solvers.MgarSolver(prob, solvers.MgarParams(cg_max=200))
    x0 = W.random_density(prob.nelem, 21, 0.2, 0.8)
    x1 = np.clip(x0 + 0.02 * W.random_vector(prob.nelem, 22), 0, 1)
    t0, st0 = s.mgcg(x0, np.zeros(prob.nnodes), 1e-8)
    T0 = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    T1 = torch.empty_like(T0)
    st = h.mgcg_solve(dev(x0), q, None, 1e-8, T0)
    assert st["rc"] == 0
    t1, st1 = s.mgar(x1, t0, 1e-8)
    sa = h.mgar_solve(dev(x1), q, T0, 1e-8, T1)
    assert sa["rc"] == 0
    tol = 1e-8 if precision == 0 else 1e-6
    assert rel_l2(host(T0), t0) < tol
    assert rel_l2(host(T1), t1) < tol
    if precision == 0:
        assert st["cg_iters"] == st0.cg_iters
        assert sa["path"] == st1.path and sa["cg_iters"] == st1.cg_iters


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("prob", [W.tiny_3d(32, 32, 32, 4), W.tiny_3d(48, 32, 16, 3)],
                         ids=["32x32x32", "48x32x16"])
def test_fused_launches_match_separate_launches(prob, precision):
    """A two-row shape for the finest apply + dot runs the CG direction update
    inside the apply (double-buffered direction), and one for the finest
    residual runs the V-cycle's first sweep inside it; any other shape runs
    them as separate launches. Same iterations, same temperature (to the
    summation order of the dot partials), both on the oracle. In mixed
    precision the same holds for the FP32 inner solver (oracle to 1e-6)."""
    import torch
    s = solvers.MgarSolver(prob, solvers.MgarParams(cg_max=200))
    x0 = W.random_density(prob.nelem, 41, 0.1, 0.9)
    x1 = np.clip(x0 + 0.03 * W.random_vector(prob.nelem, 42), 0, 1)
    t0, st0 = s.mgcg(x0, np.zeros(prob.nnodes), 1e-8)
    t1, st1 = s.mgar(x1, t0, 1e-8)
    out = {}
    for name, shape in (("fused", [2, 6, 1, 1]), ("separate", [1, 6, 1, 1])):
        h = handle(prob, precision=precision)
        for cls in range(precision + 1):
            h.mgar_tune_set(cls, 0, 1, shape)
            h.mgar_tune_set(cls, 0, 2, shape)
        q = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
        h.mgar_load_vector(dev(W.element_source(prob)), q)
        T0 = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
        T1 = torch.empty_like(T0)
        a = h.mgcg_solve(dev(x0), q, None, 1e-8, T0)
        b = h.mgar_solve(dev(x1), q, T0, 1e-8, T1)
        tol = 1e-8 if precision == 0 else 1e-6
        if precision == 0:
            assert a["cg_iters"] == st0.cg_iters and b["cg_iters"] == st1.cg_iters
        assert b["path"] == st1.path
        assert rel_l2(host(T0), t0) < tol and rel_l2(host(T1), t1) < tol
        out[name] = (host(T0), host(T1))
    for u, v in zip(out["fused"], out["separate"]):
        assert rel_l2(u, v) < (1e-12 if precision == 0 else 1e-6)
