"""Edge cases of the single-design entry points on the GPU: parameter and
state errors with their codes, and the degenerate solves (zero source, exact
initial guess, uniform void and solid designs, reanalysis from a zero
previous temperature), checked against the FP64 CPU oracle."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import solvers
from tests.gpu_util import dev, host, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

P2 = W.C0                      # 2D 40 x 40, 3 grids
P3 = W.tiny_3d(16, 16, 16, 3)


def _handle(prob, **kw):
    require_gpu()
    from paper_2210_00947_amd import mgar as M
    return M, M.Handle(M.params_for(prob, **kw))


def _load(h, prob):
    import torch
    q = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgar_load_vector(dev(W.element_source(prob)), q)
    return q


@pytest.mark.parametrize("case,code", [
    ("levels beyond divisibility", -2),     # 40 elements, 2^(5-1) = 16 does not divide
    ("coarsest grid too large", -2),        # 320^2 on 2 grids: 161^2 coarsest nodes
    ("no coarsest Dirichlet node", -3),     # fix box j = 17..19 holds no multiple of 4
    ("unknown precision", -6),
    ("mixed inner_tol out of range", -1),
    ("no basis vector", -1),
])
def test_setup_rejects_bad_parameters(case, code):
    require_gpu()
    from paper_2210_00947_amd import mgar as M
    prob, kw = P2, {}
    if case == "levels beyond divisibility":
        prob = dataclasses.replace(P2, levels=5)
    elif case == "coarsest grid too large":
        prob = dataclasses.replace(W.C1, levels=2)
    elif case == "no coarsest Dirichlet node":
        prob = dataclasses.replace(P2, fix_lo=(0, 17, 0), fix_hi=(0, 19, 0))
    elif case == "unknown precision":
        kw = {"precision": 5}
    elif case == "mixed inner_tol out of range":
        kw = {"precision": M.PREC_MIXED, "inner_tol": 1.5}
    elif case == "no basis vector":
        kw = {"n_basis": 0}
    with pytest.raises(M.MgarError) as e:
        M.Handle(M.params_for(prob, **kw))
    assert e.value.code == code


def test_reanalysis_before_any_mgcg_is_a_state_error():
    import torch
    M, h = _handle(P2)
    q = _load(h, P2)
    T = torch.zeros(P2.nnodes, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MgarError) as e:
        h.mgar_solve(dev(np.full(P2.nelem, 0.4)), q, None, 1e-8, T)
    assert e.value.code == -7


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("prob", [P2, P3], ids=["2d", "3d"])
def test_zero_source_gives_zero_in_no_iteration(prob, precision):
    import torch
    M, h = _handle(prob, precision=precision)
    q = torch.zeros(prob.nnodes, dtype=torch.float64, device="cuda")
    T = torch.full((prob.nnodes,), 7.0, dtype=torch.float64, device="cuda")
    x = dev(W.random_density(prob.nelem, 3, 0.0, 1.0))
    st = h.mgcg_solve(x, q, None, 1e-8, T)
    assert st["rc"] == 0 and st["cg_iters"] == 0
    assert np.all(host(T) == 0.0)
    # reanalysis from that (zero) temperature: nothing to solve either
    st = h.mgar_solve(x, q, T, 1e-8, T)
    assert st["rc"] == 0
    assert np.all(host(T) == 0.0)


@pytest.mark.parametrize("prob", [P2, P3], ids=["2d", "3d"])
def test_converged_initial_guess_needs_no_iteration(prob):
    import torch
    M, h = _handle(prob)
    q = _load(h, prob)
    x = dev(W.random_density(prob.nelem, 4, 0.0, 1.0))
    T = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgcg_solve(x, q, None, 1e-8, T)
    T2 = torch.empty_like(T)
    st = h.mgcg_solve(x, q, T, 1e-8, T2)
    assert st["rc"] == 0 and st["cg_iters"] == 0
    assert np.array_equal(host(T2), host(T))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("value", [0.0, 1.0], ids=["void", "solid"])
@pytest.mark.parametrize("prob", [P2, P3], ids=["2d", "3d"])
def test_uniform_designs_match_oracle(prob, value, precision):
    """All-void (conductivity kmin everywhere) and all-solid designs: the
    extremes of the SIMP law, exactly representable in BF16."""
    import torch
    M, h = _handle(prob, precision=precision)
    q = _load(h, prob)
    x = np.full(prob.nelem, value)
    s = solvers.MgarSolver(prob, solvers.MgarParams(cg_max=200))
    t_or, _ = s.mgcg(x, np.zeros(prob.nnodes), 1e-8)
    T = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    st = h.mgcg_solve(dev(x), q, None, 1e-8, T)
    assert st["rc"] == 0
    assert rel_l2(host(T), t_or) < (1e-8 if precision == 0 else 1e-6)


def test_reanalysis_from_zero_previous_temperature_falls_back_and_converges():
    """T0 = 0 makes the first basis vector zero: Gram-Schmidt drops it, the
    reduced solution fails Eq 28, and the MGCG fallback returns the solution."""
    import torch
    prob = P3
    M, h = _handle(prob)
    q = _load(h, prob)
    x0 = W.random_density(prob.nelem, 5, 0.0, 1.0)
    x1 = np.clip(x0 + 0.02 * W.random_vector(prob.nelem, 6), 0.0, 1.0)
    T = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgcg_solve(dev(x0), q, None, 1e-8, T)
    st = h.mgar_solve(dev(x1), q, None, 1e-8, T)
    assert st["rc"] == 0 and st["path"] == M.PATH_FALLBACK
    s = solvers.MgarSolver(prob, solvers.MgarParams(cg_max=200))
    t_or, _ = s.mgcg(x1, np.zeros(prob.nnodes), 1e-8)
    assert rel_l2(host(T), t_or) < 1e-7
