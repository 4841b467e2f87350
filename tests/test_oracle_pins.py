"""Pins for the CPU oracle: closed forms, invariants, exact special cases and
brute force on tiny inputs. None of these re-types an oracle formula; each is
chosen so that a plausible mistake (dropped term, wrong sign, wrong index,
transposed operand) in the oracle fails at least one of them."""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import fe, mg, solvers, topopt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- P1: element matrix

def hamming(a, b):
    return bin(a ^ b).count("1")


def test_element_matrix_2d_closed_form():
    # Q1 unit square: 2/3 on the diagonal, -1/6 along edges, -1/3 across the diagonal.
    ke = fe.element_matrix(2)
    table = {0: 2 / 3, 1: -1 / 6, 2: -1 / 3}
    for a in range(4):
        for b in range(4):
            assert ke[a, b] == pytest.approx(table[hamming(a, b)], abs=1e-15)
    assert np.allclose(np.linalg.eigvalsh(ke), [0, 2 / 3, 1, 1], atol=1e-14)


@pytest.mark.parametrize("h", [1.0, 2.0, 4.0])
def test_element_matrix_3d_closed_form(h):
    # Q1 hexahedron of edge h: h/3 diagonal, 0 along edges, -h/12 across faces and body.
    ke = fe.element_matrix(3, h)
    table = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}
    for a in range(8):
        for b in range(8):
            assert ke[a, b] == pytest.approx(h * table[hamming(a, b)], abs=1e-14)
    assert np.allclose(np.linalg.eigvalsh(ke / h),
                       [0, 1 / 6, 1 / 3, 1 / 3, 1 / 3, 1 / 2, 1 / 2, 1 / 2], atol=1e-14)


def test_element_matrix_2d_scale_invariant():
    assert np.allclose(fe.element_matrix(2, 4.0), fe.element_matrix(2, 1.0), atol=1e-15)


def test_element_load_is_volume_share():
    assert np.allclose(fe.element_load(2), 0.25)
    assert np.allclose(fe.element_load(3, 2.0), 8.0 / 8)


def test_assembled_interior_stencils():
    g2 = fe.Grid(2, 4, 4)
    K2 = fe.assemble(g2, np.ones(g2.nelem)).toarray()
    c = g2.node_id(2, 2)
    assert K2[c, c] == pytest.approx(8 / 3)
    for di, dj in itertools.product((-1, 0, 1), repeat=2):
        if (di, dj) != (0, 0):
            assert K2[c, g2.node_id(2 + di, 2 + dj)] == pytest.approx(-1 / 3)
    g3 = fe.Grid(3, 4, 4, 4)
    K3 = fe.assemble(g3, np.ones(g3.nelem)).toarray()
    c = g3.node_id(2, 2, 2)
    want = {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}
    for off in itertools.product((-1, 0, 1), repeat=3):
        n = sum(abs(o) for o in off)
        assert K3[c, g3.node_id(2 + off[0], 2 + off[1], 2 + off[2])] == pytest.approx(want[n], abs=1e-15)


def test_numbering_convention():
    g = fe.Grid(3, 3, 2, 2)
    conn = g.connectivity()
    e = g.elem_id(1, 1, 1)
    assert e == 1 + 3 * (1 + 2 * 1)
    # corner c = bx + 2 by + 4 bz
    assert conn[e, 0] == g.node_id(1, 1, 1)
    assert conn[e, 1] == g.node_id(2, 1, 1)
    assert conn[e, 2] == g.node_id(1, 2, 1)
    assert conn[e, 7] == g.node_id(2, 2, 2)
    assert g.node_id(2, 2, 2) == 2 + 4 * (2 + 3 * 2)


def test_paper_dof_counts():
    with open(os.path.join(GOLDEN, "paper_dof_counts.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for r in rows:
        d, nx, ny, nz, dofs = (int(v) for v in r[:5])
        assert fe.Grid(d, nx, ny, nz).nnodes == dofs


def test_sink_boxes():
    assert W.C0.fix_lo == (0, 18, 0) and W.C0.fix_hi == (0, 22, 0)
    assert W.C1.fix_lo[1] == 144 and W.C1.fix_hi[1] == 176
    assert W.C2.fix_lo[:2] == (26, 26) and W.C2.fix_hi[:2] == (38, 38)
    assert W.C3.fix_lo[:2] == (52, 52) and W.C3.fix_hi[:2] == (76, 76)


# ---------------------------------------------------------------- P2: patch test

@pytest.mark.parametrize("dim", [2, 3])
def test_patch_linear_field(dim):
    g = fe.Grid(dim, 5, 4, 3 if dim == 3 else 0)
    K = fe.assemble(g, np.full(g.nelem, 0.7))
    nc = g.node_coords().astype(float)
    T = 1.3 + 0.5 * nc[:, 0] - 2.0 * nc[:, 1] + (0.25 * nc[:, 2] if dim == 3 else 0)
    y = K @ T
    interior = np.ones(g.nnodes, bool)
    for a, n in enumerate([g.nx, g.ny] + ([g.nz] if dim == 3 else [])):
        interior &= (nc[:, a] > 0) & (nc[:, a] < n)
    assert np.abs(y[interior]).max() < 1e-13
    # constants are in the kernel everywhere (zero row sums)
    assert np.abs(K @ np.ones(g.nnodes)).max() < 1e-13


# apply_rows: the row-by-row element sum used to check grids too large to assemble

@pytest.mark.parametrize("dim,shape", [(2, (7, 5, 0)), (3, (5, 4, 6)), (3, (3, 3, 3))])
def test_apply_rows_equals_assembled_rows(dim, shape):
    """fe.apply_rows on every node (corners, edges, faces, interior) equals the
    rows of the assembled matrix, with per-element conductivities that differ
    everywhere, so a wrong corner index or boundary mask shows in some row."""
    g = fe.Grid(dim, *shape)
    k = W.random_density(g.nelem, 91, 1e-3, 1.0)
    x = W.random_vector(g.nnodes, 92)
    want = fe.assemble(g, k) @ x
    rows = np.arange(g.nnodes)
    got = fe.apply_rows(g, k, x, rows)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
    # an arbitrary subset in arbitrary order, with repeats
    rng = np.random.default_rng(93)
    sub = rng.integers(0, g.nnodes, 50)
    assert np.array_equal(fe.apply_rows(g, k, x, sub), got[sub])


@pytest.mark.parametrize("dim", [2, 3])
def test_apply_rows_matches_hamming_table_by_hand(dim):
    """Independent of the oracle's element matrix: each row summed by hand from
    the closed-form Hamming-distance table of the Q1 element (2D 2/3, -1/6,
    -1/3; 3D 1/3, 0, -1/12, -1/12), over the elements that contain the node."""
    table = {2: {0: 2 / 3, 1: -1 / 6, 2: -1 / 3}, 3: {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}}[dim]
    g = fe.Grid(dim, 4, 3, 2 if dim == 3 else 0)
    k = W.random_density(g.nelem, 94, 1e-3, 1.0)
    x = W.random_vector(g.nnodes, 95)
    n = [g.nx, g.ny] + ([g.nz] if dim == 3 else [])
    rows = np.arange(g.nnodes)
    got = fe.apply_rows(g, k, x, rows)
    for nid in rows:
        ijk = [int(nid % g.nnx), int((nid // g.nnx) % g.nny), int(nid // (g.nnx * g.nny))][:dim]
        y = 0.0
        for e in itertools.product(*[range(max(0, c - 1), min(c, m - 1) + 1) for c, m in zip(ijk, n)]):
            eid = e[0] + g.nx * (e[1] + (g.ny * e[2] if dim == 3 else 0))
            ci = sum((ijk[a] - e[a]) << a for a in range(dim))
            for c in range(2 ** dim):
                nb = [e[a] + ((c >> a) & 1) for a in range(dim)]
                j = nb[0] + g.nnx * (nb[1] + (g.nny * nb[2] if dim == 3 else 0))
                y += k[eid] * table[hamming(ci, c)] * x[j]
        assert abs(got[nid] - y) < 1e-13 * max(1.0, abs(y)), (nid, got[nid], y)


# ---------------------------------------------------------------- P3: 1D analytic solution

@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_slab_matches_1d_exact(dim):
    L = 8
    nz = 2 if dim == 3 else 0
    prob = W.Problem(name="slab", dim=dim, nelx=L, nely=4, nelz=nz, levels=1,
                     fix_lo=(0, 0, 0), fix_hi=(0, 4, nz), source=0.3)
    fep = fe.FEProblem(prob)
    K = fe.assemble(fep.grid, np.full(fep.grid.nelem, 2.0))[fep.free][:, fep.free]
    t = fep.to_full(solvers.exact_solve(K, fep.to_free(fep.q)))
    x = fep.grid.node_coords()[:, 0].astype(float)
    exact = (0.3 / 2.0) * (L * x - x * x / 2.0)
    assert np.abs(t - exact).max() < 1e-12 * exact.max()


# ---------------------------------------------------------------- P5: transfers and coarse ops

@pytest.mark.parametrize("dim", [2, 3])
def test_interpolation_reproduces_linear(dim):
    nx, ny, nz = 4, 6, (4 if dim == 3 else 0)
    P = mg.interpolation(dim, nx, ny, nz)
    gc = fe.Grid(dim, nx // 2, ny // 2, nz // 2 if dim == 3 else 0, h=2.0)
    gf = fe.Grid(dim, nx, ny, nz)
    cc = gc.node_coords() * 2.0
    cf = gf.node_coords().astype(float)
    lin = lambda c: 0.5 + c[:, 0] - 0.25 * c[:, 1] + 0.3 * c[:, 2]
    assert np.abs(P @ lin(cc) - lin(cf)).max() < 1e-13
    # bilinear x*y field is reproduced too (tensor-product interpolation)
    bil = lambda c: c[:, 0] * c[:, 1]
    assert np.abs(P @ bil(cc) - bil(cf)).max() < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_galerkin_equals_rediscretised_for_blockwise_uniform_k(dim):
    n = 4
    prob = W.tiny_2d(n, n, 2) if dim == 2 else W.tiny_3d(n, n, n, 2)
    rng = np.random.default_rng(3)
    kc = rng.uniform(1e-3, 1.0, (n // 2) ** dim)
    # children inherit their parent's value
    if dim == 2:
        k = np.kron(kc.reshape(n // 2, n // 2), np.ones((2, 2))).ravel()
    else:
        k = np.kron(kc.reshape(n // 2, n // 2, n // 2), np.ones((2, 2, 2))).ravel()
    h = mg.Hierarchy(prob, k)
    G = (h.P[0].T @ h.levels[0].K @ h.P[0]).toarray()
    assert np.abs(G - h.levels[1].K.toarray()).max() < 1e-13
    assert np.allclose(h.levels[1].k, kc)


def test_coarse_dirichlet_rule_c0():
    h = mg.Hierarchy(W.C0, np.ones(W.C0.nelem))
    assert [int(lv.fixed.sum()) for lv in h.levels] == [5, 3, 1]
    assert h.levels[2].grid.nnodes == 121


def test_coarse_dirichlet_rule_c3_counts():
    # counts only (no assembly at this size)
    g = fe.Grid(3, 128, 128, 128)
    fixed = fe.fixed_mask_from_box(g, W.C3.fix_lo, W.C3.fix_hi)
    assert fixed.sum() == 625


# ---------------------------------------------------------------- P6: V-cycle

@pytest.mark.parametrize("prob", [W.tiny_2d(16, 16, 3), W.tiny_3d(8, 8, 8, 3)])
def test_vcycle_symmetric_positive_contractive(prob):
    k = fe.simp(W.random_density(prob.nelem, 1, 0.05, 1.0))
    h = mg.Hierarchy(prob, k)
    n = h.levels[0].free.size
    u, v = W.random_vector(n, 1), W.random_vector(n, 2)
    Mu, Mv = h.precond(u), h.precond(v)
    assert abs(u @ Mv - Mu @ v) < 1e-12 * np.linalg.norm(u) * np.linalg.norm(Mv)
    assert u @ Mu > 0 and v @ Mv > 0
    # error propagation E = I - M K has spectral radius < 1 (power iteration)
    K = h.levels[0].K
    e = W.random_vector(n, 3)
    for _ in range(30):
        e = e - h.precond(K @ e)
        nrm = np.linalg.norm(e)
        e /= nrm
    assert nrm < 1.0


def test_vcycle_two_level_exact_when_coarse_is_all():
    # a 1-level hierarchy is an exact solve
    prob = W.tiny_2d(4, 4, 1)
    k = fe.simp(W.random_density(prob.nelem, 5, 0.1, 1.0))
    h = mg.Hierarchy(prob, k)
    b = W.random_vector(h.levels[0].free.size, 4)
    x = h.precond(b)
    assert np.linalg.norm(h.levels[0].K @ x - b) < 1e-12 * np.linalg.norm(b)


# ---------------------------------------------------------------- P4, P7: solves

@pytest.mark.parametrize("prob", [W.tiny_2d(16, 16, 3), W.tiny_3d(8, 8, 8, 3), W.tiny_2d(8, 16, 2)])
def test_mgcg_matches_dense_solve(prob):
    xphys = W.random_density(prob.nelem, 7, 0.0, 1.0)
    s = solvers.MgarSolver(prob, solvers.MgarParams(cg_max=200))
    t, st = s.mgcg(xphys, np.zeros(prob.nnodes), 1e-12)
    fep = s.fep
    Kd = fep.K_free(xphys).toarray()
    td = fep.to_full(np.linalg.solve(Kd, fep.to_free(fep.q)))
    assert st.converged
    assert np.linalg.norm(t - td) < 1e-9 * np.linalg.norm(td)
    assert np.all(t[fep.fixed] == 0)


# ---------------------------------------------------------------- P8: reanalysis

def _ca_setup(seed=11):
    prob = W.tiny_2d(16, 16, 3)
    s = solvers.MgarSolver(prob, solvers.MgarParams(n_basis=3))
    x0 = W.random_density(prob.nelem, seed, 0.2, 0.8)
    t0, _ = s.mgcg(x0, np.zeros(prob.nnodes), 1e-12)
    x1 = np.clip(x0 + 0.05 * W.random_vector(prob.nelem, seed), 0, 1)
    _, K = s._setup(x1)
    return prob, s, t0, K


def test_ca_is_galerkin_projection_brute_force():
    prob, s, t0, K = _ca_setup()
    qf = s.fep.to_free(s.q)
    R = s.basis(K, s.fep.to_free(t0))
    t, res, Q, y = s.reduced_solution(K, R, qf)
    # brute force: minimise 1/2 v^T K v - q^T v over v = R c with the raw basis
    Kd = K.toarray()
    c = np.linalg.solve(R.T @ Kd @ R, R.T @ qf)
    tb = R @ c
    assert np.linalg.norm(t - tb) < 1e-10 * np.linalg.norm(tb)
    # invariance to column order and scaling
    R2 = R[:, ::-1] * np.array([3.0, -0.5, 7.0])
    t2, _, _, _ = s.reduced_solution(K, R2, qf)
    assert np.linalg.norm(t - t2) < 1e-10 * np.linalg.norm(t)
    # invariance to the orthonormalisation method (Eq 18 uses an SVD)
    U, _, _ = np.linalg.svd(R, full_matrices=False)
    tsvd = U @ np.linalg.solve(U.T @ Kd @ U, U.T @ qf)
    assert np.linalg.norm(t - tsvd) < 1e-10 * np.linalg.norm(t)
    # Res of Eq 28 and the energy identity q^T t~ = t~^T K t~
    assert res == pytest.approx(np.linalg.norm(Kd @ t - qf) / np.linalg.norm(qf), rel=1e-10)
    assert qf @ t == pytest.approx(t @ Kd @ t, rel=1e-12)


def test_ca_single_vector_and_exact_span():
    prob, s, t0, K = _ca_setup(12)
    qf = s.fep.to_free(s.q)
    r1 = s.fep.to_free(t0)
    t, _, _, _ = s.reduced_solution(K, r1[:, None], qf)
    want = (r1 @ qf) / (r1 @ (K @ r1)) * r1
    assert np.linalg.norm(t - want) < 1e-12 * np.linalg.norm(want)
    ts = solvers.exact_solve(K, qf)
    t, res, _, _ = s.reduced_solution(K, np.stack([ts, r1], 1), qf)
    assert np.linalg.norm(t - ts) < 1e-9 * np.linalg.norm(ts)
    assert res < 1e-9


def test_ca_energy_error_nonincreasing_in_m():
    prob, s, t0, K = _ca_setup(13)
    qf = s.fep.to_free(s.q)
    ts = solvers.exact_solve(K, qf)
    Kd = K.toarray()
    errs = []
    for m in (1, 2, 3):
        s.params.n_basis = m
        R = s.basis(K, s.fep.to_free(t0))
        t, _, _, _ = s.reduced_solution(K, R, qf)
        e = t - ts
        errs.append(e @ Kd @ e)
    assert errs[1] <= errs[0] * (1 + 1e-12) and errs[2] <= errs[1] * (1 + 1e-12)


def test_ca_basis_exact_neumann_series_when_mg_exact():
    # With a 1-level hierarchy the V-cycle is an exact K0 solve, so the basis
    # is the binomial series of Eq 13-15: K0 r_i = -dK r_{i-1}.
    prob = W.tiny_2d(6, 6, 1)
    s = solvers.MgarSolver(prob, solvers.MgarParams(n_basis=3, basis_x0_zero=True))
    x0 = W.random_density(prob.nelem, 21, 0.3, 0.7)
    t0, _ = s.mgcg(x0, np.zeros(prob.nnodes), 1e-13)
    x1 = np.clip(x0 + 0.03, 0, 1)
    _, K = s._setup(x1)
    R = s.basis(K, s.fep.to_free(t0))
    K0 = s.K0.toarray()
    dK = K.toarray() - K0
    for i in (1, 2):
        assert np.linalg.norm(K0 @ R[:, i] + dK @ R[:, i - 1]) < 1e-10 * np.linalg.norm(dK @ R[:, i - 1])


def test_mgar_fallback_and_accept_paths():
    prob = W.tiny_2d(16, 16, 3)
    s = solvers.MgarSolver(prob, solvers.MgarParams(n_basis=2, eps_accept=1e-8))
    x0 = W.random_density(prob.nelem, 31, 0.2, 0.8)
    t0, _ = s.mgcg(x0, np.zeros(prob.nnodes), 1e-10)
    # same design: t_prev is already the solution, the basis spans it -> accept
    t, st = s.mgar(x0, t0, 1e-10)
    assert st.path == solvers.PATH_ACCEPT and st.res_ca < 1e-8
    # changed design with tight eps1 -> fallback, result is the solve to tol
    x1 = np.clip(x0 + 0.1, 0, 1)
    t, st = s.mgar(x1, t0, 1e-10)
    assert st.path == solvers.PATH_FALLBACK
    fep = s.fep
    td = fep.to_full(solvers.exact_solve(fep.K_free(x1), fep.to_free(fep.q)))
    assert np.linalg.norm(t - td) < 1e-7 * np.linalg.norm(td)
    assert np.allclose(s.k0, fep.kelem(x1))


# ---------------------------------------------------------------- P10: filter

@pytest.mark.parametrize("dim,r,taps", [(2, 1.5, 9), (2, 3.0, 25), (3, 2.0, 27), (3, 1.5, 19)])
def test_filter_tap_counts(dim, r, taps):
    g = fe.Grid(dim, 9, 9, 9 if dim == 3 else 0)
    H, _ = topopt.filter_matrix(g, r)
    centre = g.elem_id(4, 4, 4 if dim == 3 else 0)
    assert H[centre].nnz == taps


@pytest.mark.parametrize("dim,r", [(2, 1.5), (2, 3.0), (3, 2.0)])
def test_filter_brute_force_and_adjoint(dim, r):
    g = fe.Grid(dim, 6, 5, 4 if dim == 3 else 0)
    f = topopt.Filter(g, r)
    x = W.random_density(g.nelem, 2)
    assert np.abs(f.forward(x) - topopt.filter_brute(g, r, x)).max() < 1e-14
    assert np.abs(f.forward(np.full(g.nelem, 0.37)) - 0.37).max() < 1e-15
    gvec = W.random_vector(g.nelem, 9)
    assert f.forward(x) @ gvec == pytest.approx(x @ f.adjoint(gvec), rel=1e-13)
    assert (abs(f.H - f.H.T)).max() == 0


# ---------------------------------------------------------------- P9: sensitivities

@pytest.mark.parametrize("prob", [W.tiny_2d(6, 6, 2, filter_r=1.5), W.tiny_3d(4, 4, 4, 2)])
def test_sensitivity_finite_difference(prob):
    fep = fe.FEProblem(prob)
    filt = topopt.Filter(fep.grid, prob.filter_r)
    x = W.random_density(prob.nelem, 17, 0.2, 0.9)

    def comp(xx):
        xp = filt.forward(xx)
        t = fep.to_full(solvers.exact_solve(fep.K_free(xp), fep.to_free(fep.q)))
        return fep.q @ t, xp, t

    f0, xp, t = comp(x)
    f, dc, dv, _ = topopt.sensitivity(fep, filt, xp, t)
    assert f == pytest.approx(f0)
    Kf = fep.K_free(xp)
    tf = fep.to_free(t)
    assert f == pytest.approx(tf @ (Kf @ tf), rel=1e-12)
    for e in (0, prob.nelem // 2, prob.nelem - 1):
        eps = 1e-6
        xp_, xm_ = x.copy(), x.copy()
        xp_[e] += eps
        xm_[e] -= eps
        fd = (comp(xp_)[0] - comp(xm_)[0]) / (2 * eps)
        assert dc[e] == pytest.approx(fd, rel=1e-6)
        vd = (filt.forward(xp_).sum() - filt.forward(xm_).sum()) / (2 * eps)
        assert dv[e] == pytest.approx(vd, rel=1e-8)


# ---------------------------------------------------------------- P11: OC

def test_oc_volume_and_bounds():
    prob = W.tiny_2d(12, 12, 2)
    fep = fe.FEProblem(prob)
    filt = topopt.Filter(fep.grid, 1.5)
    x = W.random_density(prob.nelem, 4, 0.2, 0.6)
    dc = -np.abs(W.random_vector(prob.nelem, 5)) - 0.01
    _, _, dv, _ = topopt.sensitivity(fep, filt, filt.forward(x), np.zeros(prob.nnodes))
    xn, lam, steps = topopt.oc_update(x, dc, dv, filt, 0.4, 0.2)
    assert abs(filt.forward(xn).mean() - 0.4) < 1e-6
    assert np.all(xn >= 0) and np.all(xn <= 1)
    assert np.all(xn >= x - 0.2 - 1e-15) and np.all(xn <= x + 0.2 + 1e-15)
    # filtered volume equals the w . x identity with w = H^T (1 / Hs) = dv
    assert filt.forward(xn).sum() == pytest.approx(dv @ xn, rel=1e-13)
    assert 20 < steps < 120


def test_n_on():
    assert [topopt.n_on(m) for m in (50, 100, 80, 300)] == [6, 13, 10, 40]


# ---------------------------------------------------------------- loop sanity

def test_loop_c0_compliance_decreases_and_paths():
    x, xp, t, recs = topopt.run_loop(W.C0, maxit=12)
    assert [r.path for r in recs[:5]] == [0] * 5
    assert all(r.path in (1, 2) for r in recs[5:])
    assert recs[-1].compliance < recs[0].compliance
    assert abs(xp.mean() - 0.4) < 1e-6


# ---------------------------------------------------------------- continuous filtering (Eq 22-23)

def test_continuous_radii_closed_form():
    """The recurrence of Eq 22-23 reaches r_min exactly after lp steps, follows
    r0 (r_min / r0)^(k / lp) on the way (geometric), never goes below r_min and
    stays there; r0 = 1.4 L / 50 is 13.44 for the paper's 480-element side."""
    r0 = 1.4 * 480 / 50
    assert abs(r0 - 13.44) < 1e-12
    lp = 250
    radii = topopt.continuous_radii(3.0, r0, lp, 300)
    assert radii[0] == r0
    for k in range(lp + 1):
        assert abs(radii[k] - r0 * (3.0 / r0) ** (k / lp)) <= 1e-12 * r0
    assert abs(radii[lp] - 3.0) < 1e-12
    assert all(r >= 3.0 for r in radii)
    assert all(a >= b for a, b in zip(radii, radii[1:]))
    assert all(r == 3.0 for r in radii[lp + 1:])


def test_loop_radii_schedule_and_fixed():
    prob = W.paper_2d(480, 6)
    radii = topopt.loop_radii(prob, prob.maxit, {"r_min": 3.0})
    assert len(radii) == 300 and abs(radii[0] - 13.44) < 1e-12
    assert abs(radii[250] - 3.0) < 1e-12       # lp = 5/6 of 300 steps after cycle 1
    assert radii[251:] == [3.0] * 49
    assert topopt.loop_radii(W.C0, 7, None) == [W.C0.filter_r] * 7


@pytest.mark.parametrize("dim,r", [(2, 4.7), (2, 6.2), (3, 3.3)])
def test_filter_large_radius_brute_force(dim, r):
    """The sparse filter at the larger radii of the continuous schedule against
    the O(E^2) statement of Eq 6-8, constant fields preserved."""
    g = fe.Grid(dim, 13, 11, 7 if dim == 3 else 0)
    x = W.random_density(g.nelem, 71)
    filt = topopt.Filter(g, r)
    assert np.abs(filt.forward(x) - topopt.filter_brute(g, r, x)).max() < 1e-13
    assert np.abs(filt.forward(np.full(g.nelem, 0.37)) - 0.37).max() < 1e-14


def test_continuous_loop_uses_schedule():
    prob = W.tiny_2d(80, 80, 3, maxit=30)
    _, _, _, recs = topopt.run_loop(prob, maxit=6, continuous={"r_min": 1.2, "lp": 3})
    want = topopt.continuous_radii(1.2, 1.4 / 50 * 80, 3, 6)
    assert np.allclose([r.radius for r in recs], want, rtol=1e-15, atol=0)
    assert abs(recs[0].radius - 2.24) < 1e-12 and recs[3].radius == 1.2
    small = W.tiny_2d(16, 16, 2, maxit=30)
    assert topopt.loop_radii(small, 4, {"r_min": 1.5}) == [1.5] * 4


# ---------------------------------------------------------------- non-uniform source (Sec. 4.2)

def test_quadrant_source_layout_and_total():
    p = W.tiny_2d(8, 6, 2)
    qe = W.quadrant_source(p).reshape(6, 8)
    v = W.QUADRANT_SOURCES
    assert np.all(qe[:3, :4] == v[0]) and np.all(qe[:3, 4:] == v[1])
    assert np.all(qe[3:, :4] == v[2]) and np.all(qe[3:, 4:] == v[3])
    assert abs(qe.sum() - 12 * sum(v)) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_load_vector_partition_of_unity_and_linearity(dim):
    """With no Dirichlet node the nodal loads add up to the total heat
    sum_e Q_e |e| (the shape functions sum to one), and q is linear in Q."""
    g = fe.Grid(dim, 6, 4, 3 if dim == 3 else 0, h=2.0)
    none = np.zeros(g.nnodes, dtype=bool)
    qa = W.random_density(g.nelem, 81)
    qb = W.random_density(g.nelem, 82)
    vol = g.h ** dim
    la = fe.load_vector(g, qa, none)
    assert abs(la.sum() - qa.sum() * vol) < 1e-13 * qa.sum() * vol
    lab = fe.load_vector(g, 2.0 * qa + qb, none)
    assert np.abs(lab - (2.0 * la + fe.load_vector(g, qb, none))).max() < 1e-15 * np.abs(lab).max() * 10
    # a source confined to one element loads its corners only, |e| / 2^d each
    one = np.zeros(g.nelem)
    one[5] = 1.0
    l1 = fe.load_vector(g, one, none)
    corners = g.connectivity()[5]
    assert np.allclose(l1[corners], vol / 2 ** dim, rtol=0, atol=1e-15)
    assert np.count_nonzero(l1) == 2 ** dim


# ---------------------------------------------------------------- boundary smoothing (Eq 24-27)

from oracle import smoothing  # noqa: E402


@pytest.mark.parametrize("dim", [2, 3])
def test_smoothing_projection_constant_and_weights(dim):
    g = fe.Grid(dim, 5, 4, 3 if dim == 3 else 0)
    assert np.allclose(smoothing.project_to_nodes(g, np.full(g.nelem, 0.7), 1.5), 0.7, rtol=0, atol=1e-15)
    # r just above the half-diagonal: a node sees exactly its adjacent elements, equally weighted
    s = W.random_density(g.nelem, 3)
    ns = smoothing.project_to_nodes(g, s, np.sqrt(dim) / 2 + 0.01)
    for nid in (0, g.nnodes - 1, g.node_id(2, 2, 1 if dim == 3 else 0)):
        ijk = [int(nid % g.nnx), int((nid // g.nnx) % g.nny), int(nid // (g.nnx * g.nny))][:dim]
        n = [g.nx, g.ny] + ([g.nz] if dim == 3 else [])
        adj = [e for e in itertools.product(*[range(max(0, c - 1), min(c, m - 1) + 1) for c, m in zip(ijk, n)])]
        want = np.mean([s[e[0] + g.nx * (e[1] + (g.ny * e[2] if dim == 3 else 0))] for e in adj])
        assert abs(ns[nid] - want) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_lattice_weights(dim):
    """Eq 26: partition of unity, 1 at its own corner and 0 at the others, and
    exact interpolation of a linear field over the element."""
    pts = smoothing.lattice(dim, 4)
    assert pts.shape == (5 ** dim, dim)
    N = smoothing.q1_weights(dim, pts)
    assert np.allclose(N.sum(axis=1), 1.0, atol=1e-15)
    for c in range(2 ** dim):
        corner = np.array([1.0 if (c >> a) & 1 else -1.0 for a in range(dim)])
        row = np.flatnonzero((pts == corner).all(axis=1))
        assert row.size == 1 and np.allclose(N[row[0]], np.eye(2 ** dim)[c])
    coef = np.array([0.3, -1.2, 0.7][:dim])
    corner_vals = np.array([0.5 + sum(coef[a] * (1.0 if (c >> a) & 1 else -1.0) for a in range(dim))
                            for c in range(2 ** dim)])
    assert np.allclose(N @ corner_vals, 0.5 + pts @ coef, atol=1e-14)


def test_smoothed_density_cases_by_hand():
    g = fe.Grid(2, 1, 1)
    # nodes 0..3 at (0,0), (1,0), (0,1), (1,1)
    assert smoothing.smoothed_density(g, np.array([2.0, 3.0, 4.0, 5.0]), 1.0)[0] == 1.0
    assert smoothing.smoothed_density(g, np.array([2.0, 3.0, 4.0, 5.0]), 6.0)[0] == 0.0
    # linear in x through the level at the element centre: lattice columns x = 0.5, 1 exceed it
    ns = np.array([-1.0, 1.0, -1.0, 1.0])
    assert smoothing.smoothed_density(g, ns, 0.0)[0] == pytest.approx(10 / 25, abs=0)
    assert smoothing.smoothed_density(g, ns, 0.0, nsub=2)[0] == pytest.approx(3 / 9, abs=0)
    # a node exactly at the level keeps the element mixed (Eq 24 needs strict inequalities)
    ns = np.array([1.0, 2.0, 2.0, 2.0])
    assert smoothing.smoothed_density(g, ns, 1.0)[0] == pytest.approx(24 / 25, abs=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_smoothed_density_brute_force(dim):
    """Eq 24-27 with pure-Python loops over elements and lattice points."""
    g = fe.Grid(dim, 4, 3, 2 if dim == 3 else 0)
    ns = W.random_vector(g.nnodes, 61)
    level = 0.1
    got = smoothing.smoothed_density(g, ns, level, nsub=3)
    conn = g.connectivity()
    t = [-1.0, -1 / 3, 1 / 3, 1.0]
    for e in range(g.nelem):
        v = ns[conn[e]]
        if all(v > level):
            want = 1.0
        elif all(v < level):
            want = 0.0
        else:
            cnt = tot = 0
            for o in itertools.product(t, repeat=dim):
                val = 0.0
                for c in range(2 ** dim):
                    w = 1.0
                    for a in range(dim):
                        w *= (1.0 + o[a] * (1.0 if (c >> a) & 1 else -1.0)) / 2.0
                    val += w * v[c]
                cnt += val > level
                tot += 1
            want = cnt / tot
        assert got[e] == pytest.approx(want, abs=1e-15), e


def test_smoothing_level_keeps_volume():
    g = fe.Grid(2, 24, 20)
    s = -W.random_density(g.nelem, 62) - np.linspace(0, 1, g.nelem)
    rho, ns, level, vol = smoothing.smooth_boundary(g, s, 0.4, 1.5)
    target = 0.4 * g.nelem
    assert vol >= target and vol - target < 1.0           # within one element of the target
    # monotone in the level, and the level is where the volume crosses the target
    levels = np.linspace(ns.min() - 0.1, ns.max() + 0.1, 40)
    vols = [smoothing.smoothed_density(g, ns, L).sum() for L in levels]
    assert all(a >= b for a, b in zip(vols, vols[1:]))
    assert smoothing.smoothed_density(g, ns, level + 1e-9 * (ns.max() - ns.min())).sum() <= vol
    assert np.all((rho >= 0) & (rho <= 1))
