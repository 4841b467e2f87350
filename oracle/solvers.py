"""Oracle solvers: MGCG, MGAR reanalysis, and the exact sparse direct reference.

Test infrastructure only (see the package docstring).

All vectors here are free-DOF vectors (Dirichlet DOFs eliminated) unless a
function says otherwise.

MGCG: conjugate gradients preconditioned by one V-cycle (the paper's
auxiliary and reference solver, Sec. 1 and 3.2). The paper defers its details
to the MGCG literature; the reading used is standard PCG with the
Fletcher-Reeves beta, the stopping test ||r_k|| / ||q|| <= tol evaluated on
the recursive residual before every iteration, and at most cg_max iterations.

MGAR (Sec. 2.2 and 3.1):
  1. r_1 = t_0, the temperature of the previous design cycle (Sec. 3.1).
  2. r_i = MG(K0, -dK r_{i-1}, x0, P) for i = 2..m, one V-cycle on the
     hierarchy of the factorised matrix K0 (Eq 17). The paper writes the
     initial guess as r_{i-1}; that literal reading is the default and a
     zero initial guess is available as an option.
  3. Orthonormalise the basis (Eq 18 uses PCA; Gram-Schmidt spans the same
     subspace, so the reduced solution is the same): modified Gram-Schmidt
     with one re-orthogonalisation pass, dropping a column whose norm after
     projection is below 1e-10 of its norm before.
  4. Reduced system (Eq 19-21): K_R = Q^T K Q, q_R = Q^T q, y = K_R^-1 q_R,
     t~ = Q y.
  5. Reconstruction test (Eq 28): Res = ||K Q y - q|| / ||q||. Accept t~ if
     Res <= eps1; otherwise solve with MGCG started from t~ and make the
     current matrix the new K0 (Sec. 3.1).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fe, mg

PATH_MGCG, PATH_ACCEPT, PATH_FALLBACK = 0, 1, 2


@dataclasses.dataclass
class SolveStats:
    path: int = PATH_MGCG
    cg_iters: int = 0
    vcycles: int = 0
    converged: bool = True
    res_ca: float = float("nan")
    res_final: float = float("nan")
    res_history: list = dataclasses.field(default_factory=list)


def exact_solve(K, q):
    """Sparse direct reference t* = K^-1 q (LU; no CHOLMOD in this image)."""
    return spla.splu(K.tocsc()).solve(q)


def pcg(K, q, x0, tol, cg_max, precond, stats: SolveStats = None):
    """Preconditioned CG (Fletcher-Reeves). Returns (x, iterations, converged)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = q - K @ x
    qn = np.linalg.norm(q)
    p = None
    rz_old = None
    it = 0
    hist = []
    while True:
        rel = np.linalg.norm(r) / qn
        hist.append(rel)
        if rel <= tol:
            conv = True
            break
        if it >= cg_max:
            conv = False
            break
        z = precond(r)
        rz = r @ z
        if p is None:
            p = z.copy()
        else:
            p = z + (rz / rz_old) * p
        w = K @ p
        alpha = rz / (p @ w)
        x = x + alpha * p
        r = r - alpha * w
        rz_old = rz
        it += 1
    if stats is not None:
        stats.cg_iters += it
        stats.vcycles += it
        stats.converged = conv
        stats.res_final = hist[-1]
        stats.res_history = hist
    return x, it, conv


def gram_schmidt(R, drop=1e-10):
    """Modified Gram-Schmidt with one re-orthogonalisation pass over the
    columns of R; a column whose norm after projection is below ``drop`` times
    its norm before is discarded. Returns Q with orthonormal columns."""
    cols = []
    for j in range(R.shape[1]):
        v = R[:, j].astype(np.float64, copy=True)
        n0 = np.linalg.norm(v)
        if n0 == 0.0:
            continue
        for _pass in range(2):
            for qc in cols:
                v = v - (qc @ v) * qc
        n1 = np.linalg.norm(v)
        if n1 < drop * n0:
            continue
        cols.append(v / n1)
    if not cols:
        return np.zeros((R.shape[0], 0))
    return np.stack(cols, axis=1)


@dataclasses.dataclass
class MgarParams:
    n_basis: int = 2          # m (Sec. 3.2: two basis vectors)
    eps_accept: float = 1e-8  # eps1 of Eq 28
    cg_max: int = 200
    omega: float = 0.8
    basis_x0_zero: bool = False


class MgarSolver:
    """MGCG / MGAR on one problem, holding the K0 state between calls.

    ``mgcg`` solves K(xphys) t = q and makes K(xphys) the factorised matrix
    K0. ``mgar`` uses K0 (and its hierarchy) to build the reanalysis basis
    and falls back to MGCG when the reconstruction test fails."""

    def __init__(self, prob, params: MgarParams = None, qelem=None):
        self.fep = fe.FEProblem(prob, qelem)
        self.prob = prob
        self.params = params or MgarParams()
        self.k0 = None
        self.h0 = None          # hierarchy of K0
        self.K0 = None          # finest K0 (free block)

    @property
    def q(self):
        return self.fep.q

    def _setup(self, xphys):
        k = self.fep.kelem(xphys)
        K = fe.assemble(self.fep.grid, k)[self.fep.free][:, self.fep.free].tocsr()
        return k, K

    def mgcg(self, xphys, t0_full, tol, stats=None):
        """Pure MGCG solve; sets K0 := K(xphys). Returns the full temperature vector."""
        stats = stats if stats is not None else SolveStats()
        k, K = self._setup(xphys)
        hier = mg.Hierarchy(self.prob, k, omega=self.params.omega)
        qf = self.fep.to_free(self.q)
        x, _, _ = pcg(K, qf, self.fep.to_free(t0_full), tol, self.params.cg_max,
                      hier.precond, stats)
        self.k0, self.h0, self.K0 = k, hier, K
        stats.path = PATH_MGCG
        return self.fep.to_full(x), stats

    def basis(self, K, t_prev_free):
        """Reanalysis basis R (Eq 14-17), columns r_1 .. r_m, built with one
        V-cycle on the K0 hierarchy per column."""
        m = self.params.n_basis
        dK = K - self.K0
        cols = [t_prev_free.copy()]
        for _i in range(1, m):
            prev = cols[-1]
            b = -(dK @ prev)
            x0 = np.zeros_like(prev) if self.params.basis_x0_zero else prev
            cols.append(self.h0.vcycle(0, b, x0))
        return np.stack(cols, axis=1)

    def reduced_solution(self, K, R, qf):
        """Eq 18-21 and Eq 28: orthonormalise, project, solve, and measure Res.
        Returns (t~, Res, Q, y)."""
        Q = gram_schmidt(R)
        qn = np.linalg.norm(qf)
        if Q.shape[1] == 0:
            return np.zeros_like(qf), 1.0, Q, np.zeros(0)
        W = K @ Q
        KR = Q.T @ W
        qR = Q.T @ qf
        y = sla.cho_solve(sla.cho_factor(KR, lower=True), qR)
        t = Q @ y
        res = np.linalg.norm(W @ y - qf) / qn
        return t, res, Q, y

    def mgar(self, xphys, t_prev_full, tol, stats=None):
        """One MGAR solve (Sec. 3.1). Returns the full temperature vector."""
        if self.h0 is None:
            raise RuntimeError("MGAR needs a factorised K0: call mgcg first")
        stats = stats if stats is not None else SolveStats()
        k, K = self._setup(xphys)
        qf = self.fep.to_free(self.q)
        R = self.basis(K, self.fep.to_free(t_prev_full))
        stats.vcycles += self.params.n_basis - 1
        t, res, _, _ = self.reduced_solution(K, R, qf)
        stats.res_ca = res
        if res <= self.params.eps_accept:
            stats.path = PATH_ACCEPT
            stats.res_final = res
            return self.fep.to_full(t), stats
        # Reconstruction: MGCG from t~, and K becomes the new K0.
        hier = mg.Hierarchy(self.prob, k, omega=self.params.omega)
        x, _, _ = pcg(K, qf, t, tol, self.params.cg_max, hier.precond, stats)
        self.k0, self.h0, self.K0 = k, hier, K
        stats.path = PATH_FALLBACK
        return self.fep.to_full(x), stats
