"""Oracle topology-optimisation layer: filter, sensitivities, OC update, loop.

Test infrastructure only (see the package docstring).

* Density filter, Eq 6-8: rho~_e = sum_j H_ej v_j rho_j / sum_j H_ej v_j with
  the cone weight H_ej = max(0, r - ||c_e - c_j||) between element centroids
  (the paper reuses the density symbol for positions; centroid distance is
  the reading). Unit cells, so v = 1. The neighbourhood is truncated at the
  domain boundary.
* Compliance, Eq 5: f = q^T t (equal to t^T K t for the exact solution).
* Element sensitivity, Eq 10: df/drho~_e = -p (k0 - kmin) rho~_e^(p-1) t_e^T KE t_e.
* Chain rule through the filter, Eq 9 and 11: df/drho_j = sum_e H_ej / Hs_e df/drho~_e.
* Design update: the paper names only "the classical SIMP framework"; the
  optimality-criteria update with move limit 0.2, exponent 1/2 and lambda
  found by bisection on the filtered volume is used.
* Loop (Fig. 5 flow, Sec. 3.1): filter -> solve (MGCG while the 1-based cycle
  index is below N_on = floor(2 maxit / 15), MGAR afterwards) -> sensitivity
  -> update; the previous cycle's temperature seeds the next solve.
* Continuous density filtering (Sec. 2.3, Eq 22-23): the radius shrinks
  geometrically from r0 = alpha L to r_min over lp cycles, r^(k) =
  max(r_min, eta r^(k-1)) with eta = exp((ln r_min - ln(alpha L)) / lp);
  alpha = 1.4/50 and lp = 5/6 of the maximum cycle count unless stated. L is
  the side length of the design domain in element edges (the largest axis).
  Reading: cycle k (1-based) filters with r^(k-1), so the first cycle uses the
  initial radius r0 and cycle lp + 1 the minimum one.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np
import scipy.sparse as sp

from . import fe
from .solvers import MgarParams, MgarSolver, SolveStats


def filter_matrix(grid: fe.Grid, r: float):
    """Sparse cone-filter matrix H (E x E) and row sums Hs (Eq 6-8).

    Only element pairs closer than r have a positive weight; they are
    enumerated over the integer offsets within a (2 ceil(r) + 1)^d window."""
    d = grid.dim
    R = int(math.ceil(r))
    ec = grid.elem_coords()
    dims = [grid.nx, grid.ny] + ([grid.nz] if d == 3 else [])
    rows, cols, vals = [], [], []
    for off in itertools.product(range(-R, R + 1), repeat=d):
        dist = math.sqrt(sum(o * o for o in off))
        w = max(0.0, r - dist)
        if w <= 0.0:
            continue
        ok = np.ones(grid.nelem, dtype=bool)
        nb = []
        for a in range(d):
            c = ec[:, a] + off[a]
            ok &= (c >= 0) & (c < dims[a])
            nb.append(c)
        e = np.flatnonzero(ok)
        j = grid.elem_id(nb[0][ok], nb[1][ok], nb[2][ok] if d == 3 else 0)
        rows.append(e); cols.append(j); vals.append(np.full(e.size, w))
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(grid.nelem, grid.nelem))
    Hs = np.asarray(H.sum(axis=1)).ravel()
    return H, Hs


def filter_brute(grid: fe.Grid, r: float, x: np.ndarray) -> np.ndarray:
    """O(E^2) statement of Eq 6-8 for tiny grids: every pair of centroids."""
    c = grid.elem_coords().astype(np.float64) + 0.5
    out = np.empty(grid.nelem)
    for e in range(grid.nelem):
        w = np.maximum(0.0, r - np.sqrt(((c - c[e]) ** 2).sum(axis=1)))
        out[e] = (w * x).sum() / w.sum()
    return out


class Filter:
    def __init__(self, grid: fe.Grid, r: float):
        self.H, self.Hs = filter_matrix(grid, r)

    def forward(self, x):
        """rho~ = H rho / Hs (Eq 6)."""
        return (self.H @ x) / self.Hs

    def adjoint(self, g):
        """d/drho of a function of rho~ given its gradient g wrt rho~ (Eq 9, 11):
        H^T (g / Hs)."""
        return self.H.T @ (g / self.Hs)


def element_energy(grid: fe.Grid, t_full: np.ndarray) -> np.ndarray:
    """t_e^T KE t_e per element (unit conductivity)."""
    ke = fe.element_matrix(grid.dim, grid.h)
    te = t_full[grid.connectivity()]
    return np.einsum("ei,ij,ej->e", te, ke, te)


def sensitivity(fep: fe.FEProblem, filt: Filter, xphys, t_full):
    """Compliance f = q^T t (Eq 5), filtered compliance sensitivity dc (Eq 9-11)
    and filtered volume sensitivity dv. Returns (f, dc, dv, dc_tilde)."""
    p = fep.prob
    f = float(fep.q @ t_full)
    dct = -p.penal * (p.k0 - p.kmin) * np.asarray(xphys) ** (p.penal - 1.0) \
        * element_energy(fep.grid, t_full)
    dc = filt.adjoint(dct)
    dv = filt.adjoint(np.ones_like(dct))
    return f, dc, dv, dct


def oc_update(x, dc, dv, filt: Filter, volfrac, move=0.2, tol=1e-10):
    """Optimality-criteria update with lambda by bisection on the filtered
    volume: sum(H x_new / Hs) compared with volfrac * E. Returns (x_new, lambda,
    bisection steps)."""
    l1, l2 = 0.0, 1e9
    n = x.size
    steps = 0
    B = np.maximum(0.0, -dc) / dv
    xnew = x
    while (l2 - l1) / (l1 + l2) > tol:
        lmid = 0.5 * (l2 + l1)
        xnew = np.maximum(0.0, np.maximum(x - move,
                          np.minimum(1.0, np.minimum(x + move, x * np.sqrt(B / lmid)))))
        if filt.forward(xnew).sum() > volfrac * n:
            l1 = lmid
        else:
            l2 = lmid
        steps += 1
    return xnew, 0.5 * (l1 + l2), steps


@dataclasses.dataclass
class CycleRecord:
    cycle: int
    compliance: float
    path: int
    cg_iters: int
    res_ca: float
    res_final: float
    volume: float
    change: float
    radius: float = 0.0


def n_on(maxit: int) -> int:
    """Activation parameter: 2/15 of the maximum number of cycles (Sec. 3.2)."""
    return (2 * maxit) // 15


def continuous_radii(r_min, r0, lp, count):
    """Eq 22-23: the radii r^(0) = r0, r^(1), ..., r^(count-1), each step
    r^(k) = max(r_min, eta r^(k-1)) with eta = exp((ln r_min - ln r0) / lp).
    The schedule shrinks the radius, so r0 >= r_min."""
    if not r0 >= r_min:
        raise ValueError("the initial radius must not be below r_min")
    eta = math.exp((math.log(r_min) - math.log(r0)) / lp)
    radii = [float(r0)]
    while len(radii) < count:
        radii.append(max(r_min, eta * radii[-1]))
    return radii


def loop_radii(prob, maxit, continuous):
    """Filter radius of each cycle 1..maxit: the fixed prob.filter_r, or with
    `continuous` = dict(r_min, alpha = 1.4/50, lp = 5/6 prob.maxit) the
    schedule of Eq 22-23 with r0 = alpha L (cycle k uses r^(k-1)). On a domain
    so small that alpha L < r_min the radius stays r_min."""
    if not continuous:
        return [prob.filter_r] * maxit
    L = max(prob.nelx, prob.nely, prob.nelz if prob.dim == 3 else 0)
    alpha = continuous.get("alpha", 1.4 / 50)
    lp = continuous.get("lp", 5.0 * prob.maxit / 6.0)
    r_min = continuous["r_min"]
    return continuous_radii(r_min, max(alpha * L, r_min), lp, maxit)


def run_loop(prob, maxit=None, use_mgar=True, params: MgarParams = None, qelem=None,
             x_init=None, on_cycle=None, continuous=None):
    """The optimisation loop. Returns (x, xphys, t, records). continuous: None
    (fixed radius prob.filter_r) or the Eq 22-23 schedule (see loop_radii)."""
    maxit = prob.maxit if maxit is None else maxit
    params = params or MgarParams(eps_accept=prob.tol)
    solver = MgarSolver(prob, params, qelem)
    fep = solver.fep
    radii = loop_radii(prob, maxit, continuous)
    filters = {}

    def filter_for(r):
        if r not in filters:
            filters.clear()
            filters[r] = Filter(fep.grid, r)
        return filters[r]

    filt = filter_for(radii[0])
    x = np.full(fep.grid.nelem, prob.x_init) if x_init is None else np.array(x_init, float)
    t_prev = np.zeros(fep.grid.nnodes)
    non = n_on(prob.maxit)
    recs = []
    xphys = filt.forward(x)
    t = t_prev
    for k in range(1, maxit + 1):
        filt = filter_for(radii[k - 1])
        xphys = filt.forward(x)
        st = SolveStats()
        if (not use_mgar) or k < non:
            t, st = solver.mgcg(xphys, t_prev, prob.tol, st)
        else:
            t, st = solver.mgar(xphys, t_prev, prob.tol, st)
        f, dc, dv, _ = sensitivity(fep, filt, xphys, t)
        xnew, _lam, _ = oc_update(x, dc, dv, filt, prob.volfrac, prob.move)
        change = float(np.abs(xnew - x).max())
        recs.append(CycleRecord(k, f, st.path, st.cg_iters, st.res_ca, st.res_final,
                                float(xphys.mean()), change, radii[k - 1]))
        if on_cycle is not None:
            on_cycle(k, xphys, t)
        x = xnew
        t_prev = t
    return x, xphys, t, recs
