"""Oracle boundary-smoothing post-process (Sec. 2.3, Eq 24-27, Fig. 3).

Test infrastructure only (see the package docstring).

Runs once on the final design of the optimisation loop:

1. Element sensitivities s_e are projected onto the nodes in the manner of
   the density filter: ns_i = sum_e w_ie s_e / sum_e w_ie with the cone weight
   w_ie = max(0, r - |x_i - c_e|) between node i and element centroid c_e.
   Readings (the paper names neither): s_e = -df/drho_e, the filtered
   compliance sensitivity of Eq 9-11 with its sign turned so that large values
   mark material; r is a parameter (the loop's final filter radius by default).
2. Eq 24: an element is solid (1) when every one of its nodes has
   ns > ns_level, void (0) when every one has ns < ns_level, and otherwise
   gets the intermediate density ev.
3. Eq 25-27: for such an element the Q1 interpolation N_i of the nodal values
   (Eq 26, N_i(o) = prod_a (1 + xi_o,a xi_i,a) / 2 in local coordinates
   [-1, 1]^d) is evaluated at the points of a uniform lattice of n_s + 1
   points per axis over the element (its corners, the original nodes,
   included; n_s = 4 by default: the number of new points is in a figure the
   text does not reproduce, so the lattice is a reading), and ev is the
   fraction of lattice points whose value exceeds ns_level.
4. ns_level keeps the volume fraction: the post-processed volume sum_e rho_e
   is non-increasing in ns_level (a step function), so ns_level is found by
   bisection on [min ns - 1, max ns], 100 halvings or until the bracket is
   below 1e-14 of its initial width, keeping volume >= target at the lower
   end; the lower end is returned (the volume closest to the target from
   above that the bisection resolves). Every rho_e is a count of lattice
   points over their number P (a solid element counts P), so the volume is
   compared as the integer sum of the counts against target * P: the decision
   does not depend on the order in which fractions are added.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import fe


def node_projection_matrix(grid: fe.Grid, r: float):
    """Sparse (N x E) cone weights w_ie = max(0, r - |x_i - c_e|) and their row
    sums, over every element within r of node i (truncated at the boundary)."""
    d = grid.dim
    nc = grid.node_coords().astype(np.float64)[:, :d]
    R = int(np.ceil(r)) + 1
    dims = [grid.nx, grid.ny] + ([grid.nz] if d == 3 else [])
    rows, cols, vals = [], [], []
    base = grid.node_coords()[:, :d]
    for off in itertools.product(range(-R, R), repeat=d):
        ec = base + np.asarray(off)
        ok = np.ones(grid.nnodes, dtype=bool)
        for a in range(d):
            ok &= (ec[:, a] >= 0) & (ec[:, a] < dims[a])
        dist = np.sqrt(((ec + 0.5 - nc) ** 2).sum(axis=1))
        w = np.maximum(0.0, r - dist)
        ok &= w > 0.0
        i = np.flatnonzero(ok)
        e = grid.elem_id(ec[ok, 0], ec[ok, 1], ec[ok, 2] if d == 3 else 0)
        rows.append(i)
        cols.append(e)
        vals.append(w[ok])
    Wm = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(grid.nnodes, grid.nelem))
    return Wm, np.asarray(Wm.sum(axis=1)).ravel()


def project_to_nodes(grid: fe.Grid, s: np.ndarray, r: float) -> np.ndarray:
    """Step 1: nodal values ns_i = sum_e w_ie s_e / sum_e w_ie."""
    Wm, ws = node_projection_matrix(grid, r)
    return (Wm @ s) / ws


def lattice(dim: int, ns: int) -> np.ndarray:
    """Local coordinates in [-1, 1]^d of the (ns + 1)^d lattice points of one
    element, x fastest."""
    t = np.linspace(-1.0, 1.0, ns + 1)
    pts = np.array(list(itertools.product(t, repeat=dim)))[:, ::-1]
    return pts


def q1_weights(dim: int, pts: np.ndarray) -> np.ndarray:
    """Eq 26: N_c(o) = prod_a (1 + xi_o,a xi_c,a) / 2 for every lattice point o
    (rows) and local corner c = bx + 2 by + 4 bz (columns), xi_c,a = +-1."""
    out = np.ones((pts.shape[0], 2 ** dim))
    for c in range(2 ** dim):
        for a in range(dim):
            xc = 1.0 if (c >> a) & 1 else -1.0
            out[:, c] *= (1.0 + pts[:, a] * xc) / 2.0
    return out


def smoothed_counts(grid: fe.Grid, ns: np.ndarray, level: float, nsub: int = 4) -> np.ndarray:
    """Eq 24-27 for one level as integer counts out of P = (nsub + 1)^d
    lattice points per element: P (solid), 0 (void) or the number of lattice
    points above the level."""
    conn = grid.connectivity()
    nv = ns[conn]                                    # (E, 2^d) corner values
    P = (nsub + 1) ** grid.dim
    cnt = np.zeros(grid.nelem, dtype=np.int64)
    above = (nv > level).all(axis=1)
    below = (nv < level).all(axis=1)
    cnt[above] = P
    mixed = ~(above | below)
    if mixed.any():
        Nw = q1_weights(grid.dim, lattice(grid.dim, nsub))   # (P, 2^d)
        vals = nv[mixed] @ Nw.T                              # Eq 25 at every lattice point
        cnt[mixed] = (vals > level).sum(axis=1)
    return cnt


def smoothed_density(grid: fe.Grid, ns: np.ndarray, level: float, nsub: int = 4) -> np.ndarray:
    """Eq 24-27 for one level: 1, 0 or the lattice fraction ev per element."""
    return smoothed_counts(grid, ns, level, nsub) / float((nsub + 1) ** grid.dim)


def bisect_level(grid: fe.Grid, ns: np.ndarray, target: float, nsub: int = 4, steps: int = 100):
    """ns_level with sum_e rho_e(ns_level) as close to `target` from above as
    the bisection resolves: lo keeps volume >= target, hi volume < target
    (compared in lattice-point counts against target * P). Returns (level,
    rho, volume, steps taken); the level returned is lo."""
    P = (nsub + 1) ** grid.dim
    goal = target * P
    lo, hi = float(ns.min()) - 1.0, float(ns.max())
    rng = hi - lo
    taken = 0
    for _ in range(steps):
        if hi - lo <= 1e-14 * rng:
            break
        mid = 0.5 * (lo + hi)
        if float(smoothed_counts(grid, ns, mid, nsub).sum()) >= goal:
            lo = mid
        else:
            hi = mid
        taken += 1
    cnt = smoothed_counts(grid, ns, lo, nsub)
    return lo, cnt / float(P), float(cnt.sum()) / P, taken


def smooth_boundary(grid: fe.Grid, dc: np.ndarray, volfrac: float, r: float, nsub: int = 4):
    """The whole post-process from the filtered compliance sensitivities dc of
    the final design: project s = -dc onto the nodes, find the level that
    keeps volfrac * E, return (rho, ns, level, volume)."""
    ns = project_to_nodes(grid, -np.asarray(dc), r)
    level, rho, vol, _ = bisect_level(grid, ns, volfrac * grid.nelem, nsub)
    return rho, ns, level, vol


def postprocess(prob, x, r_filter, qelem=None, r_proj=None, nsub=4):
    """After the loop (Fig. 5): filter the final design with radius r_filter,
    solve, take its sensitivities, smooth (projection radius r_proj, default
    r_filter), and solve again on the smoothed densities. Returns (rho, level,
    volume, compliance before, compliance after)."""
    from . import solvers, topopt
    s = solvers.MgarSolver(prob, solvers.MgarParams(), qelem)
    filt = topopt.Filter(s.fep.grid, r_filter)
    xphys = filt.forward(x)
    t, _ = s.mgcg(xphys, np.zeros(s.fep.grid.nnodes), prob.tol)
    f0, dc, _, _ = topopt.sensitivity(s.fep, filt, xphys, t)
    rho, _, level, vol = smooth_boundary(s.fep.grid, dc, prob.volfrac, r_filter if r_proj is None else r_proj,
                                         nsub)
    t1, _ = s.mgcg(rho, t, prob.tol)
    return rho, level, vol, f0, float(s.fep.q @ t1)
