"""Oracle geometric multigrid: level hierarchy and the V-cycle.

Test infrastructure only (see the package docstring).

Follows Sec. 2.2, items (i)-(iii), and Table 1 (the V-cycle). The paper
leaves several choices open; the readings used here:

* Levels: ``levels`` grids including the finest; every axis of level l has
  n / 2^l elements of edge 2^l (the paper requires the element count per axis
  to be a multiple of 2^(nl-1)).
* Coarse operator: rediscretisation. A coarse element's conductivity is the
  arithmetic mean of its 2^d children; K_l is assembled from the element
  matrix of the coarse cell size.
* Coarse Dirichlet set: a coarse node is fixed iff the finest-grid node at
  the same position is fixed.
* Interpolation P: bi-/trilinear from level l+1 to level l, with rows of
  fixed fine nodes and columns of fixed coarse nodes removed; restriction is
  P^T exactly (Table 1, step 2).
* Smoother: damped Jacobi x += omega D^-1 (b - A x) (item (ii)), one pre- and
  one post-sweep, omega = 0.8 by default.
* Coarsest level: exact dense Cholesky solve (item (iii)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fe


def coarsen_conductivity(k: np.ndarray, dim: int, nx: int, ny: int, nz: int) -> np.ndarray:
    """Mean of the 2^d child element conductivities of every coarse element."""
    if dim == 2:
        a = k.reshape(ny // 2, 2, nx // 2, 2)
        return a.mean(axis=(1, 3)).ravel()
    a = k.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2)
    return a.mean(axis=(1, 3, 5)).ravel()


def interp_1d(n_fine_elems: int) -> sp.csr_matrix:
    """Linear interpolation from n/2 + 1 coarse nodes to n + 1 fine nodes on a line."""
    nf, nc = n_fine_elems + 1, n_fine_elems // 2 + 1
    rows, cols, vals = [], [], []
    for i in range(nf):
        if i % 2 == 0:
            rows.append(i); cols.append(i // 2); vals.append(1.0)
        else:
            rows += [i, i]; cols += [(i - 1) // 2, (i + 1) // 2]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def interpolation(dim: int, nx: int, ny: int, nz: int) -> sp.csr_matrix:
    """Full bi-/trilinear interpolation matrix (fine nodes x coarse nodes) for a
    fine grid of nx x ny (x nz) elements, in the x-fastest node numbering."""
    px, py = interp_1d(nx), interp_1d(ny)
    p = sp.kron(py, px)
    if dim == 3:
        p = sp.kron(interp_1d(nz), p)
    return p.tocsr()


class Level:
    def __init__(self, grid: fe.Grid, k: np.ndarray, fixed: np.ndarray):
        self.grid, self.k, self.fixed = grid, k, fixed
        self.free = np.flatnonzero(~fixed)
        Kfull = fe.assemble(grid, k)
        self.K = Kfull[self.free][:, self.free].tocsr()
        self.D = self.K.diagonal().copy()


class Hierarchy:
    """MG hierarchy for the conductivity field ``kelem`` on the finest grid."""

    def __init__(self, prob, kelem: np.ndarray, levels: int = None, omega: float = 0.8):
        self.dim = prob.dim
        self.L = prob.levels if levels is None else levels
        self.omega = omega
        d = prob.dim
        nx, ny, nz = prob.nelx, prob.nely, (prob.nelz if d == 3 else 0)
        for n in ((nx, ny, nz) if d == 3 else (nx, ny)):
            if n % (2 ** (self.L - 1)) != 0:
                raise ValueError("elements per axis must be a multiple of 2^(levels-1)")
        fine_grid = fe.Grid(d, nx, ny, nz)
        fine_fixed = fe.fixed_mask_from_box(fine_grid, prob.fix_lo, prob.fix_hi)
        fine_coords = fine_grid.node_coords()
        self.levels = []
        k = np.asarray(kelem, dtype=np.float64)
        for l in range(self.L):
            s = 2 ** l
            g = fe.Grid(d, nx // s, ny // s, (nz // s) if d == 3 else 0, h=float(s))
            if l == 0:
                fixed = fine_fixed
            else:
                # coarse node (I, J, K) coincides with finest node (I s, J s, K s)
                c = g.node_coords() * s
                fixed = fine_fixed[fine_grid.node_id(c[:, 0], c[:, 1], c[:, 2])]
            self.levels.append(Level(g, k, fixed))
            if l + 1 < self.L:
                k = coarsen_conductivity(k, d, g.nx, g.ny, g.nz)
        del fine_coords
        self.P = []
        for l in range(self.L - 1):
            g = self.levels[l].grid
            Pfull = interpolation(d, g.nx, g.ny, g.nz)
            fr, cr = self.levels[l].free, self.levels[l + 1].free
            self.P.append(Pfull[fr][:, cr].tocsr())
        Kc = self.levels[-1].K.toarray()
        if Kc.shape[0] == 0:
            raise ValueError("coarsest grid has no free node")
        if not np.any(self.levels[-1].fixed):
            raise ValueError("coarsest grid has no Dirichlet node (singular)")
        self.chol = sla.cho_factor(Kc, lower=True)

    def smooth(self, l, b, x):
        """One damped-Jacobi sweep on level l."""
        lv = self.levels[l]
        return x + self.omega * (b - lv.K @ x) / lv.D

    def vcycle(self, l, b, x):
        """Recursive V-cycle of Table 1 on level l: pre-smooth, restrict the
        residual with P^T, correct with the coarse solution, post-smooth. The
        coarsest level returns its exact solve."""
        if l == self.L - 1:
            return sla.cho_solve(self.chol, b)
        lv = self.levels[l]
        x = self.smooth(l, b, x)
        rc = self.P[l].T @ (b - lv.K @ x)
        ec = self.vcycle(l + 1, rc, np.zeros(self.levels[l + 1].free.size))
        x = x + self.P[l] @ ec
        x = self.smooth(l, b, x)
        return x

    def precond(self, r):
        """One V-cycle from a zero guess on the finest level: M^-1 r."""
        return self.vcycle(0, r, np.zeros_like(r))
