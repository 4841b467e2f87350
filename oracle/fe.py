"""Oracle FE layer: structured grid, element matrix, load vector, SIMP, assembly.

Test infrastructure only (see the package docstring).

Discretisation of steady isotropic conduction (Eq 2) into K t = q (Eq 3) with
bilinear quadrilateral (2D) or trilinear hexahedral (3D) elements on a
structured grid of cubic cells of edge h. The paper states no element type;
the reading used here is the standard Q1 element.

Numbering (not stated in the paper; the reading used throughout):
  node (i, j, k)      -> i + (nx+1) * (j + (ny+1) * k)
  element (ex, ey, ez) -> ex + nx * (ey + ny * ez)
  local corner c = bx + 2*by + 4*bz -> node (ex+bx, ey+by, ez+bz)
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


class Grid:
    """Structured grid of nx x ny (x nz) square/cubic cells of edge h."""

    def __init__(self, dim: int, nx: int, ny: int, nz: int = 0, h: float = 1.0):
        assert dim in (2, 3)
        self.dim, self.nx, self.ny, self.nz, self.h = dim, nx, ny, (nz if dim == 3 else 0), h
        self.nnx, self.nny = nx + 1, ny + 1
        self.nnz = (nz + 1) if dim == 3 else 1
        self.nnodes = self.nnx * self.nny * self.nnz
        self.nelem = nx * ny * (nz if dim == 3 else 1)
        self.ncorner = 2 ** dim

    def node_id(self, i, j, k=0):
        return i + self.nnx * (j + self.nny * k)

    def elem_id(self, ex, ey, ez=0):
        return ex + self.nx * (ey + self.ny * ez)

    def node_coords(self):
        """(N, 3) integer node coordinates (i, j, k)."""
        k, j, i = np.meshgrid(np.arange(self.nnz), np.arange(self.nny), np.arange(self.nnx),
                              indexing="ij")
        return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)

    def elem_coords(self):
        nzz = self.nz if self.dim == 3 else 1
        ez, ey, ex = np.meshgrid(np.arange(nzz), np.arange(self.ny), np.arange(self.nx),
                                 indexing="ij")
        return np.stack([ex.ravel(), ey.ravel(), ez.ravel()], axis=1)

    def connectivity(self):
        """(E, 2^d) node ids of each element's corners in local order c."""
        ec = self.elem_coords()
        conn = np.empty((self.nelem, self.ncorner), dtype=np.int64)
        for c in range(self.ncorner):
            bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            conn[:, c] = self.node_id(ec[:, 0] + bx, ec[:, 1] + by, ec[:, 2] + bz)
        return conn


def _corner_signs(dim):
    """Reference-coordinate sign of each local corner: -1 for b = 0, +1 for b = 1."""
    s = np.zeros((2 ** dim, dim))
    for c in range(2 ** dim):
        for a in range(dim):
            s[c, a] = 1.0 if (c >> a) & 1 else -1.0
    return s


def _gauss2():
    g = 1.0 / np.sqrt(3.0)
    return np.array([-g, g]), np.array([1.0, 1.0])


def shape_functions(dim, xi):
    """Q1 shape functions N_c(xi) = prod_a (1 + s_ca xi_a) / 2 and their
    reference gradients at one point xi in [-1, 1]^d."""
    s = _corner_signs(dim)
    n = np.ones(2 ** dim)
    dn = np.ones((2 ** dim, dim))
    for a in range(dim):
        fa = 0.5 * (1.0 + s[:, a] * xi[a])
        n *= fa
        for b in range(dim):
            dn[:, b] *= (0.5 * s[:, a]) if a == b else fa
    return n, dn


def element_matrix(dim: int, h: float = 1.0) -> np.ndarray:
    """Element conductivity matrix KE = int grad N . grad N^T over one cell of
    edge h (unit conductivity), by 2-point Gauss quadrature, which is exact
    for the Q1 element. This is the element-level form of Eq 2-3."""
    pts, wts = _gauss2()
    ke = np.zeros((2 ** dim, 2 ** dim))
    jac = h / 2.0                       # d x / d xi along every axis
    for idx in itertools.product(range(2), repeat=dim):
        xi = np.array([pts[i] for i in idx])
        w = np.prod([wts[i] for i in idx])
        _, dn = shape_functions(dim, xi)
        gx = dn / jac                   # physical gradients
        ke += w * (gx @ gx.T) * jac ** dim
    return ke


def element_load(dim: int, h: float = 1.0) -> np.ndarray:
    """Consistent nodal load of a unit source per unit volume over one cell:
    int N_c dV, by Gauss quadrature."""
    pts, wts = _gauss2()
    fe = np.zeros(2 ** dim)
    jac = h / 2.0
    for idx in itertools.product(range(2), repeat=dim):
        xi = np.array([pts[i] for i in idx])
        w = np.prod([wts[i] for i in idx])
        n, _ = shape_functions(dim, xi)
        fe += w * n * jac ** dim
    return fe


def simp(xphys, k0=1.0, kmin=1e-3, penal=3.0):
    """Modified SIMP conductivity, Eq 4: k = kmin + (k0 - kmin) * rho~^p."""
    return kmin + (k0 - kmin) * np.asarray(xphys, dtype=np.float64) ** penal


def fixed_mask_from_box(grid: Grid, lo, hi) -> np.ndarray:
    """Boolean N-mask of the Dirichlet nodes: the inclusive node box [lo, hi]."""
    nc = grid.node_coords()
    m = np.ones(grid.nnodes, dtype=bool)
    for a in range(grid.dim):
        m &= (nc[:, a] >= lo[a]) & (nc[:, a] <= hi[a])
    return m


def assemble(grid: Grid, kelem: np.ndarray) -> sp.csr_matrix:
    """Global conductivity matrix K = sum_e k_e A_e^T KE A_e over all nodes (Eq 3)."""
    ke = element_matrix(grid.dim, grid.h)
    conn = grid.connectivity()
    nc = grid.ncorner
    rows = np.repeat(conn, nc, axis=1).ravel()
    cols = np.tile(conn, (1, nc)).ravel()
    vals = (kelem[:, None] * ke.ravel()[None, :]).ravel()
    return sp.coo_matrix((vals, (rows, cols)), shape=(grid.nnodes, grid.nnodes)).tocsr()


def load_vector(grid: Grid, qelem: np.ndarray, fixed: np.ndarray) -> np.ndarray:
    """Nodal heat load q_i = sum_{e contains i} Q_e int N_i dV; zero on Dirichlet nodes.
    The load does not depend on the density (a fixed internal source)."""
    fe = element_load(grid.dim, grid.h)
    conn = grid.connectivity()
    q = np.zeros(grid.nnodes)
    np.add.at(q, conn.ravel(), (qelem[:, None] * fe[None, :]).ravel())
    q[fixed] = 0.0
    return q


class FEProblem:
    """Finest-level FE system for one problem: grid, Dirichlet set, load."""

    def __init__(self, prob, qelem=None):
        self.prob = prob
        self.grid = Grid(prob.dim, prob.nelx, prob.nely, prob.nelz)
        self.fixed = fixed_mask_from_box(self.grid, prob.fix_lo, prob.fix_hi)
        self.free = np.flatnonzero(~self.fixed)
        if qelem is None:
            qelem = np.full(self.grid.nelem, prob.source)
        self.q = load_vector(self.grid, qelem, self.fixed)

    def kelem(self, xphys):
        p = self.prob
        return simp(xphys, p.k0, p.kmin, p.penal)

    def K_free(self, xphys):
        """Free-free block of K (Dirichlet DOFs eliminated)."""
        K = assemble(self.grid, self.kelem(xphys))
        return K[self.free][:, self.free].tocsr()

    def to_free(self, v):
        return np.asarray(v)[self.free]

    def to_full(self, vf):
        out = np.zeros(self.grid.nnodes)
        out[self.free] = vf
        return out


def apply_rows(grid: Grid, kelem: np.ndarray, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(K x)_i for the selected node ids only, straight from the element sum of
    Eq 3: y_i = sum_{e contains i} k_e sum_c KE[c_i, c] x_{node(e, c)}. For
    spot checks on grids too large to assemble."""
    ke = element_matrix(grid.dim, grid.h)
    nc = grid.node_coords()[rows]
    dims = [grid.nx, grid.ny] + ([grid.nz] if grid.dim == 3 else [])
    out = np.zeros(len(rows))
    for off in itertools.product((-1, 0), repeat=grid.dim):
        ec = [nc[:, a] + off[a] for a in range(grid.dim)]
        ok = np.ones(len(rows), dtype=bool)
        for a in range(grid.dim):
            ok &= (ec[a] >= 0) & (ec[a] < dims[a])
        e = grid.elem_id(ec[0], ec[1], ec[2] if grid.dim == 3 else 0)
        e = np.where(ok, e, 0)
        ci = sum(((-off[a]) << a) for a in range(grid.dim))   # corner of node i in cell e
        acc = np.zeros(len(rows))
        for c in range(grid.ncorner):
            bx, by, bz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            nid = grid.node_id(ec[0] + bx, ec[1] + by, (ec[2] + bz) if grid.dim == 3 else 0)
            nid = np.where(ok, nid, 0)
            acc += ke[ci, c] * x[nid]
        out += np.where(ok, kelem[e] * acc, 0.0)
    return out
