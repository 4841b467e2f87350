"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes* problems and draws random numbers: grid sizes,
the Dirichlet (T = 0) node box, the per-element heat source, initial and
reseeded densities, and random vectors for operator tests. It contains none
of the method's arithmetic (no element matrices, no assembly, no solver, no
filter), so that the CPU oracle and the GPU library can both consume it
without sharing any computation.

Problem setup follows the paper's benchmark structure (Sec. 3.2 and 4.3:
unit-cell structured grid, SIMP with p = 3, k0 = 1, kmin = 1e-3, uniform
internal heat source, a small Dirichlet sink on one side, cone density
filter), at the sizes of the synthetic workloads below.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

SEED_BASE = 221000947


@dataclasses.dataclass(frozen=True)
class Problem:
    """One heat-conduction topology-optimisation problem on a structured grid.

    ``fix_lo`` / ``fix_hi`` give an inclusive box of *node* indices (i, j, k)
    on the finest grid whose temperature is held at 0. In 2D the third
    entry is 0.
    """

    name: str
    dim: int
    nelx: int
    nely: int
    nelz: int
    levels: int
    fix_lo: Tuple[int, int, int]
    fix_hi: Tuple[int, int, int]
    source: float = 0.01          # heat source per unit volume, per element
    volfrac: float = 0.4
    filter_r: float = 1.5
    move: float = 0.2
    maxit: int = 50
    tol: float = 1e-8
    x_init: float = 0.4
    penal: float = 3.0
    k0: float = 1.0
    kmin: float = 1e-3

    @property
    def nelem(self) -> int:
        return self.nelx * self.nely * (self.nelz if self.dim == 3 else 1)

    @property
    def nnodes(self) -> int:
        n = (self.nelx + 1) * (self.nely + 1)
        return n * (self.nelz + 1) if self.dim == 3 else n

    @property
    def shape_nodes(self) -> Tuple[int, ...]:
        """Node array shape in C order (slowest axis first): (z, y, x)."""
        if self.dim == 3:
            return (self.nelz + 1, self.nely + 1, self.nelx + 1)
        return (self.nely + 1, self.nelx + 1)

    @property
    def shape_elems(self) -> Tuple[int, ...]:
        if self.dim == 3:
            return (self.nelz, self.nely, self.nelx)
        return (self.nely, self.nelx)


def sink_box_2d(nelx: int, nely: int, frac: float = 0.1,
                centre: Optional[int] = None) -> Tuple[Tuple[int, int, int], Tuple[int, int, int]]:
    """Nodes (0, j) on the left edge within a centred band of ``frac`` of the height.

    Node j is fixed when |j - c| <= frac/2 * nely (c = nely/2 unless given).
    For 40 elements this is j = 18..22; for 320 it is j = 144..176.
    """
    c = nely / 2.0 if centre is None else float(centre)
    half = 0.5 * frac * nely + 1e-9
    lo = int(math.ceil(c - half))
    hi = int(math.floor(c + half))
    lo, hi = max(lo, 0), min(hi, nely)
    return (0, lo, 0), (0, hi, 0)


def sink_box_3d(nelx: int, nely: int, nelz: int, frac: float = 0.2,
                centre: Optional[Tuple[int, int]] = None):
    """Nodes (i, j, 0) on the z = 0 face inside a centred frac x frac square."""
    cx = nelx / 2.0 if centre is None else float(centre[0])
    cy = nely / 2.0 if centre is None else float(centre[1])
    hx = 0.5 * frac * nelx + 1e-9
    hy = 0.5 * frac * nely + 1e-9
    ilo, ihi = max(int(math.ceil(cx - hx)), 0), min(int(math.floor(cx + hx)), nelx)
    jlo, jhi = max(int(math.ceil(cy - hy)), 0), min(int(math.floor(cy + hy)), nely)
    return (ilo, jlo, 0), (ihi, jhi, 0)


def make_2d(name, n, levels, **kw) -> Problem:
    lo, hi = sink_box_2d(n, n)
    return Problem(name=name, dim=2, nelx=n, nely=n, nelz=0, levels=levels,
                   fix_lo=lo, fix_hi=hi, **kw)


def make_3d(name, n, levels, **kw) -> Problem:
    lo, hi = sink_box_3d(n, n, n)
    return Problem(name=name, dim=3, nelx=n, nely=n, nelz=n, levels=levels,
                   fix_lo=lo, fix_hi=hi, **kw)


# The synthetic workloads. Sizes, sources, sinks and optimiser settings.
C0 = make_2d("2d-40x40-fp64", 40, 3, volfrac=0.4, filter_r=1.5, maxit=50, x_init=0.4)
C1 = make_2d("2d-320x320-fp64", 320, 6, volfrac=0.4, filter_r=3.0, maxit=100, x_init=0.4)
C2 = make_3d("3d-64^3", 64, 5, volfrac=0.3, filter_r=2.0, maxit=50, x_init=0.3)
C3 = make_3d("3d-128^3", 128, 6, volfrac=0.3, filter_r=2.0, maxit=80, x_init=0.3)

CONFIGS = {"c0": C0, "c1": C1, "c2": C2, "c3": C3}


def tiny_2d(nx: int, ny: int, levels: int, **kw) -> Problem:
    lo, hi = sink_box_2d(nx, ny)
    return Problem(name=f"2d-{nx}x{ny}", dim=2, nelx=nx, nely=ny, nelz=0,
                   levels=levels, fix_lo=lo, fix_hi=hi, **kw)


def tiny_3d(nx: int, ny: int, nz: int, levels: int, **kw) -> Problem:
    lo, hi = sink_box_3d(nx, ny, nz)
    return Problem(name=f"3d-{nx}x{ny}x{nz}", dim=3, nelx=nx, nely=ny, nelz=nz,
                   levels=levels, fix_lo=lo, fix_hi=hi, volfrac=0.3, x_init=0.3,
                   filter_r=2.0, **kw)


def element_source(p: Problem) -> np.ndarray:
    """Per-element heat source per unit volume (uniform)."""
    return np.full(p.nelem, p.source, dtype=np.float64)


# Non-uniform source of the paper's Sec. 4.2 / Table 3 model: four sub-domains
# of the same shape with sources per unit volume Omega_1..Omega_4.
QUADRANT_SOURCES = (5e-5, 1e-4, 1.5e-4, 3e-4)


def quadrant_source(p: Problem, values=QUADRANT_SOURCES) -> np.ndarray:
    """Per-element source per unit volume on four equal quadrants cut at the
    mid-lines of x and y (through every z in 3D): Omega_1 = lower-left (x <
    nelx/2, y < nely/2), Omega_2 = lower-right, Omega_3 = upper-left, Omega_4
    = upper-right, by element centroid. The paper places the sub-domains in a
    figure that the text does not reproduce, so this placement is a reading."""
    nz = p.nelz if p.dim == 3 else 1
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(p.nely), np.arange(p.nelx), indexing="ij")
    right = (2 * ex + 1) > p.nelx
    upper = (2 * ey + 1) > p.nely
    v = np.asarray(values, dtype=np.float64)
    return v[right.astype(int) + 2 * upper.astype(int)].ravel()


def paper_2d(n: int, levels: int, volfrac: float = 0.5, maxit: int = 300, **kw) -> Problem:
    """The paper's 2D model (Sec. 3.2, 4.1): an n x n domain, sink on the middle
    tenth of the left side, source 1e-4 per unit volume, MGCG accuracy
    eps2 = 1e-6, 300 design cycles, minimum filter radius 3 (continuous
    filtering, Eq 22-23, is applied by the loop)."""
    lo, hi = sink_box_2d(n, n)
    kw.setdefault("source", 1e-4)
    kw.setdefault("tol", 1e-6)
    kw.setdefault("filter_r", 3.0)
    return Problem(name=f"paper-2d-{n}x{n}-vf{volfrac}", dim=2, nelx=n, nely=n, nelz=0, levels=levels,
                   fix_lo=lo, fix_hi=hi, volfrac=volfrac, x_init=volfrac, maxit=maxit, **kw)


def initial_density(p: Problem) -> np.ndarray:
    return np.full(p.nelem, p.x_init, dtype=np.float64)


def reseeded_density(p: Problem, r: int, lo: float = 0.3, hi: float = 0.5) -> np.ndarray:
    """Solver-only densities: i.i.d. uniform(lo, hi) per element, run r."""
    rng = np.random.default_rng(SEED_BASE + r)
    return rng.uniform(lo, hi, p.nelem)


def perturbed_density(x: np.ndarray, seed: int, amp: float = 0.02) -> np.ndarray:
    """clip(x + U(-amp, amp), 0, 1): a nearby design for reanalysis timing."""
    rng = np.random.default_rng(SEED_BASE + 7919 + seed)
    return np.clip(x + rng.uniform(-amp, amp, x.shape[0]), 0.0, 1.0)


def random_density(n: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(SEED_BASE + 104729 + seed)
    return rng.uniform(lo, hi, n)


def random_vector(n: int, seed: int) -> np.ndarray:
    """Standard normal vector for operator tests."""
    rng = np.random.default_rng(SEED_BASE + 1299709 + seed)
    return rng.standard_normal(n)


# ---------------------------------------------------------------------------
# Batched workload: many independent designs of uneven sizes.
# ---------------------------------------------------------------------------

def _levels_for(dims: List[int], max_coarse: int = 12) -> int:
    """Largest L such that every axis is divisible by 2^(L-1) with >= 2
    elements left, and the coarsest grid has at most ``max_coarse`` elements
    per axis (raising L until that holds)."""
    L = 1
    while all(d % (2 ** L) == 0 and d // (2 ** L) >= 2 for d in dims):
        L += 1
    return L


def batched_designs(seed: int = 0, n2d: int = 48, n3d: int = 8) -> List[Problem]:
    """48 2D designs with (nelx, nely) in {64,96,128,192,256}^2 and 8 3D designs
    with per-axis size in {32,40,48}; volume fraction in [0.25, 0.5]; sink
    centred on a node of the coarsest grid so every level keeps a fixed node."""
    rng = np.random.default_rng(SEED_BASE + seed)
    sizes2 = [64, 96, 128, 192, 256]
    sizes3 = [32, 40, 48]
    out: List[Problem] = []
    for d in range(n2d):
        nx, ny = (int(v) for v in rng.choice(sizes2, 2))
        L = _levels_for([nx, ny])
        step = 2 ** (L - 1)
        ncy = ny // step
        cy = int(rng.integers(1, ncy)) * step
        lo, hi = sink_box_2d(nx, ny, centre=cy)
        vf = float(rng.uniform(0.25, 0.5))
        out.append(Problem(name=f"b2d-{d}-{nx}x{ny}", dim=2, nelx=nx, nely=ny, nelz=0,
                           levels=L, fix_lo=lo, fix_hi=hi, volfrac=vf, filter_r=1.5,
                           x_init=vf, maxit=50))
    for d in range(n3d):
        nx, ny, nz = (int(v) for v in rng.choice(sizes3, 3))
        L = _levels_for([nx, ny, nz])
        step = 2 ** (L - 1)
        cx = int(rng.integers(1, nx // step)) * step
        cy = int(rng.integers(1, ny // step)) * step
        lo, hi = sink_box_3d(nx, ny, nz, centre=(cx, cy))
        vf = float(rng.uniform(0.25, 0.5))
        out.append(Problem(name=f"b3d-{d}-{nx}x{ny}x{nz}", dim=3, nelx=nx, nely=ny, nelz=nz,
                           levels=L, fix_lo=lo, fix_hi=hi, volfrac=vf, filter_r=1.5,
                           x_init=vf, maxit=50))
    return out


def unet_init(C, seed: int = 0) -> np.ndarray:
    """Initial parameters of the element-grid seed U-Net with channels C per
    level (FP32): He-uniform weights per layer (bound sqrt(6 / (k^3 ci))), zero
    biases, in the library's flat layout: per layer [co][ci][k][k][k] weights
    then co biases, layers in the order encoder (level 0 .. L-1, two 3x3x3
    convolutions each; 3 input channels), decoder (level L-2 .. 0, two each;
    the first takes the upsampled C[l+1] channels followed by the C[l] skip
    channels), 1x1x1 head to one channel."""
    L = len(C)
    shapes = []
    for l in range(L):
        shapes += [(C[l], 3 if l == 0 else C[l - 1], 3), (C[l], C[l], 3)]
    for l in range(L - 2, -1, -1):
        shapes += [(C[l], C[l + 1] + C[l], 3), (C[l], C[l], 3)]
    shapes.append((1, C[0], 1))
    rng = np.random.default_rng(SEED_BASE + 9000 + seed)
    parts = []
    for co, ci, k in shapes:
        bound = np.sqrt(6.0 / (k ** 3 * ci))
        parts.append(rng.uniform(-bound, bound, co * ci * k ** 3))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
