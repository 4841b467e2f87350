// Matrix-free conductivity stencil, grid transfers and the coarsest-grid solve.
//
// Operator (Eq 3, rediscretised on every level): y_i = sum over the 2^d cells e
// touching node i of k_e (KE x_e)_i, where KE is the Q1 element conductivity
// matrix of a cell of edge h. Its entries depend only on the Hamming distance
// between two corners:
//   2D (any h):  2/3 (same corner), -1/6 (edge), -1/3 (diagonal)
//   3D (edge h): h/3, 0 (edge), -h/12 (face diagonal), -h/12 (body diagonal)
// so in 3D only 21 of the 27 neighbours carry a weight.
//
// Every N-vector the kernels read is exactly 0 on Dirichlet nodes, and every
// N-vector they write is set to 0 there; nodes outside the grid only occur in
// cells outside the grid, whose conductivity is taken as 0.
#include <algorithm>
#include <cfloat>
#include <limits>
#include <type_traits>

#include <hip/hip_ext.h>

#include "mgar_launch.h"
#include "zbuf.h"

namespace {

constexpr int TBX = 64, TBY = 4;

template <typename T>
struct CellP {
  const T* p;
  __device__ T operator()(long long e) const { return p[e]; }
};

// Node coordinates of flat index n (x fastest); threads of the buffer kernels
// are laid out flat over the nodes, so every lane of a wave has a node.
__device__ inline void node_ijk(const Geo& g, long long n, int& i, int& j, int& k) {
  const long long r = n / g.nnx;
  i = (int)(n - r * g.nnx);
  j = (int)(r % g.nny);
  k = (int)(r / g.nny);
}

// Byte offset of node (i, j, k) / cell (ex, ey, ez), or ZOOB outside the grid.
__device__ inline unsigned node_boff(const Geo& g, int i, int j, int k, unsigned esz) {
  const bool in = i >= 0 && i < g.nnx && j >= 0 && j < g.nny && k >= 0 && k < g.nnz;
  return in ? (unsigned)(i + g.nnx * (j + g.nny * k)) * esz : ZOOB;
}
__device__ inline unsigned cell_boff(const Geo& g, int ex, int ey, int ez, unsigned esz) {
  const bool in = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny && ez >= 0 && ez < g.nz;
  return in ? (unsigned)(ex + g.nx * (ey + g.ny * ez)) * esz : ZOOB;
}

template <int DIM, bool DK, typename T, typename CL>
__device__ inline void load_cells(const Geo& g, const CL& k, const CL& kref, int i, int j, int kz,
                                  T (&kv)[2][2][2]) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ex = i - 1 + a, ey = j - 1 + b, ez = (DIM == 3) ? kz - 1 + c : 0;
        const bool in = (DIM == 3 || c == 0) && ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny &&
                        ez >= 0 && ez < g.nz;
        // clamped address, masked by a multiply: no branch around the load, so
        // all loads of a node are issued before the first wait
        const long long e = geo_elem(g, min(max(ex, 0), g.nx - 1), min(max(ey, 0), g.ny - 1),
                                     min(max(ez, 0), g.nz - 1));
        T v = T(k(e));
        if (DK) v -= T(kref(e));
        kv[c][b][a] = v * (in ? T(1) : T(0));
      }
}

// x at node (i, j, k), 0 outside the grid (clamped load times a 0/1 mask).
template <typename T>
__device__ inline T ldx(const Geo& g, const T* __restrict__ x, int i, int j, int k) {
  const bool in = i >= 0 && i < g.nnx && j >= 0 && j < g.nny && k >= 0 && k < g.nnz;
  const T v = x[geo_node(g, min(max(i, 0), g.nnx - 1), min(max(j, 0), g.nny - 1), min(max(k, 0), g.nnz - 1))];
  return v * (in ? T(1) : T(0));
}

// (K x)_i in 3D from the 3x3 windows of node planes kz-1 (A), kz (B) and kz+1
// (C), centred on the node, and the 2x2 windows of cell conductivities below
// (CA) and above (CB) it ([y][x], index 0 = the lower neighbour). With the
// trilinear element matrix only the 8 cell centres (weight h/3 on the node)
// and the 12 edge- plus 8 corner-diagonal neighbours (weight -h/12) couple;
// face neighbours have weight 0. ks returns the sum of the 8 conductivities,
// so that the diagonal of K is hc * ks. Every 3D stencil kernel evaluates this
// one expression, so results do not depend on the kernel or launch shape.
template <typename T, bool NEEDX, typename FA, typename FB, typename FC, typename GA, typename GB>
__device__ inline T apply27g(FA A, FB B, FC C, GA CA, GB CB, T hc, T hf, T& ks) {
  const T t00 = CA(0, 0) + CB(0, 0), t01 = CA(0, 1) + CB(0, 1);
  const T t10 = CA(1, 0) + CB(1, 0), t11 = CA(1, 1) + CB(1, 1);
  ks = (t00 + t01) + (t10 + t11);
  if (!NEEDX) return T(0);
  T s1 = t00 * B(0, 0) + t01 * B(0, 2) + t10 * B(2, 0) + t11 * B(2, 2);
  s1 += (CA(0, 0) + CA(1, 0)) * A(1, 0) + (CA(0, 1) + CA(1, 1)) * A(1, 2);
  s1 += (CA(0, 0) + CA(0, 1)) * A(0, 1) + (CA(1, 0) + CA(1, 1)) * A(2, 1);
  s1 += CA(0, 0) * A(0, 0) + CA(0, 1) * A(0, 2) + CA(1, 0) * A(2, 0) + CA(1, 1) * A(2, 2);
  s1 += (CB(0, 0) + CB(1, 0)) * C(1, 0) + (CB(0, 1) + CB(1, 1)) * C(1, 2);
  s1 += (CB(0, 0) + CB(0, 1)) * C(0, 1) + (CB(1, 0) + CB(1, 1)) * C(2, 1);
  s1 += CB(0, 0) * C(0, 0) + CB(0, 1) * C(0, 2) + CB(1, 0) * C(2, 0) + CB(1, 1) * C(2, 2);
  return hc * ks * B(1, 1) - hf * s1;
}

template <typename T, bool NEEDX>
__device__ inline T apply27(const T (&A)[3][3], const T (&B)[3][3], const T (&C)[3][3],
                            const T (&CA)[2][2], const T (&CB)[2][2], T hc, T hf, T& ks) {
  return apply27g<T, NEEDX>([&](int y, int x) { return A[y][x]; }, [&](int y, int x) { return B[y][x]; },
                            [&](int y, int x) { return C[y][x]; }, [&](int y, int x) { return CA[y][x]; },
                            [&](int y, int x) { return CB[y][x]; }, hc, hf, ks);
}

// (K x)_i for node (i, j, kz) given the 2^d cell conductivities around it;
// ksum returns the conductivity sum that scales the diagonal.
template <int DIM, typename T>
__device__ inline T node_apply(const Geo& g, const T* __restrict__ x, int i, int j, int kz,
                               const T (&kv)[2][2][2], T& ksum) {
  if (DIM == 2) {
    T xv[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) xv[dy][dx] = ldx(g, x, i + dx - 1, j + dy - 1, 0);
    T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int sx = a ? 2 : 0, sy = b ? 2 : 0;
        const T ke = kv[0][b][a];
        s0 += ke;
        s1 += ke * (xv[1][sx] + xv[sy][1]);
        s2 += ke * xv[sy][sx];
      }
    ksum = s0;
    return T(2.0 / 3.0) * s0 * xv[1][1] - T(1.0 / 6.0) * s1 - T(1.0 / 3.0) * s2;
  } else {
    T xv[3][3][3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int nz = (dx != 1) + (dy != 1) + (dz != 1);
          xv[dz][dy][dx] = (nz == 1) ? T(0) : ldx(g, x, i + dx - 1, j + dy - 1, kz + dz - 1);
        }
    return apply27<T, true>(xv[0], xv[1], xv[2], kv[0], kv[1], T(g.h * (1.0 / 3.0)),
                            T(g.h * (1.0 / 12.0)), ksum);
  }
}

template <int DIM, int MODE, typename T, typename CL>
__global__ __launch_bounds__(TBX* TBY) void k_stencil(Geo g, const T* __restrict__ x, CL k, CL kref,
                                                      const T* __restrict__ b,
                                                      T* __restrict__ out, T omega,
                                                      double* __restrict__ part,
                                                      const int* __restrict__ done,
                                                      unsigned* __restrict__ cnt,
                                                      double* __restrict__ rout) {
  if (done && *done) return;
  __shared__ double sh[TBX * TBY / MGAR_WAVE];
  const int i = blockIdx.x * TBX + threadIdx.x;
  const int j = blockIdx.y * TBY + threadIdx.y;
  const int kz = blockIdx.z;
  const bool valid = i < g.nnx && j < g.nny;
  double dotv = 0.0;
  if (valid) {
    const long long n = geo_node(g, i, j, kz);
    T r = T(0);
    if (!geo_fixed(g, i, j, kz)) {
      T kv[2][2][2];
      load_cells<DIM, MODE == SM_NEG_DK>(g, k, kref, i, j, kz, kv);
      T ksum = T(0);
      T y = T(0);
      if (MODE != SM_JACOBI0) {
        y = node_apply<DIM, T>(g, x, i, j, kz, kv, ksum);
      } else if (DIM == 3) {
        const T z3[3][3] = {};
        (void)apply27<T, false>(z3, z3, z3, kv[0], kv[1], T(0), T(0), ksum);
      } else {
        ksum = ((kv[0][0][0] + kv[0][0][1]) + kv[0][1][0]) + kv[0][1][1];
      }
      const T diag = T(DIM == 3 ? g.h * (1.0 / 3.0) : (2.0 / 3.0)) * ksum;
      if (MODE == SM_APPLY || MODE == SM_APPLY_DOT) {
        r = y;
        if (MODE == SM_APPLY_DOT) dotv = (double)x[n] * (double)r;
      } else if (MODE == SM_RESID) {
        r = b[n] - y;
      } else if (MODE == SM_JACOBI || MODE == SM_JACOBI_DOT) {
        r = x[n] + omega * (b[n] - y) / diag;
        if (MODE == SM_JACOBI_DOT) dotv = (double)b[n] * (double)r;
      } else if (MODE == SM_JACOBI0) {
        r = omega * b[n] / diag;
      } else if (MODE == SM_NEG_DK) {
        r = -y;
      }
    }
    out[n] = r;
  }
  if (MODE == SM_APPLY_DOT || MODE == SM_JACOBI_DOT) {
    const double s = block_sum(dotv, sh);
    if (cnt) grid_reduce(s, flat_bid(), gridDim.x * gridDim.y * gridDim.z, part, cnt, rout, sh, nullptr);
    else if (flat_tid() == 0) part[flat_bid()] = s;
  }
}

// Node-parallel stencil on buffer loads: all 2^d cell and up to 21 neighbour
// loads of a thread are issued together (no branch separates them); the
// per-node arithmetic is that of k_stencil. Threads past the grid and nodes
// outside it read 0 and store nothing.
// Node n (flat index) of grid g: writes out[n] and returns this node's term
// of the dot of modes 1 and 4 (0 past the grid).
template <int DIM, int MODE, typename T, typename CL>
__device__ inline double stencil_b_point(const Geo& g, long long n, const T* __restrict__ x, CL k,
                                         CL kref, const T* __restrict__ b, T* __restrict__ out,
                                         T omega) {
  using E = typename CL::E;
  constexpr unsigned TS = sizeof(T), ES = sizeof(E);
  constexpr bool DK = (MODE == SM_NEG_DK);
  constexpr bool CMASK = sizeof(E) == 2;   // a raw 0 of a BF16 array is not a zero conductivity
  const bool valid = n < g.nn;
  int i, j, kz;
  node_ijk(g, n, i, j, kz);   // past the grid: kz >= nnz, so every offset is out of range
  const __amdgpu_buffer_rsrc_t rx = zrsrc(x, g.nn * TS);
  const __amdgpu_buffer_rsrc_t rb = zrsrc(b, g.nn * TS);
  const __amdgpu_buffer_rsrc_t ro = zrsrc(out, g.nn * TS);
  const __amdgpu_buffer_rsrc_t rk = zrsrc(k.p, g.ne * ES);
  const __amdgpu_buffer_rsrc_t rkr = zrsrc(kref.p, g.ne * ES);
  const unsigned own = node_boff(g, i, j, kz, TS);   // ZOOB for threads past the grid
  T kv[2][2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (DIM == 2 && c == 1) { kv[c][bb][a] = T(0); continue; }
        const unsigned o = cell_boff(g, i - 1 + a, j - 1 + bb, DIM == 3 ? kz - 1 + c : 0, ES);
        T v = T(k.value(zbload<E>(rk, o)));
        if (DK) v -= T(kref.value(zbload<E>(rkr, o)));
        kv[c][bb][a] = CMASK ? v * (o < ZOOB ? T(1) : T(0)) : v;
      }
  T ksum = T(0), y = T(0), xn = T(0);
  if (DIM == 2) {
    T xv[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx)
        xv[dy][dx] = (MODE == SM_JACOBI0) ? T(0) : zbload<T>(rx, node_boff(g, i + dx - 1, j + dy - 1, 0, TS));
    xn = xv[1][1];
    T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int sx = a ? 2 : 0, sy = bb ? 2 : 0;
        const T ke = kv[0][bb][a];
        s0 += ke;
        s1 += ke * (xv[1][sx] + xv[sy][1]);
        s2 += ke * xv[sy][sx];
      }
    ksum = s0;
    y = T(2.0 / 3.0) * s0 * xv[1][1] - T(1.0 / 6.0) * s1 - T(1.0 / 3.0) * s2;
  } else {
    T xv[3][3][3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int nzr = (dx != 1) + (dy != 1) + (dz != 1);
          xv[dz][dy][dx] = (nzr == 1 || MODE == SM_JACOBI0)
                               ? T(0)
                               : zbload<T>(rx, node_boff(g, i + dx - 1, j + dy - 1, kz + dz - 1, TS));
        }
    xn = xv[1][1][1];
    if (MODE != SM_JACOBI0)
      y = apply27<T, true>(xv[0], xv[1], xv[2], kv[0], kv[1], T(g.h * (1.0 / 3.0)), T(g.h * (1.0 / 12.0)),
                           ksum);
    else
      (void)apply27<T, false>(xv[0], xv[1], xv[2], kv[0], kv[1], T(0), T(0), ksum);
  }
  if (DIM == 2 && MODE == SM_JACOBI0)
    ksum = ((kv[0][0][0] + kv[0][0][1]) + kv[0][1][0]) + kv[0][1][1];
  const T bn = (MODE == SM_RESID || MODE == SM_JACOBI || MODE == SM_JACOBI_DOT || MODE == SM_JACOBI0)
                   ? zbload<T>(rb, own)
                   : T(0);
  const T diag = T(DIM == 3 ? g.h * (1.0 / 3.0) : (2.0 / 3.0)) * ksum;
  T r = T(0);
  if (MODE == SM_APPLY || MODE == SM_APPLY_DOT) r = y;
  else if (MODE == SM_RESID) r = bn - y;
  else if (MODE == SM_JACOBI || MODE == SM_JACOBI_DOT) r = xn + omega * (bn - y) / diag;
  else if (MODE == SM_JACOBI0) r = omega * bn / diag;
  else if (MODE == SM_NEG_DK) r = -y;
  r = geo_fixed(g, i, j, kz) ? T(0) : r;
  zbstore(r, ro, own);
  const double d = (MODE == SM_APPLY_DOT) ? (double)xn * (double)r
                   : (MODE == SM_JACOBI_DOT) ? (double)bn * (double)r : 0.0;
  return valid ? d : 0.0;
}

template <int DIM, int MODE, typename T, typename CL>
__global__ __launch_bounds__(TBX* TBY) void k_stencil_b(Geo g, const T* __restrict__ x, CL k, CL kref,
                                                        const T* __restrict__ b, T* __restrict__ out,
                                                        T omega, double* __restrict__ part,
                                                        const int* __restrict__ done,
                                                        unsigned* __restrict__ cnt,
                                                        double* __restrict__ rout) {
  if (done && *done) return;
  __shared__ double sh[TBX * TBY / MGAR_WAVE];
  const long long n = (long long)blockIdx.x * (TBX * TBY) + flat_tid();
  const double d = stencil_b_point<DIM, MODE, T, CL>(g, n, x, k, kref, b, out, omega);
  if (MODE == SM_APPLY_DOT || MODE == SM_JACOBI_DOT) {
    const double s = block_sum(d, sh);
    if (cnt) grid_reduce(s, blockIdx.x, gridDim.x, part, cnt, rout, sh, nullptr);
    else if (flat_tid() == 0) part[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// 3D z-marching stencil for the large grids. A block owns a TXW x TYH tile of
// node columns and walks KZ consecutive z-planes. Each plane of x (tile plus a
// one-node halo) and each plane of cell conductivities (tile plus the cells
// below-left of it) passes through a ring of LDS slots: while node plane k is
// computed from LDS, the next ZD planes are already in flight in registers.
// A thread issues five global loads per plane (two x slots, two cell slots
// and its own b) and reads its 21 weighted neighbours from LDS. The fills are
// branch-free: every thread stores both of its slots each plane; a slot
// outside the tile halo or the grid loads from a clamped in-grid address and
// stores 0. Tiles split each row evenly (129 = 3 x 43), so no block is left
// with a single column.
// Block ids are remapped so that each XCD (blocks are dealt round-robin to the
// 8 XCDs) receives a contiguous range of tiles, z-chunk slowest: halo rows and
// planes shared by neighbouring tiles then hit in that XCD's L2.
constexpr int ZT = 256;
constexpr int XCAP = 420;   // >= (TXW+2)(TYH+2): halo-tile nodes of one plane
constexpr int CCAP = 360;   // >= (TXW+1)(TYH+1): cells of one plane around the tile
constexpr int ZSLOT = 2 * ZT;  // LDS slots per staged plane (two per thread)
static_assert(XCAP <= ZSLOT && CCAP <= ZSLOT, "two fill slots per thread must cover a plane");

__device__ inline int xcd_remap(int bid, int nb) {
  const int xcd = bid & 7, local = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return xcd * q + (xcd < r ? xcd : r) + local;
}

// Byte offset, inside one plane of extent nxl x nyl, of LDS fill slot idx:
// position (i0 - 1 + idx % W, j0 - 1 + idx / W) of the tile halo, or ZOOB when
// the slot is not a real position (past the n slots, or outside the plane).
__device__ inline unsigned zslot_off(int i0, int j0, int W, int n, int idx, int nxl, int nyl,
                                     unsigned esz) {
  const int ii = i0 - 1 + idx % W, jj = j0 - 1 + idx / W;
  const bool ok = idx < n && ii >= 0 && ii < nxl && jj >= 0 && jj < nyl;
  return ok ? (unsigned)(ii + nxl * jj) * esz : ZOOB;
}

// Offset of plane p (any int) for a slot offset: out of range -> >= ZOOB.
__device__ inline unsigned zplane(unsigned soff, int p, int np, unsigned plb) {
  return (p >= 0 && p < np) ? soff + (unsigned)p * plb : ZOOB;
}

template <int MODE, int ZD, typename T, typename CL>
__global__ __launch_bounds__(ZT) __attribute__((amdgpu_waves_per_eu((ZD == 1 || sizeof(T) == 4) ? 4 : 3))) void k_stencil_z(
    Geo g, int TXW, int TYH, int ntx, int nty, int KZ, const T* __restrict__ x, CL k, CL kref,
    const T* __restrict__ b, T* __restrict__ out, T omega, double* __restrict__ part,
    const int* __restrict__ done, unsigned* __restrict__ cnt, double* __restrict__ rout, PFuse) {
  if (done && *done) return;
  using E = typename CL::E;
  constexpr bool DK = (MODE == SM_NEG_DK);
  constexpr bool NEEDX = (MODE != SM_JACOBI0);
  constexpr bool NEEDB = (MODE == SM_RESID || MODE == SM_JACOBI || MODE == SM_JACOBI_DOT ||
                          MODE == SM_JACOBI0);
  constexpr bool DOT = (MODE == SM_APPLY_DOT || MODE == SM_JACOBI_DOT);
  constexpr unsigned TS = sizeof(T), ES = sizeof(E);
  __shared__ T Xs[2][ZSLOT];
  __shared__ T Cs[2][ZSLOT];
  __shared__ double sh[ZT / MGAR_WAVE];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int nxy = ntx * nty;
  const int txy = t % nxy, zc = t / nxy;
  const int i0 = (txy % ntx) * TXW, j0 = (txy / ntx) * TYH;
  const int XW = TXW + 2, XN = XW * (TYH + 2);
  const int CW = TXW + 1, CN = CW * (TYH + 1);
  const int tid = threadIdx.x;
  const int lx = tid % TXW, ly = tid / TXW;
  const int i = i0 + lx, j = j0 + ly;
  const bool act = ly < TYH && i < g.nnx && j < g.nny;
  const int k0 = zc * KZ;
  const int k1 = min(k0 + KZ, g.nnz);
  const unsigned plb = (unsigned)(g.nnx * g.nny) * TS;      // node plane, bytes
  const unsigned cplb = (unsigned)(g.nx * g.ny) * ES;       // cell plane, bytes
  const __amdgpu_buffer_rsrc_t rx = zrsrc(x, g.nn * TS);
  const __amdgpu_buffer_rsrc_t rb = zrsrc(b, g.nn * TS);
  const __amdgpu_buffer_rsrc_t ro = zrsrc(out, g.nn * TS);
  const __amdgpu_buffer_rsrc_t rk = zrsrc(k.p, g.ne * ES);
  const __amdgpu_buffer_rsrc_t rkr = zrsrc(kref.p, g.ne * ES);
  const unsigned own = act ? (unsigned)(i + g.nnx * j) * TS : ZOOB;   // this thread's node column
  const unsigned xs0 = zslot_off(i0, j0, XW, XN, tid, g.nnx, g.nny, TS);
  const unsigned xs1 = zslot_off(i0, j0, XW, XN, tid + ZT, g.nnx, g.nny, TS);
  const unsigned cs0 = zslot_off(i0, j0, CW, CN, tid, g.nx, g.ny, ES);
  const unsigned cs1 = zslot_off(i0, j0, CW, CN, tid + ZT, g.nx, g.ny, ES);
  // LDS index of this thread's node (x planes) and of its lower-left cell
  const int xc = act ? (ly + 1) * XW + (lx + 1) : XW + 1;
  const int cb = act ? ly * CW + lx : 0;

  // raw loads: x plane p of a slot, cell plane ez of a slot (both cell arrays
  // for the dK mode), b of this thread's node in plane p
#define ZX(so, p) (NEEDX ? zbload<T>(rx, zplane((so), (p), g.nnz, plb)) : T(0))
#define ZB(p) (NEEDB ? zbload<T>(rb, zplane(own, (p), g.nnz, plb)) : T(0))
  // cell value of a raw element pair (k, kref). An out-of-range load reads a
  // raw 0, which is a zero conductivity for FP64/FP32 cells but a density for
  // BF16 cells; those are masked by a multiply (a select on a loaded value
  // would be compiled into a branch around the load).
  constexpr bool CMASK = sizeof(E) == 2;
#define ZCV(e, er) (DK ? T(k.value(e)) - T(kref.value(er)) : T(k.value(e)))
#define ZCM(e, er, ok) (CMASK ? ZCV(e, er) * ((ok) ? T(1) : T(0)) : ZCV(e, er))

  // register queue of raw global loads: entry d holds x plane kk+1+d, cell
  // plane kk+d and b of plane kk+d for the step of node plane kk
  T qx0[ZD], qx1[ZD], qb[ZD];
  E qc0[ZD], qc1[ZD], qr0[ZD], qr1[ZD];
  // rolling register window: 3x3 of three x planes, 2x2 of two cell planes
  T W0[3][3], W1[3][3], W2[3][3], V0[2][2], V1[2][2];

  // prologue: planes k0-1 and k0 and cells k0-1 go through LDS into W0, W1, V0
  {
    const unsigned c0 = zplane(cs0, k0 - 1, g.nz, cplb), c1 = zplane(cs1, k0 - 1, g.nz, cplb);
    Xs[0][tid] = ZX(xs0, k0 - 1);
    Xs[1][tid] = ZX(xs0, k0);
    Xs[0][tid + ZT] = ZX(xs1, k0 - 1);
    Xs[1][tid + ZT] = ZX(xs1, k0);
    const E e0 = zbload<E>(rk, c0), e1 = zbload<E>(rk, c1);
    const E r0 = DK ? zbload<E>(rkr, c0) : E(0), r1 = DK ? zbload<E>(rkr, c1) : E(0);
    Cs[0][tid] = ZCM(e0, r0, c0 < ZOOB);
    Cs[0][tid + ZT] = ZCM(e1, r1, c1 < ZOOB);
  }
#pragma unroll
  for (int d = 0; d < ZD; ++d) {
    qx0[d] = ZX(xs0, k0 + 1 + d);
    qx1[d] = ZX(xs1, k0 + 1 + d);
    const unsigned c0 = zplane(cs0, k0 + d, g.nz, cplb), c1 = zplane(cs1, k0 + d, g.nz, cplb);
    qc0[d] = zbload<E>(rk, c0);
    qc1[d] = zbload<E>(rk, c1);
    qr0[d] = DK ? zbload<E>(rkr, c0) : E(0);
    qr1[d] = DK ? zbload<E>(rkr, c1) : E(0);
    qb[d] = ZB(k0 + d);
  }
  __syncthreads();
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      W0[dy][dx] = Xs[0][xc + (dy - 1) * XW + dx - 1];
      W1[dy][dx] = Xs[1][xc + (dy - 1) * XW + dx - 1];
    }
#pragma unroll
  for (int bb = 0; bb < 2; ++bb)
#pragma unroll
    for (int a = 0; a < 2; ++a) V0[bb][a] = Cs[0][cb + bb * CW + a];
  __syncthreads();

  const bool colfix = act && i >= g.f0x && i <= g.f1x && j >= g.f0y && j <= g.f1y;
  const T hc = T(g.h * (1.0 / 3.0)), hf = T(g.h * (1.0 / 12.0));
  double dotv = 0.0;

  // One node plane kk: stage plane kk+1 and cells kk through LDS slot s, read
  // this thread's window of them into C and CB, refill the load queue, and
  // apply the stencil with A (plane kk-1), B (plane kk), C (plane kk+1),
  // CA (cells below), CB (cells above). The body has no branch, so the loads
  // of the queue stay in flight across steps.
#define ZSTEP(A, B, C, CA, CB, s)                                                            \
  {                                                                                          \
    Xs[s][tid] = qx0[0];                                                                     \
    Xs[s][tid + ZT] = qx1[0];                                                                \
    Cs[s][tid] = ZCM(qc0[0], qr0[0], cs0 < ZOOB && kk < g.nz);                               \
    Cs[s][tid + ZT] = ZCM(qc1[0], qr1[0], cs1 < ZOOB && kk < g.nz);                          \
    const T bn = qb[0];                                                                      \
    _Pragma("unroll") for (int d = 0; d + 1 < ZD; ++d) {                                     \
      qx0[d] = qx0[d + 1]; qx1[d] = qx1[d + 1];                                              \
      qc0[d] = qc0[d + 1]; qc1[d] = qc1[d + 1];                                              \
      qr0[d] = qr0[d + 1]; qr1[d] = qr1[d + 1];                                              \
      qb[d] = qb[d + 1];                                                                     \
    }                                                                                        \
    __syncthreads();                                                                         \
    if (NEEDX) {                                                                             \
      _Pragma("unroll") for (int dy = 0; dy < 3; ++dy)                                       \
      _Pragma("unroll") for (int dx = 0; dx < 3; ++dx)                                       \
        C[dy][dx] = Xs[s][xc + (dy - 1) * XW + dx - 1];                                      \
    }                                                                                        \
    _Pragma("unroll") for (int bb = 0; bb < 2; ++bb)                                         \
    _Pragma("unroll") for (int a = 0; a < 2; ++a) CB[bb][a] = Cs[s][cb + bb * CW + a];       \
    {                                                                                        \
      const int pf = kk + ZD;                                                                \
      qx0[ZD - 1] = ZX(xs0, pf + 1);                                                         \
      qx1[ZD - 1] = ZX(xs1, pf + 1);                                                         \
      const unsigned c0 = zplane(cs0, pf, g.nz, cplb), c1 = zplane(cs1, pf, g.nz, cplb);     \
      qc0[ZD - 1] = zbload<E>(rk, c0);                                                       \
      qc1[ZD - 1] = zbload<E>(rk, c1);                                                       \
      if (DK) qr0[ZD - 1] = zbload<E>(rkr, c0);                                              \
      if (DK) qr1[ZD - 1] = zbload<E>(rkr, c1);                                              \
      qb[ZD - 1] = ZB(pf);                                                                   \
    }                                                                                        \
    T ks;                                                                                    \
    const T y = apply27<T, NEEDX>(A, B, C, CA, CB, hc, hf, ks);                              \
    const T xcv = NEEDX ? B[1][1] : T(0);                                                    \
    const T diag = hc * ks;                                                                  \
    T r = T(0);                                                                              \
    if (MODE == SM_APPLY || MODE == SM_APPLY_DOT) r = y;                                     \
    else if (MODE == SM_RESID) r = bn - y;                                                   \
    else if (MODE == SM_JACOBI || MODE == SM_JACOBI_DOT) r = xcv + omega * (bn - y) / diag;  \
    else if (MODE == SM_JACOBI0) r = omega * bn / diag;                                      \
    else if (MODE == SM_NEG_DK) r = -y;                                                      \
    r = (colfix && kk >= g.f0z && kk <= g.f1z) ? T(0) : r;                                   \
    if (MODE == SM_APPLY_DOT) dotv += act ? (double)xcv * (double)r : 0.0;                   \
    if (MODE == SM_JACOBI_DOT) dotv += act ? (double)bn * (double)r : 0.0;                   \
    zbstore(r, ro, own + (unsigned)kk * plb);                                                \
    ++kk;                                                                                    \
  }

  // Six steps rotate the three x windows and the two cell windows back to
  // their starting roles, so the window never moves between registers.
  int kk = k0;
  while (kk + 6 <= k1) {
    ZSTEP(W0, W1, W2, V0, V1, 0)
    ZSTEP(W1, W2, W0, V1, V0, 1)
    ZSTEP(W2, W0, W1, V0, V1, 0)
    ZSTEP(W0, W1, W2, V1, V0, 1)
    ZSTEP(W1, W2, W0, V0, V1, 0)
    ZSTEP(W2, W0, W1, V1, V0, 1)
  }
  if (kk < k1) ZSTEP(W0, W1, W2, V0, V1, 0)
  if (kk < k1) ZSTEP(W1, W2, W0, V1, V0, 1)
  if (kk < k1) ZSTEP(W2, W0, W1, V0, V1, 0)
  if (kk < k1) ZSTEP(W0, W1, W2, V1, V0, 1)
  if (kk < k1) ZSTEP(W1, W2, W0, V0, V1, 0)
#undef ZSTEP
#undef ZX
#undef ZB
#undef ZCV
#undef ZCM
  if (DOT) {
    const double sum = block_sum(dotv, sh);
    if (cnt) grid_reduce(sum, blockIdx.x, gridDim.x, part, cnt, rout, sh, nullptr);
    else if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// Two-row variant of the z-marching stencil: each thread computes the nodes
// (i, j) and (i, j + 1) of every plane, so a block's tile is twice as tall for
// the same 256 threads. The two nodes share their x window (4 x 3 per plane
// instead of 2 x 3 x 3) and cell window (3 x 2 instead of 2 x 2 x 2): fewer
// LDS reads and more independent arithmetic per thread. Same per-node formula
// (apply27g) as every other stencil kernel.
constexpr int XCAP2 = 3 * ZT;  // x fill slots per plane (three per thread)
constexpr int CCAP2 = 2 * ZT;  // cell fill slots per plane (two per thread)

template <int MODE, int ZD, typename T, typename CL>
__global__ __launch_bounds__(ZT) void k_stencil_z2(
    Geo g, int TXW, int TYH, int ntx, int nty, int KZ, const T* __restrict__ x, CL k, CL kref,
    const T* __restrict__ b, T* __restrict__ out, T omega, double* __restrict__ part,
    const int* __restrict__ done, unsigned* __restrict__ cnt, double* __restrict__ rout, PFuse fu) {
  using E = typename CL::E;
  constexpr bool PU = (MODE == SM_PAPPLY_DOT);   // x holds z; staged value z + beta p_old
  constexpr bool J0R = (MODE == SM_J0RESID);     // x holds b; staged value w b / diag
  constexpr bool XF = PU || J0R;                 // staged x formed from two inputs
  constexpr bool DK = (MODE == SM_NEG_DK);
  constexpr bool NEEDX = (MODE != SM_JACOBI0);
  constexpr bool NEEDB = (MODE == SM_RESID || MODE == SM_JACOBI || MODE == SM_JACOBI_DOT ||
                          MODE == SM_JACOBI0 || J0R);
  constexpr bool DOT = (MODE == SM_APPLY_DOT || MODE == SM_JACOBI_DOT || PU);
  constexpr bool CMASK = sizeof(E) == 2;
  constexpr unsigned TS = sizeof(T), ES = sizeof(E);
  __shared__ T Xs[2][XCAP2];
  __shared__ T Cs[2][CCAP2];
  __shared__ double sh[ZT / MGAR_WAVE];
  // The scalars of the fused steps (stopping test of the previous iteration,
  // direction update) are read in one round with the done flag, and the raw
  // loads of the first planes go out before the block reduction that needs
  // them: a block's first plane loads do not wait behind a chain of dependent
  // scalar reads.
  const bool chk = J0R && fu.chk;
  int dn = done ? *done : 0;
  double rzv = 0.0;   // this thread's share of the r.z (PU) or ||r||^2 (chk) partials
  int sit = 0;
  double rzh0 = 0.0, rzh1 = 0.0, sqq = 0.0;
  if (PU || chk) {
    rzv = thread_partials(fu.rzp, fu.nrz, threadIdx.x, ZT);
    if (PU) {
      sit = fu.st->it;
      rzh0 = fu.st->rz[0];
      rzh1 = fu.st->rz[1];
    } else {
      dn |= fu.st->done;
      sit = fu.st->itn;
      sqq = fu.st->qq;
    }
  }
  if (dn) return;
  T beta = T(0);
  const T* pold = nullptr;
  T* pnew = nullptr;
  if (PU) {
    pold = reinterpret_cast<const T*>(fu.pbuf[(sit + 1) & 1]);
    pnew = reinterpret_cast<T*>(fu.pbuf[sit & 1]);
  }
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int nxy = ntx * nty;
  const int txy = t % nxy, zc = t / nxy;
  const int i0 = (txy % ntx) * TXW, j0 = (txy / ntx) * TYH;
  const int XW = TXW + 2, XN = XW * (TYH + 2);
  const int CW = TXW + 1, CN = CW * (TYH + 1);
  const int tid = threadIdx.x;
  const int lx = tid % TXW, ly = tid / TXW;   // ly: pair of rows 2ly, 2ly + 1 of the tile
  const int i = i0 + lx, j = j0 + 2 * ly;
  const bool actp = 2 * ly < TYH && i < g.nnx;
  const bool act0 = actp && j < g.nny, act1 = actp && j + 1 < g.nny;
  const int k0 = zc * KZ;
  const int k1 = min(k0 + KZ, g.nnz);
  const unsigned plb = (unsigned)(g.nnx * g.nny) * TS;
  const unsigned cplb = (unsigned)(g.nx * g.ny) * ES;
  const __amdgpu_buffer_rsrc_t rx = zrsrc(x, g.nn * TS);
  const __amdgpu_buffer_rsrc_t rb = zrsrc(b, g.nn * TS);
  const __amdgpu_buffer_rsrc_t ro = zrsrc(out, g.nn * TS);
  const __amdgpu_buffer_rsrc_t rk = zrsrc(k.p, g.ne * ES);
  const __amdgpu_buffer_rsrc_t rkr = zrsrc(kref.p, g.ne * ES);
  if (J0R) {
    pold = reinterpret_cast<const T*>(fu.diag);
    pnew = reinterpret_cast<T*>(fu.xout);
  }
  const __amdgpu_buffer_rsrc_t rp = zrsrc(XF ? pold : x, g.nn * TS);
  const __amdgpu_buffer_rsrc_t rpn = zrsrc(XF ? pnew : out, g.nn * TS);
  const unsigned own0 = act0 ? (unsigned)(i + g.nnx * j) * TS : ZOOB;
  const unsigned own1 = act1 ? (unsigned)(i + g.nnx * (j + 1)) * TS : ZOOB;
  const unsigned xs0 = zslot_off(i0, j0, XW, XN, tid, g.nnx, g.nny, TS);
  const unsigned xs1 = zslot_off(i0, j0, XW, XN, tid + ZT, g.nnx, g.nny, TS);
  const unsigned xs2 = zslot_off(i0, j0, XW, XN, tid + 2 * ZT, g.nnx, g.nny, TS);
  const unsigned cs0 = zslot_off(i0, j0, CW, CN, tid, g.nx, g.ny, ES);
  const unsigned cs1 = zslot_off(i0, j0, CW, CN, tid + ZT, g.nx, g.ny, ES);
  // LDS index of the top-left of this thread's x window (4 rows x 3) and cell
  // window (3 rows x 2); inactive threads read a valid in-tile window
  const int xw = actp ? (2 * ly) * XW + lx : 0;
  const int cw = actp ? (2 * ly) * CW + lx : 0;

#define ZX(so, p) (NEEDX ? zbload<T>(rx, zplane((so), (p), g.nnz, plb)) : T(0))
#define ZB(own, p) (NEEDB ? zbload<T>(rb, zplane((own), (p), g.nnz, plb)) : T(0))
#define ZCV(e, er) (DK ? T(k.value(e)) - T(kref.value(er)) : T(k.value(e)))
#define ZCM(e, er, ok) (CMASK ? ZCV(e, er) * ((ok) ? T(1) : T(0)) : ZCV(e, er))

  // second input of a fused mode at a slot and plane (p_old, or the diagonal),
  // and the staged value formed from the pair (u = x input, v = second input).
  // A slot outside the grid loads 0 for both; max(v, DBL_MIN) keeps its sweep 0.
#define ZP(so, p) (XF ? zbload<T>(rp, zplane((so), (p), g.nnz, plb)) : T(0))
#define ZFORM(u, v) (PU ? (u) + beta * (v) : J0R ? omega * (u) / fmax((v), TMIN) : (u))
  constexpr T TMIN = std::numeric_limits<T>::min();
  constexpr int ZQP = XF ? ZD : 1;
  T qx0[ZD], qx1[ZD], qx2[ZD], qb0[ZD], qb1[ZD];
  T qp0[ZQP], qp1[ZQP], qp2[ZQP];
  E qc0[ZD], qc1[ZD], qr0[ZD], qr1[ZD];
  T W0[4][3], W1[4][3], W2[4][3], V0[3][2], V1[3][2];

  // raw loads of planes k0 - 1 and k0 (x, second input, first cell plane)
  // and of the queue
  T px[3][2], pp[3][2];
  E pe[2], pr[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    px[0][a] = ZX(xs0, k0 - 1 + a);
    px[1][a] = ZX(xs1, k0 - 1 + a);
    px[2][a] = ZX(xs2, k0 - 1 + a);
    pp[0][a] = ZP(xs0, k0 - 1 + a);
    pp[1][a] = ZP(xs1, k0 - 1 + a);
    pp[2][a] = ZP(xs2, k0 - 1 + a);
  }
  const unsigned pc0 = zplane(cs0, k0 - 1, g.nz, cplb), pc1 = zplane(cs1, k0 - 1, g.nz, cplb);
  pe[0] = zbload<E>(rk, pc0);
  pe[1] = zbload<E>(rk, pc1);
  pr[0] = DK ? zbload<E>(rkr, pc0) : E(0);
  pr[1] = DK ? zbload<E>(rkr, pc1) : E(0);
#pragma unroll
  for (int d = 0; d < ZD; ++d) {
    qx0[d] = ZX(xs0, k0 + 1 + d);
    qx1[d] = ZX(xs1, k0 + 1 + d);
    qx2[d] = ZX(xs2, k0 + 1 + d);
    if (XF) {
      qp0[d] = ZP(xs0, k0 + 1 + d);
      qp1[d] = ZP(xs1, k0 + 1 + d);
      qp2[d] = ZP(xs2, k0 + 1 + d);
    }
    const unsigned c0 = zplane(cs0, k0 + d, g.nz, cplb), c1 = zplane(cs1, k0 + d, g.nz, cplb);
    qc0[d] = zbload<E>(rk, c0);
    qc1[d] = zbload<E>(rk, c1);
    qr0[d] = DK ? zbload<E>(rkr, c0) : E(0);
    qr1[d] = DK ? zbload<E>(rkr, c1) : E(0);
    qb0[d] = ZB(own0, k0 + d);
    qb1[d] = ZB(own1, k0 + d);
  }
  // fused stopping test of the previous iteration (same test as k_cg_check):
  // every block sums the ||r||^2 partials in the same order and takes the same
  // decision; the iteration count comes from st->itn, which no block of this
  // kernel writes
  if (chk) {
    CgState* st = fu.st;
    const double rr = block_sum(rzv, sh);
    const bool conv = sqrt(rr) <= fu.tol * sqrt(sqq);
    const bool stop = conv || sit >= fu.cg_max;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->it = sit;
      st->rr = rr;
      if (stop) {
        st->done = 1;
        st->converged = conv ? 1 : 0;
        st->iters = sit;
      }
    }
    if (stop) return;
  }
  // direction update: beta from the r.z partials (every block sums them in the
  // same order, so all hold the same value) and the stored r.z history
  if (PU) {
    const double rz = block_sum(rzv, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) fu.st->rz[sit & 1] = rz;
    beta = (T)((sit == 0) ? 0.0 : rz / ((sit - 1) & 1 ? rzh1 : rzh0));
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    Xs[a][tid] = ZFORM(px[0][a], pp[0][a]);
    Xs[a][tid + ZT] = ZFORM(px[1][a], pp[1][a]);
    Xs[a][tid + 2 * ZT] = ZFORM(px[2][a], pp[2][a]);
  }
  Cs[0][tid] = ZCM(pe[0], pr[0], pc0 < ZOOB);
  Cs[0][tid + ZT] = ZCM(pe[1], pr[1], pc1 < ZOOB);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      W0[r][dx] = Xs[0][xw + r * XW + dx];
      W1[r][dx] = Xs[1][xw + r * XW + dx];
    }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int a = 0; a < 2; ++a) V0[r][a] = Cs[0][cw + r * CW + a];
  __syncthreads();

  const bool colfix0 = act0 && i >= g.f0x && i <= g.f1x && j >= g.f0y && j <= g.f1y;
  const bool colfix1 = act1 && i >= g.f0x && i <= g.f1x && j + 1 >= g.f0y && j + 1 <= g.f1y;
  const T hc = T(g.h * (1.0 / 3.0)), hf = T(g.h * (1.0 / 12.0));
  double dotv = 0.0;

#define ZNODE(A, B, C, CA, CB, R0, bn, colfix, act, own)                                        \
  {                                                                                          \
    T ks;                                                                                    \
    const T y = apply27g<T, NEEDX>([&](int yy, int xx) { return A[R0 + yy][xx]; },          \
                                   [&](int yy, int xx) { return B[R0 + yy][xx]; },          \
                                   [&](int yy, int xx) { return C[R0 + yy][xx]; },          \
                                   [&](int yy, int xx) { return CA[R0 + yy][xx]; },         \
                                   [&](int yy, int xx) { return CB[R0 + yy][xx]; }, hc, hf, ks); \
    const T xcv = NEEDX ? B[R0 + 1][1] : T(0);                                               \
    const T diag = hc * ks;                                                                  \
    T r = T(0);                                                                              \
    if (MODE == SM_APPLY || MODE == SM_APPLY_DOT || PU) r = y;                               \
    else if (MODE == SM_RESID || J0R) r = bn - y;                                            \
    else if (MODE == SM_JACOBI || MODE == SM_JACOBI_DOT) r = xcv + omega * (bn - y) / diag;  \
    else if (MODE == SM_JACOBI0) r = omega * bn / diag;                                      \
    else if (MODE == SM_NEG_DK) r = -y;                                                      \
    r = (colfix && kk >= g.f0z && kk <= g.f1z) ? T(0) : r;                                   \
    if (MODE == SM_APPLY_DOT || PU) dotv += act ? (double)xcv * (double)r : 0.0;             \
    if (MODE == SM_JACOBI_DOT) dotv += act ? (double)bn * (double)r : 0.0;                   \
    zbstore(r, ro, own + (unsigned)kk * plb);                                                \
    if (XF) zbstore(xcv, rpn, own + (unsigned)kk * plb);                                     \
  }

#define ZSTEP2(A, B, C, CA, CB, s)                                                           \
  {                                                                                          \
    Xs[s][tid] = XF ? ZFORM(qx0[0], qp0[0]) : qx0[0];                                        \
    Xs[s][tid + ZT] = XF ? ZFORM(qx1[0], qp1[0]) : qx1[0];                                   \
    Xs[s][tid + 2 * ZT] = XF ? ZFORM(qx2[0], qp2[0]) : qx2[0];                               \
    Cs[s][tid] = ZCM(qc0[0], qr0[0], cs0 < ZOOB && kk < g.nz);                               \
    Cs[s][tid + ZT] = ZCM(qc1[0], qr1[0], cs1 < ZOOB && kk < g.nz);                          \
    const T bn0 = qb0[0], bn1 = qb1[0];                                                      \
    _Pragma("unroll") for (int d = 0; d + 1 < ZD; ++d) {                                     \
      qx0[d] = qx0[d + 1]; qx1[d] = qx1[d + 1]; qx2[d] = qx2[d + 1];                         \
      if (XF) { qp0[d] = qp0[d + 1]; qp1[d] = qp1[d + 1]; qp2[d] = qp2[d + 1]; }              \
      qc0[d] = qc0[d + 1]; qc1[d] = qc1[d + 1];                                              \
      qr0[d] = qr0[d + 1]; qr1[d] = qr1[d + 1];                                              \
      qb0[d] = qb0[d + 1]; qb1[d] = qb1[d + 1];                                              \
    }                                                                                        \
    __syncthreads();                                                                         \
    if (NEEDX) {                                                                             \
      _Pragma("unroll") for (int rr = 0; rr < 4; ++rr)                                       \
      _Pragma("unroll") for (int dx = 0; dx < 3; ++dx)                                       \
        C[rr][dx] = Xs[s][xw + rr * XW + dx];                                                \
    }                                                                                        \
    _Pragma("unroll") for (int rr = 0; rr < 3; ++rr)                                         \
    _Pragma("unroll") for (int a = 0; a < 2; ++a) CB[rr][a] = Cs[s][cw + rr * CW + a];       \
    {                                                                                        \
      const int pf = kk + ZD;                                                                \
      qx0[ZD - 1] = ZX(xs0, pf + 1);                                                         \
      qx1[ZD - 1] = ZX(xs1, pf + 1);                                                         \
      qx2[ZD - 1] = ZX(xs2, pf + 1);                                                         \
      if (XF) {                                                                              \
        qp0[ZD - 1] = ZP(xs0, pf + 1);                                                       \
        qp1[ZD - 1] = ZP(xs1, pf + 1);                                                       \
        qp2[ZD - 1] = ZP(xs2, pf + 1);                                                       \
      }                                                                                      \
      const unsigned c0 = zplane(cs0, pf, g.nz, cplb), c1 = zplane(cs1, pf, g.nz, cplb);     \
      qc0[ZD - 1] = zbload<E>(rk, c0);                                                       \
      qc1[ZD - 1] = zbload<E>(rk, c1);                                                       \
      if (DK) qr0[ZD - 1] = zbload<E>(rkr, c0);                                              \
      if (DK) qr1[ZD - 1] = zbload<E>(rkr, c1);                                              \
      qb0[ZD - 1] = ZB(own0, pf);                                                            \
      qb1[ZD - 1] = ZB(own1, pf);                                                            \
    }                                                                                        \
    ZNODE(A, B, C, CA, CB, 0, bn0, colfix0, act0, own0)                                      \
    ZNODE(A, B, C, CA, CB, 1, bn1, colfix1, act1, own1)                                      \
    ++kk;                                                                                    \
  }

  int kk = k0;
  while (kk + 6 <= k1) {
    ZSTEP2(W0, W1, W2, V0, V1, 0)
    ZSTEP2(W1, W2, W0, V1, V0, 1)
    ZSTEP2(W2, W0, W1, V0, V1, 0)
    ZSTEP2(W0, W1, W2, V1, V0, 1)
    ZSTEP2(W1, W2, W0, V0, V1, 0)
    ZSTEP2(W2, W0, W1, V1, V0, 1)
  }
  if (kk < k1) ZSTEP2(W0, W1, W2, V0, V1, 0)
  if (kk < k1) ZSTEP2(W1, W2, W0, V1, V0, 1)
  if (kk < k1) ZSTEP2(W2, W0, W1, V0, V1, 0)
  if (kk < k1) ZSTEP2(W0, W1, W2, V1, V0, 1)
  if (kk < k1) ZSTEP2(W1, W2, W0, V0, V1, 0)
#undef ZSTEP2
#undef ZNODE
#undef ZFORM
#undef ZP
#undef ZX
#undef ZB
#undef ZCV
#undef ZCM
  if (DOT) {
    const double sum = block_sum(dotv, sh);
    if (cnt) grid_reduce(sum, blockIdx.x, gridDim.x, part, cnt, rout, sh, nullptr);
    else if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// Restriction r_c = P^T r_f: coarse node (I,J,K) gathers the fine nodes
// (2I+a, 2J+b, 2K+c), a,b,c in {-1,0,1}, with weight prod(1 if 0 else 1/2).
template <int DIM, typename T>
__global__ __launch_bounds__(TBX* TBY) void k_restrict(Geo gf, Geo gc, const T* __restrict__ rf,
                                                       T* __restrict__ rc,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  const int I = blockIdx.x * TBX + threadIdx.x;
  const int J = blockIdx.y * TBY + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= gc.nnx || J >= gc.nny) return;
  T s = T(0);
  if (!geo_fixed(gc, I, J, K)) {
#pragma unroll
    for (int c = (DIM == 3 ? -1 : 0); c <= (DIM == 3 ? 1 : 0); ++c) {
      T sy = T(0);
#pragma unroll
      for (int b = -1; b <= 1; ++b) {
        T sx = T(0);
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
          const T v = ldx(gf, rf, 2 * I + a, 2 * J + b, 2 * K + c);
          sx += T(a == 0 ? 1.0 : 0.5) * v;
        }
        sy += T(b == 0 ? 1.0 : 0.5) * sx;
      }
      s += T(c == 0 ? 1.0 : 0.5) * sy;
    }
  }
  rc[geo_node(gc, I, J, K)] = s;
}

// Interpolation and correction x_f += P x_c (bi-/trilinear; fixed fine rows are 0).
template <int DIM, typename T>
__global__ __launch_bounds__(TBX* TBY) void k_prolong(Geo gf, Geo gc, const T* __restrict__ xc,
                                                      T* __restrict__ xf,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.x * TBX + threadIdx.x;
  const int j = blockIdx.y * TBY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= gf.nnx || j >= gf.nny) return;
  if (geo_fixed(gf, i, j, k)) return;
  const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
  const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (DIM == 3 && (k & 1)) ? 2 : 1;
  const T wi = T((i & 1) ? 0.5 : 1.0), wj = T((j & 1) ? 0.5 : 1.0),
          wk = T((DIM == 3 && (k & 1)) ? 0.5 : 1.0);
  T s = T(0);
  for (int c = 0; c < nk; ++c) {
    T sy = T(0);
    for (int b = 0; b < nj; ++b) {
      T sx = T(0);
      for (int a = 0; a < ni; ++a) sx += xc[geo_node(gc, I0 + a, J0 + b, K0 + c)];
      sy += wi * sx;
    }
    s += wj * sy;
  }
  xf[geo_node(gf, i, j, k)] += wk * s;
}

// Buffer-load forms of the two transfers: every load of a thread in flight at
// once, nothing outside the grid read, same arithmetic as the kernels above.
template <int DIM, typename T>
__device__ inline T restrict_b_point(const Geo& gf, const Geo& gc, long long nc,
                                     const T* __restrict__ rf, T* __restrict__ rc) {
  constexpr unsigned TS = sizeof(T);
  int I, J, K;
  node_ijk(gc, nc, I, J, K);
  const __amdgpu_buffer_rsrc_t rr = zrsrc(rf, gf.nn * TS);
  const __amdgpu_buffer_rsrc_t ro = zrsrc(rc, gc.nn * TS);
  T s = T(0);
#pragma unroll
  for (int c = (DIM == 3 ? -1 : 0); c <= (DIM == 3 ? 1 : 0); ++c) {
    T sy = T(0);
#pragma unroll
    for (int bb = -1; bb <= 1; ++bb) {
      T sx = T(0);
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        const T v = zbload<T>(rr, node_boff(gf, 2 * I + a, 2 * J + bb, 2 * K + c, TS));
        sx += T(a == 0 ? 1.0 : 0.5) * v;
      }
      sy += T(bb == 0 ? 1.0 : 0.5) * sx;
    }
    s += T(c == 0 ? 1.0 : 0.5) * sy;
  }
  s = geo_fixed(gc, I, J, K) ? T(0) : s;
  zbstore(s, ro, node_boff(gc, I, J, K, TS));
  return s;
}

template <int DIM, typename T>
__global__ __launch_bounds__(TBX* TBY) void k_restrict_b(Geo gf, Geo gc, const T* __restrict__ rf,
                                                         T* __restrict__ rc,
                                                         const int* __restrict__ done) {
  if (done && *done) return;
  restrict_b_point<DIM, T>(gf, gc, (long long)blockIdx.x * (TBX * TBY) + flat_tid(), rf, rc);
}

// Diagonal of K per node (3D): h/3 times the sum of the node's 8 cells, in the
// association of the node formula. Used by the fused first sweep + residual.
template <typename T, typename CL>
__global__ __launch_bounds__(TBX* TBY) void k_diag(Geo g, CL k, T* __restrict__ diag) {
  using E = typename CL::E;
  constexpr unsigned ES = sizeof(E);
  constexpr bool CMASK = sizeof(E) == 2;   // a raw 0 of a BF16 array is not a zero conductivity
  const long long n = (long long)blockIdx.x * (TBX * TBY) + flat_tid();
  int i, j, kz;
  node_ijk(g, n, i, j, kz);
  const __amdgpu_buffer_rsrc_t rk = zrsrc(k.p, g.ne * ES);
  T kv[2][2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const unsigned o = cell_boff(g, i - 1 + a, j - 1 + bb, kz - 1 + c, ES);
        const T v = T(k.value(zbload<E>(rk, o)));
        kv[c][bb][a] = CMASK ? v * (o < ZOOB ? T(1) : T(0)) : v;
      }
  const T t00 = kv[0][0][0] + kv[1][0][0], t01 = kv[0][0][1] + kv[1][0][1];
  const T t10 = kv[0][1][0] + kv[1][1][0], t11 = kv[0][1][1] + kv[1][1][1];
  const T ks = (t00 + t01) + (t10 + t11);
  zbstore(T(g.h * (1.0 / 3.0)) * ks, zrsrc(diag, g.nn * sizeof(T)), node_boff(g, i, j, kz, sizeof(T)));
}

// Restriction followed by the first (zero-start) damped Jacobi sweep of the
// coarse grid, per coarse node: b_c = P^T r_f is stored, then
// x_c = omega b_c / diag(K_c) (0 at Dirichlet nodes). Same arithmetic as the
// restriction kernel followed by the stencil kernels in their sweep-from-zero
// mode (diagonal = h/3 resp. 2/3 times the sum of the node's cells, summed in
// the order of the node formula).
template <int DIM, typename T, typename CL>
__global__ __launch_bounds__(TBX* TBY) void k_restrict_j0(Geo gf, Geo gc, const T* __restrict__ rf,
                                                          CL kc, T* __restrict__ bc, T* __restrict__ xc,
                                                          T omega, const int* __restrict__ done) {
  if (done && *done) return;
  using E = typename CL::E;
  constexpr unsigned TS = sizeof(T), ES = sizeof(E);
  constexpr bool CMASK = sizeof(E) == 2;
  const long long n = (long long)blockIdx.x * (TBX * TBY) + flat_tid();
  const T bn = restrict_b_point<DIM, T>(gf, gc, n, rf, bc);
  int i, j, kz;
  node_ijk(gc, n, i, j, kz);
  const __amdgpu_buffer_rsrc_t rk = zrsrc(kc.p, gc.ne * ES);
  T kv[2][2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (DIM == 2 && c == 1) { kv[c][bb][a] = T(0); continue; }
        const unsigned o = cell_boff(gc, i - 1 + a, j - 1 + bb, DIM == 3 ? kz - 1 + c : 0, ES);
        const T v = T(kc.value(zbload<E>(rk, o)));
        kv[c][bb][a] = CMASK ? v * (o < ZOOB ? T(1) : T(0)) : v;
      }
  T ksum;
  if (DIM == 3) {
    const T t00 = kv[0][0][0] + kv[1][0][0], t01 = kv[0][0][1] + kv[1][0][1];
    const T t10 = kv[0][1][0] + kv[1][1][0], t11 = kv[0][1][1] + kv[1][1][1];
    ksum = (t00 + t01) + (t10 + t11);
  } else {
    ksum = ((kv[0][0][0] + kv[0][0][1]) + kv[0][1][0]) + kv[0][1][1];
  }
  const T diag = T(DIM == 3 ? gc.h * (1.0 / 3.0) : (2.0 / 3.0)) * ksum;
  T r = omega * bn / diag;
  r = geo_fixed(gc, i, j, kz) ? T(0) : r;
  zbstore(r, zrsrc(xc, gc.nn * TS), node_boff(gc, i, j, kz, TS));
}

template <int DIM, typename T>
__device__ inline void prolong_b_point(const Geo& gf, const Geo& gc, long long nf,
                                       const T* __restrict__ xc, T* __restrict__ xf) {
  constexpr unsigned TS = sizeof(T);
  int i, j, k;
  node_ijk(gf, nf, i, j, k);
  const __amdgpu_buffer_rsrc_t rc = zrsrc(xc, gc.nn * TS);
  const __amdgpu_buffer_rsrc_t rf = zrsrc(xf, gf.nn * TS);
  // fixed fine rows of P are 0: such nodes (and threads past the grid) use an
  // out-of-range offset, so they read 0 and their store is dropped
  const unsigned own = geo_fixed(gf, i, j, k) ? ZOOB : node_boff(gf, i, j, k, TS);
  const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
  // second coarse neighbour along an axis only for odd fine indices
  const T mi = T(i & 1), mj = T(j & 1), mk = T(DIM == 3 ? (k & 1) : 0);
  const T wi = T((i & 1) ? 0.5 : 1.0), wj = T((j & 1) ? 0.5 : 1.0),
          wk = T((DIM == 3 && (k & 1)) ? 0.5 : 1.0);
  T v[2][2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        v[c][bb][a] = (DIM == 2 && c == 1) ? T(0) : zbload<T>(rc, node_boff(gc, I0 + a, J0 + bb, K0 + c, TS));
  const T xo = zbload<T>(rf, own);
  T sc[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T s0 = v[c][0][0] + mi * v[c][0][1];
    const T s1 = v[c][1][0] + mi * v[c][1][1];
    sc[c] = wi * s0 + mj * (wi * s1);
  }
  const T s = wj * sc[0] + mk * (wj * sc[1]);
  zbstore(xo + wk * s, rf, own);
}

// The same correction organised per coarse node (I, J, K): its thread loads
// the 2^d coarse values of the cell above it once and updates the 2^d fine
// nodes (2I + a, 2J + b, 2K + c), a, b, c in {0, 1}, whose interpolation uses
// exactly those corners; per fine node the arithmetic is that of
// prolong_b_point. Fine nodes past the grid or fixed are skipped by an
// out-of-range offset.
template <int DIM, typename T>
__device__ inline void prolong_b8_point(const Geo& gf, const Geo& gc, long long nc,
                                        const T* __restrict__ xc, T* __restrict__ xf) {
  constexpr unsigned TS = sizeof(T);
  int I, J, K;
  node_ijk(gc, nc, I, J, K);   // past the coarse grid: its fine nodes are skipped below
  const __amdgpu_buffer_rsrc_t rc = zrsrc(xc, gc.nn * TS);
  const __amdgpu_buffer_rsrc_t rf = zrsrc(xf, gf.nn * TS);
  T v[2][2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        v[c][bb][a] = (DIM == 2 && c == 1) ? T(0) : zbload<T>(rc, node_boff(gc, I + a, J + bb, K + c, TS));
#pragma unroll
  for (int fc = 0; fc < (DIM == 3 ? 2 : 1); ++fc)
#pragma unroll
    for (int fb = 0; fb < 2; ++fb)
#pragma unroll
      for (int fa = 0; fa < 2; ++fa) {
        const int i = 2 * I + fa, j = 2 * J + fb, k = (DIM == 3) ? 2 * K + fc : 0;
        const bool in = nc < gc.nn && i < gf.nnx && j < gf.nny && k < gf.nnz;
        const unsigned own = (in && !geo_fixed(gf, i, j, k)) ? node_boff(gf, i, j, k, TS) : ZOOB;
        const T mi = T(fa), mj = T(fb), mk = T(DIM == 3 ? fc : 0);
        const T wi = T(fa ? 0.5 : 1.0), wj = T(fb ? 0.5 : 1.0), wk = T((DIM == 3 && fc) ? 0.5 : 1.0);
        const T xo = zbload<T>(rf, own);
        T sc[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const T s0 = v[c][0][0] + mi * v[c][0][1];
          const T s1 = v[c][1][0] + mi * v[c][1][1];
          sc[c] = wi * s0 + mj * (wi * s1);
        }
        const T s = wj * sc[0] + mk * (wj * sc[1]);
        zbstore(xo + wk * s, rf, own);
      }
}

template <int DIM, typename T>
__global__ __launch_bounds__(TBX* TBY) void k_prolong_b8(Geo gf, Geo gc, const T* __restrict__ xc,
                                                         T* __restrict__ xf,
                                                         const int* __restrict__ done) {
  if (done && *done) return;
  prolong_b8_point<DIM, T>(gf, gc, (long long)blockIdx.x * (TBX * TBY) + flat_tid(), xc, xf);
}

template <int DIM, typename T>
__global__ __launch_bounds__(TBX* TBY) void k_prolong_b(Geo gf, Geo gc, const T* __restrict__ xc,
                                                        T* __restrict__ xf,
                                                        const int* __restrict__ done) {
  if (done && *done) return;
  prolong_b_point<DIM, T>(gf, gc, (long long)blockIdx.x * (TBX * TBY) + flat_tid(), xc, xf);
}

// Interpolation followed by one damped Jacobi sweep, per fine node, for small
// grids where launches dominate: the interpolated iterate xa = xpre + P xc is
// formed on the fly at the node and its stencil neighbours (from a 3^d block
// of coarse values; the same expression per fine node as k_prolong_b8, and
// Dirichlet nodes keep xpre), then out = xa + w D^-1 (b - K xa) with the node
// formula of the stencil kernels. Results equal the two separate launches.
template <int DIM, typename T, typename CL>
__global__ __launch_bounds__(TBX* TBY) void k_prolong_jacobi(Geo gf, Geo gc, const T* __restrict__ xc,
                                                             const T* __restrict__ xpre, CL k,
                                                             const T* __restrict__ b, T* __restrict__ out,
                                                             T omega, const int* __restrict__ done) {
  if (done && *done) return;
  using E = typename CL::E;
  constexpr unsigned TS = sizeof(T), ES = sizeof(E);
  constexpr bool CMASK = sizeof(E) == 2;
  constexpr int NZ = DIM == 3 ? 3 : 1;
  const long long n = (long long)blockIdx.x * (TBX * TBY) + flat_tid();
  int i, j, kz;
  node_ijk(gf, n, i, j, kz);   // past the grid: kz >= nnz, every offset out of range
  const __amdgpu_buffer_rsrc_t rc = zrsrc(xc, gc.nn * TS);
  const __amdgpu_buffer_rsrc_t rp = zrsrc(xpre, gf.nn * TS);
  const __amdgpu_buffer_rsrc_t rb = zrsrc(b, gf.nn * TS);
  const __amdgpu_buffer_rsrc_t rk = zrsrc(k.p, gf.ne * ES);
  const int Ib = (i >> 1) - 1, Jb = (j >> 1) - 1, Kb = DIM == 3 ? (kz >> 1) - 1 : 0;
  T cv[NZ][3][3];
#pragma unroll
  for (int c = 0; c < NZ; ++c)
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
      for (int a = 0; a < 3; ++a)
        cv[c][bb][a] = zbload<T>(rc, node_boff(gc, Ib + a, Jb + bb, DIM == 3 ? Kb + c : 0, TS));
  T kv[2][2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (DIM == 2 && c == 1) { kv[c][bb][a] = T(0); continue; }
        const unsigned o = cell_boff(gf, i - 1 + a, j - 1 + bb, DIM == 3 ? kz - 1 + c : 0, ES);
        const T v = T(k.value(zbload<E>(rk, o)));
        kv[c][bb][a] = CMASK ? v * (o < ZOOB ? T(1) : T(0)) : v;
      }
  const unsigned own = node_boff(gf, i, j, kz, TS);   // ZOOB past the grid (kz >= nnz)
  const T bn = zbload<T>(rb, own);
  // Per axis and fine offset d in {-1, 0, 1}, the fine node i + d interpolates
  // between coarse entries lo and hi of the 3-block: lo + m * hi, weighted w
  // (m = 1, w = 1/2 on odd fine indices, else m = 0, w = 1). Only lo depends on
  // the parity of i (a select between two registers); every array index is a
  // compile-time constant, so the block stays in registers.
  const int px = i & 1, py = j & 1, pz = DIM == 3 ? (kz & 1) : 0;
  const T fx = T(px), fy = T(py), fz = T(pz);
  // a or b by a 0/1 weight: exact for finite values, and (unlike a select of two
  // array elements, which is compiled into an indexed access) keeps the block in
  // registers
  auto pick = [](T a, T b, T f) __attribute__((always_inline)) { return a * (T(1) - f) + b * f; };
  auto mw = [](int p, int d, T& m, T& w) __attribute__((always_inline)) {
    const int odd = (p + d) & 1;
    m = T(odd);
    w = T(odd ? 0.5 : 1.0);
  };
  // x: X[dx][zz][yy] = cv[zz][yy][lo] + m_x cv[zz][yy][hi]
  T X[3][NZ][3];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) {
    T m, w;
    mw(px, dx - 1, m, w);
    (void)w;
#pragma unroll
    for (int zz = 0; zz < NZ; ++zz)
#pragma unroll
      for (int yy = 0; yy < 3; ++yy) {
        const T* row = cv[zz][yy];
        const T lo = dx == 0 ? pick(row[0], row[1], fx) : dx == 1 ? row[1] : pick(row[1], row[2], fx);
        const T hi = dx == 0 ? row[1] : row[2];
        X[dx][zz][yy] = lo + m * hi;
      }
  }
  // y: Y[dx][dy][zz] = w_x X[dx][zz][lo] + m_y (w_x X[dx][zz][hi])
  T Y[3][3][NZ];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) {
    T mx, wx;
    mw(px, dx - 1, mx, wx);
    (void)mx;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      T my, wy;
      mw(py, dy - 1, my, wy);
      (void)wy;
#pragma unroll
      for (int zz = 0; zz < NZ; ++zz) {
        const T* col = X[dx][zz];
        const T lo = dy == 0 ? pick(col[0], col[1], fy) : dy == 1 ? col[1] : pick(col[1], col[2], fy);
        const T hi = dy == 0 ? col[1] : col[2];
        Y[dx][dy][zz] = wx * lo + my * (wx * hi);
      }
    }
  }
  // z, and the interpolated iterate at fine node (i + dx - 1, j + dy - 1, kz + dz - 1)
  auto xa_at = [&](int dx, int dy, int dz) __attribute__((always_inline)) -> T {
    const int ii = i + dx - 1, jj = j + dy - 1, kk = DIM == 3 ? kz + dz - 1 : kz;
    const unsigned o = node_boff(gf, ii, jj, kk, TS);
    const T xo = zbload<T>(rp, o);
    T my, wy, mz, wz;
    mw(py, dy - 1, my, wy);
    (void)my;
    if (DIM == 3) mw(pz, dz - 1, mz, wz);
    else { mz = T(0); wz = T(1); }
    const T* zc = Y[dx][dy];
    T lo, hi;
    if (DIM == 3) {
      lo = dz == 0 ? pick(zc[0], zc[1], fz) : dz == 1 ? zc[1] : pick(zc[1], zc[NZ - 1], fz);
      hi = dz == 0 ? zc[1] : zc[NZ - 1];
    } else {
      lo = zc[0];
      hi = zc[0];
    }
    const T s = wy * lo + mz * (wy * hi);
    const bool in = o < ZOOB, fixed = geo_fixed(gf, ii, jj, kk);
    const T xa = fixed ? xo : xo + wz * s;
    return xa * (in ? T(1) : T(0));
  };
  T y, ksum, xn;
  if (DIM == 2) {
    T xv[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) xv[dy][dx] = xa_at(dx, dy, 1);
    xn = xv[1][1];
    T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int sx = a ? 2 : 0, sy = bb ? 2 : 0;
        const T ke = kv[0][bb][a];
        s0 += ke;
        s1 += ke * (xv[1][sx] + xv[sy][1]);
        s2 += ke * xv[sy][sx];
      }
    ksum = s0;
    y = T(2.0 / 3.0) * s0 * xv[1][1] - T(1.0 / 6.0) * s1 - T(1.0 / 3.0) * s2;
  } else {
    T xv[3][3][3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int nzr = (dx != 1) + (dy != 1) + (dz != 1);
          xv[dz][dy][dx] = (nzr == 1) ? T(0) : xa_at(dx, dy, dz);   // face neighbours: weight 0
        }
    xn = xv[1][1][1];
    y = apply27<T, true>(xv[0], xv[1], xv[2], kv[0], kv[1], T(gf.h * (1.0 / 3.0)), T(gf.h * (1.0 / 12.0)), ksum);
  }
  const T diag = T(DIM == 3 ? gf.h * (1.0 / 3.0) : (2.0 / 3.0)) * ksum;
  T r = xn + omega * (bn - y) / diag;
  r = geo_fixed(gf, i, j, kz) ? T(0) : r;
  zbstore(r, zrsrc(out, gf.nn * TS), own);
}

// Coarse conductivity: mean of the 2^d children.
template <int DIM, typename CL, typename TO>
__global__ void k_coarsen(Geo gf, Geo gc, CL kf, TO* __restrict__ kc) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= gc.ne) return;
  const int ex = (int)(e % gc.nx);
  const long long r = e / gc.nx;
  const int ey = (int)(r % gc.ny);
  const int ez = (int)(r / gc.ny);
  double s = 0.0;
  for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        s += (double)kf(geo_elem(gf, 2 * ex + a, 2 * ey + b, DIM == 3 ? 2 * ez + c : 0));
  kc[e] = (TO)(s * (DIM == 3 ? 0.125 : 0.25));
}

// Q1 element matrix entry between local corners ca, cb for cell edge h.
template <int DIM>
__device__ inline double ke_entry(int ca, int cb, double h) {
  const int hd = __popc(ca ^ cb);
  if (DIM == 2) return hd == 0 ? 2.0 / 3.0 : (hd == 1 ? -1.0 / 6.0 : -1.0 / 3.0);
  return h * (hd == 0 ? 1.0 / 3.0 : (hd == 1 ? 0.0 : -1.0 / 12.0));
}

constexpr int CB_THREADS = 1024;
constexpr int CB_MAXN = 1024;
constexpr int CB_KCAP = 1024;   // cells of a coarsest grid of at most 128 nodes

constexpr int CB_NB = 16;   // pivot block of the blocked elimination

// Coarsest grid: assemble the dense N_c x N_c matrix (identity rows/columns on
// Dirichlet nodes), then invert it in place by block Gauss-Jordan elimination
// without pivoting (valid for SPD matrices: every pivot block is SPD) and
// symmetrise. One workgroup. Block step with pivot block D = A_kk (rows and
// columns kb .. kb + kw):
//   D^-1 by scalar Gauss-Jordan in LDS,
//   A_kj <- D^-1 A_kj (j != k), A_kk <- D^-1          (P = the new block row, kept in LDS),
//   A_ij <- A_ij - A_ik P_kj (i, j != k),
//   A_ik <- -A_ik D^-1 (i != k).
// Each step reads and writes every entry of A once (the unblocked form does so
// once per pivot), so the matrix in global memory is swept n / 16 times.
template <int DIM, typename CL>
__device__ inline void coarse_build_body(const Geo& g, CL k, double* __restrict__ A,
                                         int* __restrict__ status) {
  __shared__ double P[CB_NB * CB_MAXN];
  __shared__ double D[CB_NB][CB_NB + 1];
  const int n = (int)g.nn;
  const int t = threadIdx.x;
  for (long long idx = t; idx < (long long)n * n; idx += CB_THREADS) A[idx] = 0.0;
  __syncthreads();
  for (int i = t; i < n; i += CB_THREADS) {
    const int ii = i % g.nnx, jj = (i / g.nnx) % g.nny, kk = i / (g.nnx * g.nny);
    if (geo_fixed(g, ii, jj, kk)) {
      A[(long long)i * n + i] = 1.0;
      continue;
    }
    for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int ex = ii - 1 + a, ey = jj - 1 + b, ez = (DIM == 3) ? kk - 1 + c : 0;
          if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny || ez < 0 || ez >= g.nz) continue;
          const double ke = (double)k(geo_elem(g, ex, ey, ez));
          // corner of node i in this cell
          const int ci = (1 - a) + 2 * (1 - b) + (DIM == 3 ? 4 * (1 - c) : 0);
          for (int cc = 0; cc < (DIM == 3 ? 8 : 4); ++cc) {
            const int ni = ex + (cc & 1), nj = ey + ((cc >> 1) & 1),
                      nk = (DIM == 3) ? ez + ((cc >> 2) & 1) : 0;
            if (geo_fixed(g, ni, nj, nk)) continue;
            A[(long long)i * n + geo_node(g, ni, nj, nk)] += ke * ke_entry<DIM>(ci, cc, g.h);
          }
        }
  }
  __syncthreads();
  int bad = 0;
  const int dr = t / CB_NB, dc = t % CB_NB;   // threads t < CB_NB^2: one entry of D each
  const int njt = (n + 3) / 4;                 // 4 x 4 tiles of the trailing update
  for (int kb = 0; kb < n; kb += CB_NB) {
    const int kw = min(CB_NB, n - kb);
    // D^-1 (entries past kw: identity, untouched by the steps below)
    if (t < CB_NB * CB_NB)
      D[dr][dc] = (dr < kw && dc < kw) ? A[(long long)(kb + dr) * n + kb + dc] : (dr == dc ? 1.0 : 0.0);
    __syncthreads();
    for (int p = 0; p < kw; ++p) {
      double piv = 1.0, rp = 0.0, cp = 0.0, old = 0.0;
      if (t < CB_NB * CB_NB) {
        piv = D[p][p];
        rp = D[p][dc];
        cp = D[dr][p];
        old = D[dr][dc];
      }
      __syncthreads();
      if (!(piv > 0.0)) bad = 1;
      if (t < CB_NB * CB_NB && dr < kw && dc < kw) {
        const double inv = 1.0 / piv;
        double v;
        if (dr == p && dc == p) v = inv;
        else if (dr == p) v = rp * inv;
        else if (dc == p) v = -cp * inv;
        else v = old - cp * rp * inv;
        D[dr][dc] = v;
      }
      __syncthreads();
    }
    // P = D^-1 A_k* (block columns k: D^-1), written to LDS and to rows kb.. of A;
    // column j is read and written by one thread only
    for (int j = t; j < n; j += CB_THREADS) {
      if (j >= kb && j < kb + kw) {
        for (int r = 0; r < kw; ++r) {
          const double v = D[r][j - kb];
          P[r * n + j] = v;
          A[(long long)(kb + r) * n + j] = v;
        }
      } else {
        double a[CB_NB];
#pragma unroll
        for (int c = 0; c < CB_NB; ++c) a[c] = (c < kw) ? A[(long long)(kb + c) * n + j] : 0.0;
        for (int r = 0; r < kw; ++r) {
          double v = 0.0;
#pragma unroll
          for (int c = 0; c < CB_NB; ++c) v += D[r][c] * a[c];
          P[r * n + j] = v;
          A[(long long)(kb + r) * n + j] = v;
        }
      }
    }
    __syncthreads();
    // A_ij -= A_ik P_kj for rows and columns outside block k (A_ik not written
    // in this pass), 4 x 4 tiles per thread
    for (int q = t; q < njt * njt; q += CB_THREADS) {
      const int i0 = (q / njt) * 4, j0 = (q % njt) * 4;
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      // unrolled by 2 so that two columns' loads of a tile are in flight
      // together (entries past kw contribute 0)
#pragma unroll 2
      for (int c = 0; c < CB_NB; ++c) {
        double ci[4], pj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          ci[a] = (c < kw && i0 + a < n) ? A[(long long)(i0 + a) * n + kb + c] : 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) pj[b] = (c < kw && j0 + b < n) ? P[c * n + j0 + b] : 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += ci[a] * pj[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int i = i0 + a;
        if (i >= n || (i >= kb && i < kb + kw)) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int j = j0 + b;
          if (j >= n || (j >= kb && j < kb + kw)) continue;
          A[(long long)i * n + j] -= acc[a][b];
        }
      }
    }
    __syncthreads();
    // A_ik <- -A_ik D^-1 for rows outside block k (one thread per row)
    for (int i = t; i < n; i += CB_THREADS) {
      if (i >= kb && i < kb + kw) continue;
      double a[CB_NB];
#pragma unroll
      for (int c = 0; c < CB_NB; ++c) a[c] = (c < kw) ? A[(long long)i * n + kb + c] : 0.0;
      for (int r = 0; r < kw; ++r) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < CB_NB; ++c) v += a[c] * D[c][r];
        A[(long long)i * n + kb + r] = -v;
      }
    }
    __syncthreads();
  }
  // symmetrise
  const int tc = t & 31, tr = t >> 5;
  for (int i = tr; i < n; i += CB_THREADS / 32)
    for (int j = tc; j < n; j += 32)
      if (j > i) {
        const double v = 0.5 * (A[(long long)i * n + j] + A[(long long)j * n + i]);
        A[(long long)i * n + j] = v;
        A[(long long)j * n + i] = v;
      }
  if (t == 0 && bad) status[0] = 1;
}

template <int DIM, typename CL>
__global__ __launch_bounds__(CB_THREADS) void k_coarse_build(Geo g, CL k, double* __restrict__ A,
                                                             int* __restrict__ status) {
  coarse_build_body<DIM, CL>(g, k, A, status);
}

// Register-resident variant for n <= 128: thread (tr, tc) of a 32 x 32 layout
// owns entries (tr + 32a, tc + 32b), a, b < 4, for the whole elimination; only
// the pivot row and column pass through LDS. Unblocked (scalar) Gauss-Jordan:
// one pivot per step.
template <int DIM, typename CL>
__device__ inline void coarse_build_reg_body(const Geo& g, CL k, double* __restrict__ A,
                                             int* __restrict__ status) {
  __shared__ double colp[2][128];   // pivot column / row, double-buffered by step parity
  __shared__ double rowp[2][128];
  __shared__ double kc[CB_KCAP];
  const int n = (int)g.nn;
  const int t = threadIdx.x;
  const int tc = t & 31, tr = t >> 5;
  // cell conductivities staged in LDS once (the assembly reads each many times)
  for (int e = t; e < (int)g.ne; e += CB_THREADS) kc[e] = (double)k(e);
  __syncthreads();
  // Entry (i, j) straight from the element sum: the cells shared by nodes i
  // and j, each adding k_e KE[c_i][c_j]; identity rows/columns on Dirichlet
  // nodes. No memory round trips.
  int ci3[4][3], cj3[4][3];
  bool fi[4], fj[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = min(tr + 32 * a, n - 1), j = min(tc + 32 * a, n - 1);
    ci3[a][0] = i % g.nnx; ci3[a][1] = (i / g.nnx) % g.nny; ci3[a][2] = i / (g.nnx * g.nny);
    cj3[a][0] = j % g.nnx; cj3[a][1] = (j / g.nnx) % g.nny; cj3[a][2] = j / (g.nnx * g.nny);
    fi[a] = geo_fixed(g, ci3[a][0], ci3[a][1], ci3[a][2]);
    fj[a] = geo_fixed(g, cj3[a][0], cj3[a][1], cj3[a][2]);
  }
  double R[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = tr + 32 * a, j = tc + 32 * b;
      double v = 0.0;
      if (i < n && j < n) {
        if (fi[a] || fj[b]) {
          v = (i == j) ? 1.0 : 0.0;
        } else {
          const int dx = cj3[b][0] - ci3[a][0], dy = cj3[b][1] - ci3[a][1], dz = cj3[b][2] - ci3[a][2];
          if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) {
            for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
              for (int bb = 0; bb < 2; ++bb)
                for (int aa = 0; aa < 2; ++aa) {
                  const int ex = ci3[a][0] - 1 + aa, ey = ci3[a][1] - 1 + bb,
                            ez = (DIM == 3) ? ci3[a][2] - 1 + c : 0;
                  if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny || ez < 0 || ez >= g.nz) continue;
                  // j must be a corner of this cell
                  const int bx = cj3[b][0] - ex, by = cj3[b][1] - ey, bz = (DIM == 3) ? cj3[b][2] - ez : 0;
                  if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                  const int cci = (1 - aa) + 2 * (1 - bb) + (DIM == 3 ? 4 * (1 - c) : 0);
                  const int ccj = bx + 2 * by + 4 * bz;
                  v += kc[geo_elem(g, ex, ey, ez)] * ke_entry<DIM>(cci, ccj, g.h);
                }
          }
        }
      }
      R[a][b] = v;
    }
  // Elimination: the slot pa of the pivot is a compile-time index (outer loop
  // unrolled), so the register tile is never indexed at run time. Entries past
  // n are 0 and stay 0. Step p
  // publishes its pivot row and column in buffer p & 1: the barrier of step
  // p + 1 orders the reads of step p before the writes of step p + 2, so one
  // barrier per step suffices.
  int bad = 0;
#pragma unroll
  for (int pa = 0; pa < 4; ++pa) {
    for (int pr = 0; pr < 32; ++pr) {
      const int p = pa * 32 + pr;
      if (p >= n) break;
      double* rowb = rowp[p & 1];
      double* colb = colp[p & 1];
      if (tr == pr) {
#pragma unroll
        for (int b = 0; b < 4; ++b) rowb[tc + 32 * b] = R[pa][b];
      }
      if (tc == pr) {
#pragma unroll
        for (int a = 0; a < 4; ++a) colb[tr + 32 * a] = R[a][pa];
      }
      __syncthreads();
      const double piv = rowb[p];
      if (!(piv > 0.0)) bad = 1;
      const double inv = 1.0 / piv;
      double rj[4], ci[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) rj[b] = rowb[tc + 32 * b] * inv;
#pragma unroll
      for (int a = 0; a < 4; ++a) ci[a] = colb[tr + 32 * a];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) R[a][b] -= ci[a] * rj[b];
      // pivot row: a_pj / a_pp, a_pp -> 1 / a_pp; pivot column: -a_ip / a_pp
      if (tr == pr) {
#pragma unroll
        for (int b = 0; b < 4; ++b) R[pa][b] = (tc + 32 * b == p) ? inv : rj[b];
      }
      if (tc == pr) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
          if (tr + 32 * a != p) R[a][pa] = -ci[a] * inv;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = tr + 32 * a, j = tc + 32 * b;
      if (i < n && j < n) A[i * n + j] = R[a][b];
    }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = tr + 32 * a, j = tc + 32 * b;
      if (i < n && j < n && j > i) {
        const double v = 0.5 * (A[i * n + j] + A[j * n + i]);
        A[i * n + j] = v;
        A[j * n + i] = v;
      }
    }
  if (t == 0 && bad) status[0] = 1;
}

template <int DIM, typename CL>
__global__ __launch_bounds__(CB_THREADS) void k_coarse_build_reg(Geo g, CL k, double* __restrict__ A,
                                                                 int* __restrict__ status) {
  coarse_build_reg_body<DIM, CL>(g, k, A, status);
}

// x = A^-1 b on the coarsest grid (A symmetric: column reads are coalesced).
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(int n, const double* __restrict__ A,
                                                      const T* __restrict__ b, T* __restrict__ x,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += A[(long long)j * n + i] * (double)b[j];
  x[i] = (T)s;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(TBX* TBY) void k_mask_copy(Geo g, const TI* __restrict__ in,
                                                        TO* __restrict__ out) {
  const int i = blockIdx.x * TBX + threadIdx.x;
  const int j = blockIdx.y * TBY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nnx || j >= g.nny) return;
  const long long n = geo_node(g, i, j, k);
  out[n] = geo_fixed(g, i, j, k) ? TO(0) : (TO)in[n];
}

// ---------------------------------------------------------------------------
// V-cycle tail: one workgroup runs the down-sweep, the coarsest solve and the
// up-sweep of the bottom grids, exchanging data through LDS between steps
// (barriers instead of kernel boundaries). Node loops are strided over the
// 1024 threads; node coordinates are recovered by division (small grids).
constexpr int TT = 1024;

__device__ inline void tnode_ijk(const Geo& g, int n, int& i, int& j, int& k) {
  const int pl = g.nnx * g.nny;
  k = n / pl;
  const int r = n - k * pl;
  j = r / g.nnx;
  i = r - j * g.nnx;
}

// LDS layout of the tail: every grid but the coarsest keeps its node vectors
// and cells with a one-entry halo of zeros on each side, so a neighbour or a
// cell is one indexed read with no bounds test; the coarsest grid (solved
// through its inverse, which is indexed by node number) is unpadded.
struct TPad {
  int sx, sxy;     // node strides of the padded layout
  int cx, cxy;     // cell strides
};
template <int DIM>
__device__ inline TPad tpad(const Geo& g) {
  TPad p;
  p.sx = g.nnx + 2;
  p.sxy = p.sx * (g.nny + 2);
  p.cx = g.nx + 2;
  p.cxy = p.cx * (g.ny + 2);
  return p;
}
template <int DIM>
__device__ inline int pnode(const TPad& p, int i, int j, int k) {
  return (i + 1) + p.sx * (j + 1) + (DIM == 3 ? p.sxy * (k + 1) : 0);
}
template <int DIM>
__device__ inline int pcell(const TPad& p, int ex, int ey, int ez) {
  return (ex + 1) + p.cx * (ey + 1) + (DIM == 3 ? p.cxy * (ez + 1) : 0);
}

template <int DIM, int MODE, typename T>
__device__ void tail_stencil(const Geo& g, const T* x, const T* k, const T* b, T* out, T omega) {
  const TPad pd = tpad<DIM>(g);
  for (int n = threadIdx.x; n < (int)g.nn; n += TT) {
    int i, j, kz;
    tnode_ijk(g, n, i, j, kz);
    const int P = pnode<DIM>(pd, i, j, kz);
    T r = T(0);
    if (!geo_fixed(g, i, j, kz)) {
      T kv[2][2][2];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
          for (int a = 0; a < 2; ++a)
            kv[c][bb][a] = (DIM == 2 && c == 1) ? T(0) : k[pcell<DIM>(pd, i - 1 + a, j - 1 + bb, kz - 1 + c)];
      T ks = T(0), y = T(0);
      if (MODE == SM_JACOBI0) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int a = 0; a < 2; ++a) ks += kv[c][bb][a];
      } else if (DIM == 2) {
        T xv[3][3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) xv[dy][dx] = x[P + (dx - 1) + pd.sx * (dy - 1)];
        T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int sx = a ? 2 : 0, sy = bb ? 2 : 0;
            const T ke = kv[0][bb][a];
            s0 += ke;
            s1 += ke * (xv[1][sx] + xv[sy][1]);
            s2 += ke * xv[sy][sx];
          }
        ks = s0;
        y = T(2.0 / 3.0) * s0 * xv[1][1] - T(1.0 / 6.0) * s1 - T(1.0 / 3.0) * s2;
      } else {
        T xv[3][3][3];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
              const int nzr = (dx != 1) + (dy != 1) + (dz != 1);
              xv[dz][dy][dx] = (nzr == 1) ? T(0) : x[P + (dx - 1) + pd.sx * (dy - 1) + pd.sxy * (dz - 1)];
            }
        y = apply27<T, true>(xv[0], xv[1], xv[2], kv[0], kv[1], T(g.h * (1.0 / 3.0)), T(g.h * (1.0 / 12.0)), ks);
      }
      const T diag = T(DIM == 3 ? g.h * (1.0 / 3.0) : (2.0 / 3.0)) * ks;
      if (MODE == SM_JACOBI0) r = omega * b[P] / diag;
      else if (MODE == SM_RESID) r = b[P] - y;
      else r = x[P] + omega * (b[P] - y) / diag;   // SM_JACOBI
    }
    out[P] = r;
  }
}

// rc = P^T rf; rf padded, rc padded unless cpad is false (the coarsest grid)
template <int DIM, typename T>
__device__ void tail_restrict(const Geo& gf, const Geo& gc, const T* rf, T* rc, bool cpad) {
  const TPad pf = tpad<DIM>(gf), pc = tpad<DIM>(gc);
  for (int n = threadIdx.x; n < (int)gc.nn; n += TT) {
    int I, J, K;
    tnode_ijk(gc, n, I, J, K);
    T s = T(0);
    if (!geo_fixed(gc, I, J, K)) {
#pragma unroll
      for (int c = (DIM == 3 ? -1 : 0); c <= (DIM == 3 ? 1 : 0); ++c) {
        T sy = T(0);
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb) {
          T sx = T(0);
#pragma unroll
          for (int a = -1; a <= 1; ++a)
            sx += T(a == 0 ? 1.0 : 0.5) * rf[pnode<DIM>(pf, 2 * I + a, 2 * J + bb, 2 * K + c)];
          sy += T(bb == 0 ? 1.0 : 0.5) * sx;
        }
        s += T(c == 0 ? 1.0 : 0.5) * sy;
      }
    }
    rc[cpad ? pnode<DIM>(pc, I, J, K) : n] = s;
  }
}

// xf += P xc on free fine nodes; xf padded, xc padded unless cpad is false
template <int DIM, typename T>
__device__ void tail_prolong(const Geo& gf, const Geo& gc, const T* xc, T* xf, bool cpad) {
  const TPad pf = tpad<DIM>(gf), pc = tpad<DIM>(gc);
  for (int n = threadIdx.x; n < (int)gf.nn; n += TT) {
    int i, j, k;
    tnode_ijk(gf, n, i, j, k);
    if (geo_fixed(gf, i, j, k)) continue;
    const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (DIM == 3 && (k & 1)) ? 2 : 1;
    const T wi = T((i & 1) ? 0.5 : 1.0), wj = T((j & 1) ? 0.5 : 1.0),
            wk = T((DIM == 3 && (k & 1)) ? 0.5 : 1.0);
    // the 2^d coarse corners, the upper ones weighted 0 on even fine indices
    // (their indices stay in the grid): no branch around the loads
    const T mi = T(ni - 1), mj = T(nj - 1), mk = T(nk - 1);
    const int I1 = I0 + ni - 1, J1 = J0 + nj - 1, K1 = K0 + nk - 1;
    auto cv = [&](int a, int b, int c) -> T {
      return xc[cpad ? pnode<DIM>(pc, a, b, c) : a + gc.nnx * (b + gc.nny * c)];
    };
    T sc[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int kc = c ? K1 : K0;
      const T sx0 = cv(I0, J0, kc) + mi * cv(I1, J0, kc);
      const T sx1 = cv(I0, J1, kc) + mi * cv(I1, J1, kc);
      sc[c] = wi * sx0 + mj * (wi * sx1);
    }
    const T s = wj * sc[0] + mk * (wj * sc[1]);
    xf[pnode<DIM>(pf, i, j, k)] += wk * s;
  }
}

// x = A^-1 b with A symmetric (n <= 1024): `tpr` threads per row, each summing
// a strided share of the columns (in column order), combined by a wave shuffle
// tree. For n <= 128 a thread's share is at most CPRE columns, which it loads
// into registers at the start of the tail (CoarsePre), so the global-memory
// latency of A overlaps the down-sweep instead of following it.
constexpr int CPRE = 16;
struct CoarsePre {
  int n, tpr, row, sub;
  double a[CPRE];
};

__device__ inline void tail_coarse_prefetch(int n, const double* __restrict__ A, CoarsePre& P) {
  int tpr = 1;
  while (tpr * 2 * n <= TT && tpr < 64) tpr *= 2;
  P.n = n;
  P.tpr = tpr;
  P.row = threadIdx.x / tpr;
  P.sub = threadIdx.x % tpr;
  if (n > 128) return;
  const int rc = min(P.row, n - 1);
#pragma unroll
  for (int u = 0; u < CPRE; ++u) {
    const int jj = P.sub + u * tpr, jc = min(jj, n - 1);
    P.a[u] = A[(long long)jc * n + rc];   // clamped: in range; columns past n get weight 0 below
  }
}

template <typename T>
__device__ void tail_coarse(const CoarsePre& P, const double* __restrict__ A, const T* b, T* x) {
  const int n = P.n, tpr = P.tpr, row = P.row, sub = P.sub;
  double s = 0.0;
  if (row < n) {
    if (n <= 128) {
#pragma unroll
      for (int u = 0; u < CPRE; ++u) {
        const int jj = sub + u * tpr, jc = min(jj, n - 1);
        s += P.a[u] * ((double)b[jc] * (jj < n ? 1.0 : 0.0));
      }
    } else {
      for (int jj = sub; jj < n; jj += tpr) s += A[(long long)jj * n + row] * (double)b[jj];
    }
  }
  for (int o = tpr / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, MGAR_WAVE);
  if (row < n && sub == 0) x[row] = (T)s;
}

template <int DIM, typename T>
__device__ inline void vtail_body(const TailSpec& TS, const T* __restrict__ bin, T* __restrict__ xout,
                                  const double* __restrict__ Ainv, T omega) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int nl = TS.nl;
  // halos (and everything else) start at 0
  for (int e = threadIdx.x; e < TS.lds_elems; e += TT) lds[e] = T(0);
  __syncthreads();
  for (int l = 0; l + 1 < nl; ++l) {
    const Geo& g = TS.g[l];
    const TPad pd = tpad<DIM>(g);
    const T* kg = static_cast<const T*>(TS.k[l]);
    for (int e = threadIdx.x; e < (int)g.ne; e += TT) {
      const int ex = e % g.nx, r = e / g.nx, ey = r % g.ny, ez = r / g.ny;
      lds[TS.off_k[l] + pcell<DIM>(pd, ex, ey, ez)] = kg[e];
    }
  }
  {
    const Geo& g = TS.g[0];
    const TPad pd = tpad<DIM>(g);
    for (int n = threadIdx.x; n < (int)g.nn; n += TT) {
      int i, j, k;
      tnode_ijk(g, n, i, j, k);
      lds[TS.off_b[0] + (nl > 1 ? pnode<DIM>(pd, i, j, k) : n)] = bin[n];
    }
  }
  // issued after the loads above, so waiting for those does not wait for these
  CoarsePre cp;
  tail_coarse_prefetch((int)TS.g[nl - 1].nn, Ainv, cp);
  __syncthreads();
  for (int l = 0; l + 1 < nl; ++l) {
    const Geo& g = TS.g[l];
    T* b = lds + TS.off_b[l];
    T* xa = lds + TS.off_xa[l];
    T* xb = lds + TS.off_xb[l];
    const T* kk = lds + TS.off_k[l];
    tail_stencil<DIM, SM_JACOBI0, T>(g, nullptr, kk, b, xa, omega);
    __syncthreads();
    tail_stencil<DIM, SM_RESID, T>(g, xa, kk, b, xb, omega);
    __syncthreads();
    tail_restrict<DIM, T>(g, TS.g[l + 1], xb, lds + TS.off_b[l + 1], l + 2 < nl);
    __syncthreads();
  }
  tail_coarse(cp, Ainv, lds + TS.off_b[nl - 1], lds + TS.off_xa[nl - 1]);
  __syncthreads();
  const T* xfin = lds + TS.off_xa[nl - 1];
  for (int l = nl - 2; l >= 0; --l) {
    const Geo& g = TS.g[l];
    T* xa = lds + TS.off_xa[l];
    T* xb = lds + TS.off_xb[l];
    tail_prolong<DIM, T>(g, TS.g[l + 1], xfin, xa, l + 2 < nl);
    __syncthreads();
    tail_stencil<DIM, SM_JACOBI, T>(g, xa, lds + TS.off_k[l], lds + TS.off_b[l], xb, omega);
    __syncthreads();
    xfin = xb;
  }
  {
    const Geo& g = TS.g[0];
    const TPad pd = tpad<DIM>(g);
    for (int n = threadIdx.x; n < (int)g.nn; n += TT) {
      int i, j, k;
      tnode_ijk(g, n, i, j, k);
      xout[n] = xfin[nl > 1 ? pnode<DIM>(pd, i, j, k) : n];
    }
  }
}

template <int DIM, typename T>
__global__ __launch_bounds__(TT) void k_vtail(TailSpec TS, const T* __restrict__ bin,
                                              T* __restrict__ xout,
                                              const double* __restrict__ Ainv, T omega,
                                              const int* __restrict__ done) {
  if (done && *done) return;
  vtail_body<DIM, T>(TS, bin, xout, Ainv, omega);
}

dim3 node_grid(const Geo& g) {
  return dim3((g.nnx + TBX - 1) / TBX, (g.nny + TBY - 1) / TBY, g.nnz);
}
// flat launch of the buffer kernels: one thread per node
dim3 flat_grid(const Geo& g) { return dim3((unsigned)((g.nn + TBX * TBY - 1) / (TBX * TBY))); }

// Buffer kernels need every array of the grid below 2 GiB (32-bit offsets).
bool grid_fits_buffers(const Geo& g) { return g.nn * 8 < (1LL << 31) && g.ne * 8 < (1LL << 31); }

template <int DIM, typename T, typename CL>
void stencil_dispatch(const Geo& g, int mode, const T* x, CL k, CL kref, const T* b, T* out, T omega,
                      double* part, const int* done, unsigned* cnt, double* rout, hipStream_t s,
                      hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 grid = node_grid(g), fgrid = flat_grid(g), blk(TBX, TBY, 1);
  const bool buf = grid_fits_buffers(g);
  // with events: launched through hipExtLaunchKernelGGL, which records them at
  // the start and end of the kernel itself
#define SCALL(M)                                                                                   \
  do {                                                                                             \
    if (buf)                                                                                       \
      hipExtLaunchKernelGGL((k_stencil_b<DIM, M, T, CL>), fgrid, blk, 0, s, ev0, ev1, 0, g, x, k, kref, b, \
                            out, omega, part, done, cnt, rout);                                    \
    else                                                                                           \
      hipExtLaunchKernelGGL((k_stencil<DIM, M, T, CL>), grid, blk, 0, s, ev0, ev1, 0, g, x, k, kref, b, \
                            out, omega, part, done, cnt, rout);                                    \
  } while (0)
  switch (mode) {
    case SM_APPLY: SCALL(SM_APPLY); break;
    case SM_APPLY_DOT: SCALL(SM_APPLY_DOT); break;
    case SM_RESID: SCALL(SM_RESID); break;
    case SM_JACOBI: SCALL(SM_JACOBI); break;
    case SM_JACOBI_DOT: SCALL(SM_JACOBI_DOT); break;
    case SM_JACOBI0: SCALL(SM_JACOBI0); break;
    case SM_NEG_DK: SCALL(SM_NEG_DK); break;
  }
#undef SCALL
}

constexpr int ZMARCH_MIN_NODES = 20000;
constexpr int ZKZ = 16;   // default z-planes per block (with a two-plane load queue)

struct ZShape { int TXW, TYH, ntx, nty, nzc; };

ZShape zmarch_shape(const Geo& g, const StencilCfg& c) {
  ZShape z;
  z.ntx = c.ntx;
  z.TXW = (g.nnx + z.ntx - 1) / z.ntx;
  int tyh = ZT / z.TXW;
  tyh = std::min(tyh, XCAP / (z.TXW + 2) - 2);
  tyh = std::min(tyh, CCAP / (z.TXW + 1) - 1);
  z.TYH = std::max(tyh, 1);
  if (c.kind == 2) {   // two rows per thread: an even tile height
    tyh = 2 * (ZT / z.TXW);
    tyh = std::min(tyh, XCAP2 / (z.TXW + 2) - 2);
    tyh = std::min(tyh, CCAP2 / (z.TXW + 1) - 1);
    z.TYH = std::max(tyh & ~1, 2);
  }
  z.nty = (g.nny + z.TYH - 1) / z.TYH;
  z.nzc = (g.nnz + c.kz - 1) / c.kz;
  return z;
}

template <int M, int ZD, bool TWO, typename T, typename CL>
constexpr auto zmarch_kernel() {
  if constexpr (TWO) return &k_stencil_z2<M, ZD, T, CL>;
  else return &k_stencil_z<M, ZD, T, CL>;
}

template <int ZD, bool TWO, typename T, typename CL>
void zmarch_launch(const Geo& g, const ZShape& z, int kz, int mode, const T* x, CL k, CL kref,
                   const T* b, T* out, T omega, double* part, const int* done, unsigned* cnt,
                   double* rout, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, const PFuse& fu = PFuse{}) {
  const int nb = z.ntx * z.nty * z.nzc;
  // With events, the launch goes through hipExtLaunchKernelGGL, which records
  // them at the start and end of the kernel itself (no dispatch latency).
#define ZKER(M) (zmarch_kernel<M, ZD, TWO, T, CL>())
#define ZCALL(M)                                                                                 \
  do {                                                                                           \
    if (ev0)                                                                                     \
      hipExtLaunchKernelGGL(ZKER(M), dim3(nb), dim3(ZT), 0, s, ev0, ev1, 0, g, z.TXW, z.TYH,     \
                            z.ntx, z.nty, kz, x, k, kref, b, out, omega, part, done, cnt, rout, fu); \
    else                                                                                         \
      hipLaunchKernelGGL(ZKER(M), dim3(nb), dim3(ZT), 0, s, g, z.TXW, z.TYH, z.ntx, z.nty, kz, x, \
                         k, kref, b, out, omega, part, done, cnt, rout, fu);                     \
  } while (0)
  switch (mode) {
    case SM_APPLY: ZCALL(SM_APPLY); break;
    case SM_APPLY_DOT: ZCALL(SM_APPLY_DOT); break;
    case SM_RESID: ZCALL(SM_RESID); break;
    case SM_JACOBI: ZCALL(SM_JACOBI); break;
    case SM_JACOBI_DOT: ZCALL(SM_JACOBI_DOT); break;
    case SM_JACOBI0: ZCALL(SM_JACOBI0); break;
    case SM_NEG_DK: ZCALL(SM_NEG_DK); break;
    case SM_PAPPLY_DOT:   // the finest operators of the FP64 and the FP32 solver
      if constexpr (TWO && (std::is_same_v<CL, CellD> || std::is_same_v<CL, CellF>)) ZCALL(SM_PAPPLY_DOT);
      break;
    case SM_J0RESID:   // finest V-cycle grids; one queue depth: a deeper one exceeds 256 VGPRs
      if constexpr (TWO && ZD == 1 && (std::is_same_v<CL, CellD> || std::is_same_v<CL, CellB>))
        ZCALL(SM_J0RESID);
      break;
  }
#undef ZCALL
#undef ZKER
}

// ---------------------------------------------------------------------------
// Batched launches over several designs (FP64). Each block finds its work item
// by bisection over the items' first blocks and runs the same per-node code as
// the single-grid buffer kernels on that item's grid and arrays.
__device__ inline int bitem_find(const BItem* __restrict__ items, int nit, int blk) {
  int lo = 0, hi = nit - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ inline bool bskip(const int* skip, int sstride, int design) {
  return skip && skip[(long long)design * sstride] != 0;
}

// A cell loader moved to a design's cells (element offset eoff).
template <typename CL>
__device__ inline CL cl_at(CL c, long long eoff) {
  c.p += eoff;
  return c;
}

template <int DIM, int MODE, typename T, typename CL>
__global__ __launch_bounds__(TBX* TBY) void kb_stencil(const BItem* __restrict__ items, int nit,
                                                       const T* __restrict__ x, CL k, CL kref,
                                                       const T* __restrict__ b, T* __restrict__ out,
                                                       T omega, double* __restrict__ part,
                                                       const int* __restrict__ skip, int sstride) {
  __shared__ double sh[TBX * TBY / MGAR_WAVE];
  const BItem& it = items[bitem_find(items, nit, blockIdx.x)];
  if (bskip(skip, sstride, it.design)) return;
  const Geo g = it.g;
  const long long n = (long long)(blockIdx.x - it.first) * (blockDim.x * blockDim.y) + flat_tid();
  const double d = stencil_b_point<DIM, MODE, T, CL>(
      g, n, x + it.off, cl_at(k, it.eoff), cl_at(kref.p ? kref : k, it.eoff),
      b ? b + it.off : x + it.off, out + it.off, omega);
  if (MODE == SM_APPLY_DOT || MODE == SM_JACOBI_DOT) {
    const double s = block_sum(d, sh);
    if (flat_tid() == 0) part[blockIdx.x] = s;
  }
}

template <int DIM, typename T>
__global__ __launch_bounds__(TBX* TBY) void kb_restrict(const BItem* __restrict__ items, int nit,
                                                        const T* __restrict__ rf, T* __restrict__ rc,
                                                        const int* __restrict__ skip, int sstride) {
  const BItem& it = items[bitem_find(items, nit, blockIdx.x)];
  if (bskip(skip, sstride, it.design)) return;
  const Geo gf = it.g, gc = it.gc;
  restrict_b_point<DIM, T>(gf, gc, (long long)(blockIdx.x - it.first) * (blockDim.x * blockDim.y) + flat_tid(),
                           rf + it.off, rc + it.coff);
}

template <int DIM, typename T>
__global__ __launch_bounds__(TBX* TBY) void kb_prolong(const BItem* __restrict__ items, int nit,
                                                       const T* __restrict__ xc, T* __restrict__ xf,
                                                       const int* __restrict__ skip, int sstride) {
  const BItem& it = items[bitem_find(items, nit, blockIdx.x)];
  if (bskip(skip, sstride, it.design)) return;
  const Geo gf = it.g, gc = it.gc;
  prolong_b8_point<DIM, T>(gf, gc, (long long)(blockIdx.x - it.first) * (blockDim.x * blockDim.y) + flat_tid(),
                           xc + it.coff, xf + it.off);
}

// coarse cells of item it.gc from fine cells of it.g (one thread per coarse
// cell), summed in the order of k_coarsen
template <int DIM, typename CL, typename TO>
__global__ __launch_bounds__(TBX* TBY) void kb_coarsen(const BItem* __restrict__ items, int nit, CL kf,
                                                       TO* __restrict__ kc, const int* __restrict__ skip,
                                                       int sstride) {
  const BItem& it = items[bitem_find(items, nit, blockIdx.x)];
  if (bskip(skip, sstride, it.design)) return;
  const Geo gf = it.g, gc = it.gc;
  const long long e = (long long)(blockIdx.x - it.first) * (blockDim.x * blockDim.y) + flat_tid();
  if (e >= gc.ne) return;
  const int ex = (int)(e % gc.nx);
  const long long r = e / gc.nx;
  const int ey = (int)(r % gc.ny);
  const int ez = (int)(r / gc.ny);
  const CL f = cl_at(kf, it.eoff);
  using V = decltype(f(0));
  V s = V(0);
  for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
    for (int bb = 0; bb < 2; ++bb)
      for (int a = 0; a < 2; ++a) s += f(geo_elem(gf, 2 * ex + a, 2 * ey + bb, DIM == 3 ? 2 * ez + c : 0));
  kc[it.ceoff + e] = (TO)(s * V(DIM == 3 ? 0.125 : 0.25));
}

template <typename TI, typename TO>
__global__ __launch_bounds__(TBX* TBY) void kb_mask_copy(const BItem* __restrict__ items, int nit,
                                                         const TI* __restrict__ in, TO* __restrict__ out) {
  const BItem& it = items[bitem_find(items, nit, blockIdx.x)];
  const Geo g = it.g;
  const long long n = (long long)(blockIdx.x - it.first) * (blockDim.x * blockDim.y) + flat_tid();
  if (n >= g.nn) return;
  int i, j, k;
  node_ijk(g, n, i, j, k);
  out[it.off + n] = geo_fixed(g, i, j, k) ? TO(0) : (TO)in[it.off + n];
}

template <int DIM, typename T>
__global__ __launch_bounds__(TT) void kb_vtail(const BTail* __restrict__ jobs, double omega,
                                               const int* __restrict__ skip, int sstride) {
  const BTail& jb = jobs[blockIdx.x];
  if (bskip(skip, sstride, jb.design)) return;
  vtail_body<DIM, T>(jb.ts, static_cast<const T*>(jb.bin), static_cast<T*>(jb.xout), jb.A, (T)omega);
}

template <int DIM, bool REG, typename CL>
__global__ __launch_bounds__(CB_THREADS) void kb_coarse_build(const BCoarse* __restrict__ jobs,
                                                              int* __restrict__ status,
                                                              const int* __restrict__ skip,
                                                              int sstride) {
  const BCoarse& jb = jobs[blockIdx.x];
  if (bskip(skip, sstride, jb.design)) return;
  const Geo g = jb.g;
  const CL k{static_cast<const typename CL::E*>(jb.k)};
  if (REG) coarse_build_reg_body<DIM, CL>(g, k, jb.A, status + jb.design);
  else coarse_build_body<DIM, CL>(g, k, jb.A, status + jb.design);
}

}  // namespace

StencilCfg stencil_default_cfg(const Geo& g) {
  StencilCfg c{0, 0, 0, 0};
  if (g.dim == 3 && g.nn >= ZMARCH_MIN_NODES) {
    // two-row z-march with z-chunks sized for about two blocks per CU
    StencilCfg z2{2, 4, 1, (g.nnx + 63) / 64};
    const ZShape s = zmarch_shape(g, z2);
    const long long cols = (long long)s.ntx * s.nty;
    z2.kz = (int)std::min<long long>(16, std::max<long long>(4, (g.nnz * cols + 511) / 512));
    const StencilCfg z{1, ZKZ, 2, (g.nnx + 63) / 64};
    if (stencil_cfg_valid(g, z2)) c = z2;
    else if (stencil_cfg_valid(g, z)) c = z;
  }
  return c;
}

bool stencil_cfg_valid(const Geo& g, const StencilCfg& c) {
  if (c.kind == 0) return true;
  if ((c.kind != 1 && c.kind != 2) || g.dim != 3) return false;
  if (c.kz < 1 || c.kz > 64 || c.zd < 1 || c.zd > (c.kind == 2 ? 2 : 4)) return false;
  if (c.ntx < 1 || c.ntx > g.nnx) return false;
  const int txw = (g.nnx + c.ntx - 1) / c.ntx;
  if (txw > (c.kind == 2 ? 128 : 64) || txw < 4) return false;
  if (g.nn * 8 >= (1LL << 31) || g.ne * 8 >= (1LL << 31)) return false;   // 32-bit buffer offsets
  const ZShape z = zmarch_shape(g, c);
  const long long xn = (long long)(z.TXW + 2) * (z.TYH + 2), cn = (long long)(z.TXW + 1) * (z.TYH + 1);
  if (c.kind == 2)   // whole row pairs; a pair's 4-row window stays inside the staged tile
    return z.TYH % 2 == 0 && xn <= XCAP2 && cn <= CCAP2 && (long long)z.TXW * (z.TYH / 2) <= ZT;
  return xn <= XCAP && cn <= CCAP && (long long)z.TXW * z.TYH <= ZT;
}

int stencil_candidates(const Geo& g, StencilCfg* out, int cap) {
  int n = 0;
  auto add = [&](StencilCfg c) {
    if (n >= cap || !stencil_cfg_valid(g, c)) return;
    for (int i = 0; i < n; ++i)
      if (out[i].kind == c.kind && out[i].kz == c.kz && out[i].zd == c.zd && out[i].ntx == c.ntx) return;
    out[n++] = c;
  };
  add(stencil_default_cfg(g));
  if (g.dim != 3) return n;
  add(StencilCfg{0, 0, 0, 0});
  const int kzs[] = {4, 6, 8, 12, 16, 24};
  const int widths[] = {64, 32};
  for (int w : widths)
    for (int zd = 1; zd <= 4; ++zd)
      for (int kz : kzs) add(StencilCfg{1, kz, zd, (g.nnx + w - 1) / w});
  const int kzs2[] = {4, 6, 8, 10, 12, 14, 16, 24};
  const int widths2[] = {128, 64, 32};
  for (int w : widths2)
    for (int zd = 1; zd <= 2; ++zd)
      for (int kz : kzs2) add(StencilCfg{2, kz, zd, (g.nnx + w - 1) / w});
  return n;
}

static StencilCfg resolve_cfg(const Geo& g, const StencilCfg* cfg) {
  return (cfg && stencil_cfg_valid(g, *cfg)) ? *cfg : stencil_default_cfg(g);
}

int stencil_num_partials(const Geo& g, const StencilCfg* cfg) {
  const StencilCfg c = resolve_cfg(g, cfg);
  if (c.kind == 1 || c.kind == 2) {
    const ZShape z = zmarch_shape(g, c);
    return z.ntx * z.nty * z.nzc;
  }
  const dim3 grid = grid_fits_buffers(g) ? flat_grid(g) : node_grid(g);
  return (int)(grid.x * grid.y * grid.z);
}

bool stencil_records_events(const Geo& g, const StencilCfg* cfg) {
  (void)g;
  (void)cfg;
  return true;   // every stencil launch path takes kernel start/end events
}

bool papply_supported(const Geo& g, const StencilCfg* cfg) { return resolve_cfg(g, cfg).kind == 2; }

template <typename T, typename CL>
int launch_papply_dot_t(const Geo& g, const T* z, CL k, T* out, double* part, const int* done,
                        hipStream_t s, const PFuse& pf, const StencilCfg* cfg, hipEvent_t ev0,
                        hipEvent_t ev1) {
  const StencilCfg c = resolve_cfg(g, cfg);
  if (c.kind != 2) return -1;
  const ZShape z2 = zmarch_shape(g, c);
  if (c.zd == 2)
    zmarch_launch<2, true, T, CL>(g, z2, c.kz, SM_PAPPLY_DOT, z, k, k, nullptr, out, T(0), part, done,
                                  nullptr, nullptr, s, ev0, ev1, pf);
  else
    zmarch_launch<1, true, T, CL>(g, z2, c.kz, SM_PAPPLY_DOT, z, k, k, nullptr, out, T(0), part, done,
                                  nullptr, nullptr, s, ev0, ev1, pf);
  return z2.ntx * z2.nty * z2.nzc;
}
template int launch_papply_dot_t<double, CellD>(const Geo&, const double*, CellD, double*, double*,
                                                const int*, hipStream_t, const PFuse&, const StencilCfg*,
                                                hipEvent_t, hipEvent_t);
template int launch_papply_dot_t<float, CellF>(const Geo&, const float*, CellF, float*, double*,
                                               const int*, hipStream_t, const PFuse&, const StencilCfg*,
                                               hipEvent_t, hipEvent_t);

template <typename T, typename CL>
bool launch_j0resid_t(const Geo& g, const T* b, CL k, const T* diag, T* xout, T* out, double omega,
                      const int* done, hipStream_t s, const StencilCfg* cfg, const PFuse* check) {
  const StencilCfg c = resolve_cfg(g, cfg);
  if (c.kind != 2) return false;
  const ZShape z2 = zmarch_shape(g, c);
  PFuse pf{};
  if (check && std::is_same_v<T, double>) {
    pf = *check;
    pf.chk = 1;
    done = nullptr;
  }
  pf.diag = diag;
  pf.xout = xout;
  zmarch_launch<1, true, T, CL>(g, z2, c.kz, SM_J0RESID, b, k, k, b, out, (T)omega, nullptr, done,
                                nullptr, nullptr, s, nullptr, nullptr, pf);
  return true;
}
template bool launch_j0resid_t<double, CellD>(const Geo&, const double*, CellD, const double*, double*,
                                              double*, double, const int*, hipStream_t, const StencilCfg*,
                                              const PFuse*);
template bool launch_j0resid_t<float, CellB>(const Geo&, const float*, CellB, const float*, float*, float*,
                                             double, const int*, hipStream_t, const StencilCfg*, const PFuse*);

template <typename T, typename CL>
void launch_diag_t(const Geo& g, CL k, T* diag, hipStream_t s) {
  k_diag<T, CL><<<flat_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, k, diag);
}
template void launch_diag_t<double, CellD>(const Geo&, CellD, double*, hipStream_t);
template void launch_diag_t<float, CellB>(const Geo&, CellB, float*, hipStream_t);

template <typename T, typename CL>
int launch_stencil_t(const Geo& g, int mode, const T* x, CL k, CL kref, const T* b, T* out,
                     double omega, double* part, const int* done, hipStream_t s, unsigned* cnt,
                     double* rout, hipEvent_t ev0, hipEvent_t ev1, const StencilCfg* cfg) {
  const StencilCfg c = resolve_cfg(g, cfg);
  if (c.kind == 1 || c.kind == 2) {
    const ZShape z = zmarch_shape(g, c);
#define ZL(D, TWO) \
  zmarch_launch<D, TWO, T, CL>(g, z, c.kz, mode, x, k, kref, b, out, (T)omega, part, done, cnt, rout, s, ev0, ev1)
    if (c.kind == 2) {
      if (c.zd == 2) ZL(2, true);
      else ZL(1, true);
    } else if (c.zd == 4) ZL(4, false);
    else if (c.zd == 3) ZL(3, false);
    else if (c.zd == 2) ZL(2, false);
    else ZL(1, false);
#undef ZL
  } else if (g.dim == 2) {
    stencil_dispatch<2, T, CL>(g, mode, x, k, kref, b, out, (T)omega, part, done, cnt, rout, s, ev0, ev1);
  } else {
    stencil_dispatch<3, T, CL>(g, mode, x, k, kref, b, out, (T)omega, part, done, cnt, rout, s, ev0, ev1);
  }
  return (mode == SM_APPLY_DOT || mode == SM_JACOBI_DOT) ? stencil_num_partials(g, &c) : 0;
}

template int launch_stencil_t<double, CellD>(const Geo&, int, const double*, CellD, CellD, const double*,
                                             double*, double, double*, const int*, hipStream_t,
                                             unsigned*, double*, hipEvent_t, hipEvent_t,
                                             const StencilCfg*);
template int launch_stencil_t<float, CellF>(const Geo&, int, const float*, CellF, CellF, const float*,
                                            float*, double, double*, const int*, hipStream_t,
                                            unsigned*, double*, hipEvent_t, hipEvent_t,
                                            const StencilCfg*);
template int launch_stencil_t<float, CellB>(const Geo&, int, const float*, CellB, CellB, const float*,
                                            float*, double, double*, const int*, hipStream_t,
                                            unsigned*, double*, hipEvent_t, hipEvent_t,
                                            const StencilCfg*);

int launch_stencil(const Geo& g, int mode, const double* x, const double* k, const double* kref,
                   const double* b, double* out, double omega, double* part, const int* done,
                   hipStream_t s, unsigned* cnt, double* rout, hipEvent_t ev0, hipEvent_t ev1,
                   const StencilCfg* cfg) {
  return launch_stencil_t<double, CellD>(g, mode, x, CellD{k}, CellD{kref}, b, out, omega, part, done, s,
                                         cnt, rout, ev0, ev1, cfg);
}

template <typename T>
void launch_restrict_t(const Geo& gf, const Geo& gc, const T* rf, T* rc, const int* done, hipStream_t s) {
  const dim3 grid = node_grid(gc), blk(TBX, TBY, 1);
  if (grid_fits_buffers(gf)) {
    if (gf.dim == 2) k_restrict_b<2, T><<<flat_grid(gc), blk, 0, s>>>(gf, gc, rf, rc, done);
    else k_restrict_b<3, T><<<flat_grid(gc), blk, 0, s>>>(gf, gc, rf, rc, done);
  } else {
    if (gf.dim == 2) k_restrict<2, T><<<grid, blk, 0, s>>>(gf, gc, rf, rc, done);
    else k_restrict<3, T><<<grid, blk, 0, s>>>(gf, gc, rf, rc, done);
  }
}
template void launch_restrict_t<double>(const Geo&, const Geo&, const double*, double*, const int*, hipStream_t);
template void launch_restrict_t<float>(const Geo&, const Geo&, const float*, float*, const int*, hipStream_t);

template <typename T, typename CL>
bool launch_restrict_j0_t(const Geo& gf, const Geo& gc, const T* rf, CL kc, T* bc, T* xc, double omega,
                          const int* done, hipStream_t s) {
  if (!grid_fits_buffers(gf) || !grid_fits_buffers(gc)) return false;
  const dim3 blk(TBX, TBY, 1);
  if (gf.dim == 2) k_restrict_j0<2, T, CL><<<flat_grid(gc), blk, 0, s>>>(gf, gc, rf, kc, bc, xc, (T)omega, done);
  else k_restrict_j0<3, T, CL><<<flat_grid(gc), blk, 0, s>>>(gf, gc, rf, kc, bc, xc, (T)omega, done);
  return true;
}
template bool launch_restrict_j0_t<double, CellD>(const Geo&, const Geo&, const double*, CellD, double*,
                                                  double*, double, const int*, hipStream_t);
template bool launch_restrict_j0_t<float, CellF>(const Geo&, const Geo&, const float*, CellF, float*,
                                                 float*, double, const int*, hipStream_t);

template <typename T>
void launch_prolong_t(const Geo& gf, const Geo& gc, const T* xc, T* xf, const int* done, hipStream_t s) {
  const dim3 grid = node_grid(gf), blk(TBX, TBY, 1);
  if (grid_fits_buffers(gf)) {
    if (gf.dim == 2) k_prolong_b8<2, T><<<flat_grid(gc), blk, 0, s>>>(gf, gc, xc, xf, done);
    else k_prolong_b8<3, T><<<flat_grid(gc), blk, 0, s>>>(gf, gc, xc, xf, done);
  } else {
    if (gf.dim == 2) k_prolong<2, T><<<grid, blk, 0, s>>>(gf, gc, xc, xf, done);
    else k_prolong<3, T><<<grid, blk, 0, s>>>(gf, gc, xc, xf, done);
  }
}
template void launch_prolong_t<double>(const Geo&, const Geo&, const double*, double*, const int*, hipStream_t);
template void launch_prolong_t<float>(const Geo&, const Geo&, const float*, float*, const int*, hipStream_t);

template <typename T, typename CL>
bool launch_prolong_jacobi_t(const Geo& gf, const Geo& gc, const T* xc, const T* xpre, CL k, const T* b,
                             T* out, double omega, const int* done, hipStream_t s) {
  if (!grid_fits_buffers(gf)) return false;
  const dim3 blk(TBX, TBY, 1);
  if (gf.dim == 2)
    k_prolong_jacobi<2, T, CL><<<flat_grid(gf), blk, 0, s>>>(gf, gc, xc, xpre, k, b, out, (T)omega, done);
  else
    k_prolong_jacobi<3, T, CL><<<flat_grid(gf), blk, 0, s>>>(gf, gc, xc, xpre, k, b, out, (T)omega, done);
  return true;
}
template bool launch_prolong_jacobi_t<double, CellD>(const Geo&, const Geo&, const double*, const double*,
                                                     CellD, const double*, double*, double, const int*,
                                                     hipStream_t);
template bool launch_prolong_jacobi_t<float, CellF>(const Geo&, const Geo&, const float*, const float*, CellF,
                                                    const float*, float*, double, const int*, hipStream_t);

template <typename CL, typename TO>
void launch_coarsen_t(const Geo& gf, const Geo& gc, CL kf, TO* kc, hipStream_t s) {
  const int nb = (int)((gc.ne + 255) / 256);
  if (gf.dim == 2) k_coarsen<2, CL, TO><<<nb, 256, 0, s>>>(gf, gc, kf, kc);
  else k_coarsen<3, CL, TO><<<nb, 256, 0, s>>>(gf, gc, kf, kc);
}
template void launch_coarsen_t<CellD, double>(const Geo&, const Geo&, CellD, double*, hipStream_t);
template void launch_coarsen_t<CellF, float>(const Geo&, const Geo&, CellF, float*, hipStream_t);
template void launch_coarsen_t<CellB, float>(const Geo&, const Geo&, CellB, float*, hipStream_t);

template <typename CL>
void launch_coarse_build_t(const Geo& g, CL k, double* A, int* status, hipStream_t s) {
  if (g.nn <= 128) {
    if (g.dim == 2) k_coarse_build_reg<2, CL><<<1, CB_THREADS, 0, s>>>(g, k, A, status);
    else k_coarse_build_reg<3, CL><<<1, CB_THREADS, 0, s>>>(g, k, A, status);
  } else {
    if (g.dim == 2) k_coarse_build<2, CL><<<1, CB_THREADS, 0, s>>>(g, k, A, status);
    else k_coarse_build<3, CL><<<1, CB_THREADS, 0, s>>>(g, k, A, status);
  }
}
template void launch_coarse_build_t<CellD>(const Geo&, CellD, double*, int*, hipStream_t);
template void launch_coarse_build_t<CellF>(const Geo&, CellF, double*, int*, hipStream_t);
template void launch_coarse_build_t<CellB>(const Geo&, CellB, double*, int*, hipStream_t);

template <typename T>
void launch_coarse_solve_t(const Geo& g, const double* A, const T* b, T* x, const int* done,
                           hipStream_t s) {
  const int n = (int)g.nn;
  k_coarse_solve<T><<<(n + 255) / 256, 256, 0, s>>>(n, A, b, x, done);
}
template void launch_coarse_solve_t<double>(const Geo&, const double*, const double*, double*, const int*, hipStream_t);
template void launch_coarse_solve_t<float>(const Geo&, const double*, const float*, float*, const int*, hipStream_t);

bool tail_plan(const Geo* g, const void* const* k, int lt, int L, size_t elem, TailSpec* T) {
  const int nl = L - lt;
  if (nl < 1 || nl > MGAR_MAX_TAIL) return false;
  // grids above the coarsest: node vectors and cells with a one-entry halo;
  // the coarsest: its right side and solution only, unpadded
  int off = 0;
  for (int l = 0; l < nl; ++l) {
    const Geo& gl = g[lt + l];
    T->g[l] = gl;
    T->k[l] = k[lt + l];
    const bool last = l + 1 == nl, d3 = gl.dim == 3;
    const int nn = last ? (int)gl.nn : (gl.nnx + 2) * (gl.nny + 2) * (d3 ? gl.nnz + 2 : 1);
    const int ne = last ? 0 : (gl.nx + 2) * (gl.ny + 2) * (d3 ? gl.nz + 2 : 1);
    T->off_b[l] = off; off += nn;
    T->off_xa[l] = off; off += nn;
    T->off_xb[l] = off; off += last ? 0 : nn;
    T->off_k[l] = off; off += ne;
  }
  T->nl = nl;
  T->lds_elems = off;
  T->elem = (int)elem;
  return (size_t)off * elem <= 64 * 1024 && g[lt].nn <= 4096;
}

template <typename T>
void launch_vtail_t(const TailSpec& TS, const T* b_in, T* x_out, const double* Ainv, double omega,
                    const int* done, hipStream_t s) {
  const size_t lds = sizeof(T) * (size_t)TS.lds_elems;
  if (TS.g[0].dim == 2) k_vtail<2, T><<<1, TT, lds, s>>>(TS, b_in, x_out, Ainv, (T)omega, done);
  else k_vtail<3, T><<<1, TT, lds, s>>>(TS, b_in, x_out, Ainv, (T)omega, done);
}
template void launch_vtail_t<double>(const TailSpec&, const double*, double*, const double*, double, const int*, hipStream_t);
template void launch_vtail_t<float>(const TailSpec&, const float*, float*, const double*, double, const int*, hipStream_t);

template <typename TI, typename TO>
void launch_mask_copy_t(const Geo& g, const TI* in, TO* out, hipStream_t s) {
  k_mask_copy<TI, TO><<<node_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, in, out);
}
template void launch_mask_copy_t<double, double>(const Geo&, const double*, double*, hipStream_t);
template void launch_mask_copy_t<double, float>(const Geo&, const double*, float*, hipStream_t);
template void launch_mask_copy_t<float, double>(const Geo&, const float*, double*, hipStream_t);

// ---------------------------------------------------------------- batched launchers

int batch_item_blocks(const Geo& g, int bs) { return (int)((g.nn + bs - 1) / bs); }

template <typename T, typename CL>
void launch_bstencil_t(int dim, int mode, const BItem* items, int nit, int nblk, int bs, const T* x, CL k, CL kref,
                       const T* b, T* out, double omega, double* part, const int* skip, int sstride,
                       hipStream_t s) {
  if (nblk <= 0) return;
  const dim3 blk(bs, 1, 1);
#define BCALL(D, M) \
  kb_stencil<D, M, T, CL><<<nblk, blk, 0, s>>>(items, nit, x, k, kref, b, out, (T)omega, part, skip, sstride)
#define BMODES(D)                                                 \
  switch (mode) {                                                 \
    case SM_APPLY: BCALL(D, SM_APPLY); break;                     \
    case SM_APPLY_DOT: BCALL(D, SM_APPLY_DOT); break;             \
    case SM_RESID: BCALL(D, SM_RESID); break;                     \
    case SM_JACOBI: BCALL(D, SM_JACOBI); break;                   \
    case SM_JACOBI_DOT: BCALL(D, SM_JACOBI_DOT); break;           \
    case SM_JACOBI0: BCALL(D, SM_JACOBI0); break;                 \
    case SM_NEG_DK: BCALL(D, SM_NEG_DK); break;                   \
  }
  if (dim == 2) { BMODES(2) } else { BMODES(3) }
#undef BMODES
#undef BCALL
}
template void launch_bstencil_t<double, CellD>(int, int, const BItem*, int, int, int, const double*, CellD, CellD,
                                               const double*, double*, double, double*, const int*, int,
                                               hipStream_t);
template void launch_bstencil_t<float, CellF>(int, int, const BItem*, int, int, int, const float*, CellF, CellF,
                                              const float*, float*, double, double*, const int*, int,
                                              hipStream_t);
template void launch_bstencil_t<float, CellB>(int, int, const BItem*, int, int, int, const float*, CellB, CellB,
                                              const float*, float*, double, double*, const int*, int,
                                              hipStream_t);

void launch_bstencil(int dim, int mode, const BItem* items, int nit, int nblk, int bs, const double* x,
                     const double* k, const double* kref, const double* b, double* out, double omega,
                     double* part, const int* skip, int sstride, hipStream_t s) {
  launch_bstencil_t<double, CellD>(dim, mode, items, nit, nblk, bs, x, CellD{k}, CellD{kref}, b, out, omega, part,
                                   skip, sstride, s);
}

template <typename T>
void launch_brestrict_t(int dim, const BItem* items, int nit, int nblk, int bs, const T* rf, T* rc, const int* skip,
                        int sstride, hipStream_t s) {
  if (nblk <= 0) return;
  const dim3 blk(bs, 1, 1);
  if (dim == 2) kb_restrict<2, T><<<nblk, blk, 0, s>>>(items, nit, rf, rc, skip, sstride);
  else kb_restrict<3, T><<<nblk, blk, 0, s>>>(items, nit, rf, rc, skip, sstride);
}
template void launch_brestrict_t<double>(int, const BItem*, int, int, int, const double*, double*, const int*, int,
                                         hipStream_t);
template void launch_brestrict_t<float>(int, const BItem*, int, int, int, const float*, float*, const int*, int,
                                        hipStream_t);

template <typename T>
void launch_bprolong_t(int dim, const BItem* items, int nit, int nblk, int bs, const T* xc, T* xf, const int* skip,
                       int sstride, hipStream_t s) {
  if (nblk <= 0) return;
  const dim3 blk(bs, 1, 1);
  if (dim == 2) kb_prolong<2, T><<<nblk, blk, 0, s>>>(items, nit, xc, xf, skip, sstride);
  else kb_prolong<3, T><<<nblk, blk, 0, s>>>(items, nit, xc, xf, skip, sstride);
}
template void launch_bprolong_t<double>(int, const BItem*, int, int, int, const double*, double*, const int*, int,
                                        hipStream_t);
template void launch_bprolong_t<float>(int, const BItem*, int, int, int, const float*, float*, const int*, int,
                                       hipStream_t);

template <typename CL, typename TO>
void launch_bcoarsen_t(int dim, const BItem* items, int nit, int nblk, int bs, CL kf, TO* kc, const int* skip,
                       int sstride, hipStream_t s) {
  if (nblk <= 0) return;
  const dim3 blk(bs, 1, 1);
  if (dim == 2) kb_coarsen<2, CL, TO><<<nblk, blk, 0, s>>>(items, nit, kf, kc, skip, sstride);
  else kb_coarsen<3, CL, TO><<<nblk, blk, 0, s>>>(items, nit, kf, kc, skip, sstride);
}
template void launch_bcoarsen_t<CellD, double>(int, const BItem*, int, int, int, CellD, double*, const int*, int,
                                               hipStream_t);
template void launch_bcoarsen_t<CellB, float>(int, const BItem*, int, int, int, CellB, float*, const int*, int,
                                              hipStream_t);
template void launch_bcoarsen_t<CellF, float>(int, const BItem*, int, int, int, CellF, float*, const int*, int,
                                              hipStream_t);

void launch_brestrict(int dim, const BItem* items, int nit, int nblk, int bs, const double* rf, double* rc,
                      const int* skip, int sstride, hipStream_t s) {
  launch_brestrict_t<double>(dim, items, nit, nblk, bs, rf, rc, skip, sstride, s);
}
void launch_bprolong(int dim, const BItem* items, int nit, int nblk, int bs, const double* xc, double* xf,
                     const int* skip, int sstride, hipStream_t s) {
  launch_bprolong_t<double>(dim, items, nit, nblk, bs, xc, xf, skip, sstride, s);
}
void launch_bcoarsen(int dim, const BItem* items, int nit, int nblk, int bs, const double* kf, double* kc,
                     const int* skip, int sstride, hipStream_t s) {
  launch_bcoarsen_t<CellD, double>(dim, items, nit, nblk, bs, CellD{kf}, kc, skip, sstride, s);
}

template <typename TI, typename TO>
void launch_bmask_copy_t(const BItem* items, int nit, int nblk, int bs, const TI* in, TO* out, hipStream_t s) {
  if (nblk <= 0) return;
  kb_mask_copy<TI, TO><<<nblk, dim3(bs, 1, 1), 0, s>>>(items, nit, in, out);
}
template void launch_bmask_copy_t<double, float>(const BItem*, int, int, int, const double*, float*, hipStream_t);
template void launch_bmask_copy_t<float, double>(const BItem*, int, int, int, const float*, double*, hipStream_t);

void launch_bmask_copy(const BItem* items, int nit, int nblk, int bs, const double* in, double* out,
                       hipStream_t s) {
  launch_bmask_copy_t<double, double>(items, nit, nblk, bs, in, out, s);
}

template <typename T>
void launch_bvtail_t(int dim, const BTail* jobs, int njobs, int lds_elems, double omega, const int* skip,
                     int sstride, hipStream_t s) {
  if (njobs <= 0) return;
  const size_t lds = sizeof(T) * (size_t)lds_elems;
  if (dim == 2) kb_vtail<2, T><<<njobs, TT, lds, s>>>(jobs, omega, skip, sstride);
  else kb_vtail<3, T><<<njobs, TT, lds, s>>>(jobs, omega, skip, sstride);
}
template void launch_bvtail_t<double>(int, const BTail*, int, int, double, const int*, int, hipStream_t);
template void launch_bvtail_t<float>(int, const BTail*, int, int, double, const int*, int, hipStream_t);

void launch_bvtail(int dim, const BTail* jobs, int njobs, int lds_elems, double omega,
                   const int* skip, int sstride, hipStream_t s) {
  launch_bvtail_t<double>(dim, jobs, njobs, lds_elems, omega, skip, sstride, s);
}

template <typename CL>
void launch_bcoarse_build_t(int dim, const BCoarse* jobs, int njobs, bool reg, int* status, const int* skip,
                            int sstride, hipStream_t s) {
  if (njobs <= 0) return;
  if (reg) {
    if (dim == 2) kb_coarse_build<2, true, CL><<<njobs, CB_THREADS, 0, s>>>(jobs, status, skip, sstride);
    else kb_coarse_build<3, true, CL><<<njobs, CB_THREADS, 0, s>>>(jobs, status, skip, sstride);
  } else {
    if (dim == 2) kb_coarse_build<2, false, CL><<<njobs, CB_THREADS, 0, s>>>(jobs, status, skip, sstride);
    else kb_coarse_build<3, false, CL><<<njobs, CB_THREADS, 0, s>>>(jobs, status, skip, sstride);
  }
}
template void launch_bcoarse_build_t<CellD>(int, const BCoarse*, int, bool, int*, const int*, int, hipStream_t);
template void launch_bcoarse_build_t<CellF>(int, const BCoarse*, int, bool, int*, const int*, int, hipStream_t);

void launch_bcoarse_build(int dim, const BCoarse* jobs, int njobs, bool reg, int* status,
                          const int* skip, int sstride, hipStream_t s) {
  launch_bcoarse_build_t<CellD>(dim, jobs, njobs, reg, status, skip, sstride, s);
}
