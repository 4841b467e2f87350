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
#include "mgar_launch.h"

namespace {

constexpr int TBX = 64, TBY = 4;

template <int DIM, bool DK>
__device__ inline void load_cells(const Geo& g, const double* __restrict__ k,
                                  const double* __restrict__ kref, int i, int j, int kz,
                                  double (&kv)[2][2][2]) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ex = i - 1 + a, ey = j - 1 + b, ez = (DIM == 3) ? kz - 1 + c : 0;
        const bool in = (DIM == 3 || c == 0) && ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny &&
                        ez >= 0 && ez < g.nz;
        double v = 0.0;
        if (in) {
          const long long e = geo_elem(g, ex, ey, ez);
          v = k[e];
          if (DK) v -= kref[e];
        }
        kv[c][b][a] = v;
      }
}

__device__ inline double ldx(const Geo& g, const double* __restrict__ x, int i, int j, int k) {
  const bool in = i >= 0 && i < g.nnx && j >= 0 && j < g.nny && k >= 0 && k < g.nnz;
  return in ? x[geo_node(g, i, j, k)] : 0.0;
}

// (K x)_i for node (i, j, kz) given the 2^d cell conductivities around it.
template <int DIM>
__device__ inline double node_apply(const Geo& g, const double* __restrict__ x, int i, int j,
                                    int kz, const double (&kv)[2][2][2], double& ksum) {
  if (DIM == 2) {
    double xv[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) xv[dy][dx] = ldx(g, x, i + dx - 1, j + dy - 1, 0);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int sx = a ? 2 : 0, sy = b ? 2 : 0;
        const double ke = kv[0][b][a];
        s0 += ke;
        s1 += ke * (xv[1][sx] + xv[sy][1]);
        s2 += ke * xv[sy][sx];
      }
    ksum = s0;
    return (2.0 / 3.0) * s0 * xv[1][1] - (1.0 / 6.0) * s1 - (1.0 / 3.0) * s2;
  } else {
    double xv[3][3][3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int nz = (dx != 1) + (dy != 1) + (dz != 1);
          xv[dz][dy][dx] = (nz == 1) ? 0.0 : ldx(g, x, i + dx - 1, j + dy - 1, kz + dz - 1);
        }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int sx = a ? 2 : 0, sy = b ? 2 : 0, sz = c ? 2 : 0;
          const double ke = kv[c][b][a];
          s0 += ke;
          s1 += ke * (xv[1][sy][sx] + xv[sz][1][sx] + xv[sz][sy][1] + xv[sz][sy][sx]);
        }
    ksum = s0;
    return g.h * ((1.0 / 3.0) * s0 * xv[1][1][1] - (1.0 / 12.0) * s1);
  }
}

template <int DIM, int MODE>
__global__ __launch_bounds__(TBX* TBY) void k_stencil(Geo g, const double* __restrict__ x,
                                                      const double* __restrict__ k,
                                                      const double* __restrict__ kref,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ out, double omega,
                                                      double* __restrict__ part,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[TBX * TBY / MGAR_WAVE];
  const int i = blockIdx.x * TBX + threadIdx.x;
  const int j = blockIdx.y * TBY + threadIdx.y;
  const int kz = blockIdx.z;
  const bool valid = i < g.nnx && j < g.nny;
  double dotv = 0.0;
  if (valid) {
    const long long n = geo_node(g, i, j, kz);
    double r = 0.0;
    if (!geo_fixed(g, i, j, kz)) {
      double kv[2][2][2];
      load_cells<DIM, MODE == SM_NEG_DK>(g, k, kref, i, j, kz, kv);
      double ksum = 0.0;
      double y = 0.0;
      if (MODE != SM_JACOBI0) {
        y = node_apply<DIM>(g, x, i, j, kz, kv, ksum);
      } else {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int a = 0; a < 2; ++a) ksum += kv[c][bb][a];
      }
      const double diag = (DIM == 3 ? g.h * (1.0 / 3.0) : (2.0 / 3.0)) * ksum;
      if (MODE == SM_APPLY || MODE == SM_APPLY_DOT) {
        r = y;
        if (MODE == SM_APPLY_DOT) dotv = x[n] * r;
      } else if (MODE == SM_RESID) {
        r = b[n] - y;
      } else if (MODE == SM_JACOBI || MODE == SM_JACOBI_DOT) {
        r = x[n] + omega * (b[n] - y) / diag;
        if (MODE == SM_JACOBI_DOT) dotv = b[n] * r;
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
    if (flat_tid() == 0) part[flat_bid()] = s;
  }
}

// Restriction r_c = P^T r_f: coarse node (I,J,K) gathers the fine nodes
// (2I+a, 2J+b, 2K+c), a,b,c in {-1,0,1}, with weight prod(1 if 0 else 1/2).
template <int DIM>
__global__ __launch_bounds__(TBX* TBY) void k_restrict(Geo gf, Geo gc, const double* __restrict__ rf,
                                                       double* __restrict__ rc,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  const int I = blockIdx.x * TBX + threadIdx.x;
  const int J = blockIdx.y * TBY + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= gc.nnx || J >= gc.nny) return;
  double s = 0.0;
  if (!geo_fixed(gc, I, J, K)) {
#pragma unroll
    for (int c = (DIM == 3 ? -1 : 0); c <= (DIM == 3 ? 1 : 0); ++c) {
      double sy = 0.0;
#pragma unroll
      for (int b = -1; b <= 1; ++b) {
        double sx = 0.0;
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
          const double v = ldx(gf, rf, 2 * I + a, 2 * J + b, 2 * K + c);
          sx += (a == 0 ? 1.0 : 0.5) * v;
        }
        sy += (b == 0 ? 1.0 : 0.5) * sx;
      }
      s += (c == 0 ? 1.0 : 0.5) * sy;
    }
  }
  rc[geo_node(gc, I, J, K)] = s;
}

// Interpolation and correction x_f += P x_c (bi-/trilinear; fixed fine rows are 0).
template <int DIM>
__global__ __launch_bounds__(TBX* TBY) void k_prolong(Geo gf, Geo gc, const double* __restrict__ xc,
                                                      double* __restrict__ xf,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.x * TBX + threadIdx.x;
  const int j = blockIdx.y * TBY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= gf.nnx || j >= gf.nny) return;
  if (geo_fixed(gf, i, j, k)) return;
  const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
  const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (DIM == 3 && (k & 1)) ? 2 : 1;
  const double wi = (i & 1) ? 0.5 : 1.0, wj = (j & 1) ? 0.5 : 1.0,
               wk = (DIM == 3 && (k & 1)) ? 0.5 : 1.0;
  double s = 0.0;
  for (int c = 0; c < nk; ++c) {
    double sy = 0.0;
    for (int b = 0; b < nj; ++b) {
      double sx = 0.0;
      for (int a = 0; a < ni; ++a) sx += xc[geo_node(gc, I0 + a, J0 + b, K0 + c)];
      sy += wi * sx;
    }
    s += wj * sy;
  }
  xf[geo_node(gf, i, j, k)] += wk * s;
}

// Coarse conductivity: mean of the 2^d children.
template <int DIM>
__global__ void k_coarsen(Geo gf, Geo gc, const double* __restrict__ kf, double* __restrict__ kc) {
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
        s += kf[geo_elem(gf, 2 * ex + a, 2 * ey + b, DIM == 3 ? 2 * ez + c : 0)];
  kc[e] = s * (DIM == 3 ? 0.125 : 0.25);
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

// Coarsest grid: assemble the dense N_c x N_c matrix (identity rows/columns on
// Dirichlet nodes), then invert it in place by Gauss-Jordan elimination without
// pivoting (valid for SPD matrices) and symmetrise. One workgroup.
template <int DIM>
__global__ __launch_bounds__(CB_THREADS) void k_coarse_build(Geo g, const double* __restrict__ k,
                                                             double* __restrict__ A,
                                                             int* __restrict__ status) {
  __shared__ double colp[CB_MAXN];
  __shared__ double rowp[CB_MAXN];
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
          const double ke = k[geo_elem(g, ex, ey, ez)];
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
  const int tc = t & 31, tr = t >> 5;  // 32 x 32 thread layout for the updates
  int bad = 0;
  for (int p = 0; p < n; ++p) {
    for (int idx = t; idx < n; idx += CB_THREADS) {
      colp[idx] = A[(long long)idx * n + p];
      rowp[idx] = A[(long long)p * n + idx];
    }
    __syncthreads();
    const double piv = rowp[p];
    if (!(piv > 0.0)) bad = 1;
    const double inv = 1.0 / piv;
    for (int i = tr; i < n; i += CB_THREADS / 32) {
      const double ci = colp[i];
      for (int j = tc; j < n; j += 32) {
        double v;
        if (i == p && j == p) v = inv;
        else if (i == p) v = rowp[j] * inv;
        else if (j == p) v = -ci * inv;
        else v = A[(long long)i * n + j] - ci * rowp[j] * inv;
        A[(long long)i * n + j] = v;
      }
    }
    __syncthreads();
  }
  // symmetrise
  for (int i = tr; i < n; i += CB_THREADS / 32)
    for (int j = tc; j < n; j += 32)
      if (j > i) {
        const double v = 0.5 * (A[(long long)i * n + j] + A[(long long)j * n + i]);
        A[(long long)i * n + j] = v;
        A[(long long)j * n + i] = v;
      }
  if (t == 0 && bad) status[0] = 1;
}

// x = A^-1 b on the coarsest grid (A symmetric: column reads are coalesced).
__global__ __launch_bounds__(256) void k_coarse_solve(int n, const double* __restrict__ A,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ x,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += A[(long long)j * n + i] * b[j];
  x[i] = s;
}

__global__ __launch_bounds__(TBX* TBY) void k_mask_copy(Geo g, const double* __restrict__ in,
                                                        double* __restrict__ out) {
  const int i = blockIdx.x * TBX + threadIdx.x;
  const int j = blockIdx.y * TBY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nnx || j >= g.nny) return;
  const long long n = geo_node(g, i, j, k);
  out[n] = geo_fixed(g, i, j, k) ? 0.0 : in[n];
}

dim3 node_grid(const Geo& g) {
  return dim3((g.nnx + TBX - 1) / TBX, (g.nny + TBY - 1) / TBY, g.nnz);
}

template <int DIM>
void stencil_dispatch(const Geo& g, int mode, const double* x, const double* k, const double* kref,
                      const double* b, double* out, double omega, double* part, const int* done,
                      hipStream_t s) {
  const dim3 grid = node_grid(g), blk(TBX, TBY, 1);
  switch (mode) {
    case SM_APPLY: k_stencil<DIM, SM_APPLY><<<grid, blk, 0, s>>>(g, x, k, kref, b, out, omega, part, done); break;
    case SM_APPLY_DOT: k_stencil<DIM, SM_APPLY_DOT><<<grid, blk, 0, s>>>(g, x, k, kref, b, out, omega, part, done); break;
    case SM_RESID: k_stencil<DIM, SM_RESID><<<grid, blk, 0, s>>>(g, x, k, kref, b, out, omega, part, done); break;
    case SM_JACOBI: k_stencil<DIM, SM_JACOBI><<<grid, blk, 0, s>>>(g, x, k, kref, b, out, omega, part, done); break;
    case SM_JACOBI_DOT: k_stencil<DIM, SM_JACOBI_DOT><<<grid, blk, 0, s>>>(g, x, k, kref, b, out, omega, part, done); break;
    case SM_JACOBI0: k_stencil<DIM, SM_JACOBI0><<<grid, blk, 0, s>>>(g, x, k, kref, b, out, omega, part, done); break;
    case SM_NEG_DK: k_stencil<DIM, SM_NEG_DK><<<grid, blk, 0, s>>>(g, x, k, kref, b, out, omega, part, done); break;
  }
}

}  // namespace

int stencil_num_partials(const Geo& g) {
  const dim3 grid = node_grid(g);
  return (int)(grid.x * grid.y * grid.z);
}

int launch_stencil(const Geo& g, int mode, const double* x, const double* k, const double* kref,
                   const double* b, double* out, double omega, double* part, const int* done,
                   hipStream_t s) {
  if (g.dim == 2) stencil_dispatch<2>(g, mode, x, k, kref, b, out, omega, part, done, s);
  else stencil_dispatch<3>(g, mode, x, k, kref, b, out, omega, part, done, s);
  return (mode == SM_APPLY_DOT || mode == SM_JACOBI_DOT) ? stencil_num_partials(g) : 0;
}

void launch_restrict(const Geo& gf, const Geo& gc, const double* rf, double* rc, const int* done,
                     hipStream_t s) {
  const dim3 grid = node_grid(gc), blk(TBX, TBY, 1);
  if (gf.dim == 2) k_restrict<2><<<grid, blk, 0, s>>>(gf, gc, rf, rc, done);
  else k_restrict<3><<<grid, blk, 0, s>>>(gf, gc, rf, rc, done);
}

void launch_prolong(const Geo& gf, const Geo& gc, const double* xc, double* xf, const int* done,
                    hipStream_t s) {
  const dim3 grid = node_grid(gf), blk(TBX, TBY, 1);
  if (gf.dim == 2) k_prolong<2><<<grid, blk, 0, s>>>(gf, gc, xc, xf, done);
  else k_prolong<3><<<grid, blk, 0, s>>>(gf, gc, xc, xf, done);
}

void launch_coarsen(const Geo& gf, const Geo& gc, const double* kf, double* kc, hipStream_t s) {
  const int nb = (int)((gc.ne + 255) / 256);
  if (gf.dim == 2) k_coarsen<2><<<nb, 256, 0, s>>>(gf, gc, kf, kc);
  else k_coarsen<3><<<nb, 256, 0, s>>>(gf, gc, kf, kc);
}

void launch_coarse_build(const Geo& g, const double* k, double* A, int* status, hipStream_t s) {
  if (g.dim == 2) k_coarse_build<2><<<1, CB_THREADS, 0, s>>>(g, k, A, status);
  else k_coarse_build<3><<<1, CB_THREADS, 0, s>>>(g, k, A, status);
}

void launch_coarse_solve(const Geo& g, const double* A, const double* b, double* x,
                         const int* done, hipStream_t s) {
  const int n = (int)g.nn;
  k_coarse_solve<<<(n + 255) / 256, 256, 0, s>>>(n, A, b, x, done);
}

void launch_mask_copy(const Geo& g, const double* in, double* out, hipStream_t s) {
  k_mask_copy<<<node_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, in, out);
}
