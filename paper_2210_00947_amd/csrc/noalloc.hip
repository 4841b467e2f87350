// Residual check that allocates nothing: ||q - K(xphys) T|| / ||q|| over the
// free nodes (the criterion of mgar_residual), for callers that cannot
// allocate device memory (code under stream capture, serving loops).
//
// The block partial sums live in `scratch`, a file-scope device array of
// NA_MAX_BLOCKS * 2 doubles (64 KiB). Host code never passes the array's name
// to a kernel: at the first call on a device, with that device current, its
// device address is looked up once (hipGetSymbolAddress) and kept per device;
// kernels take that address as an argument. Every call on one GPU shares that
// GPU's copy of the array, which keeps the last call's partials: two calls of
// one process that overlap on the same GPU (on different streams or host
// threads) race on it and must be ordered by the caller. The grid-stride
// kernel writes every partial that the final kernel reads, so nothing has to
// start at zero and no state carries from one call to the next.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "mgar.h"
#include "mgar_launch.h"

namespace {

constexpr int NA_THREADS = 256;
constexpr int NA_MAX_BLOCKS = 4096;      // partials: NA_MAX_BLOCKS * 2 doubles
constexpr int NA_MAX_DEVICES = 64;
constexpr long long NA_MAX_NODES = (1LL << 31) - 1;

static __device__ __align__(256) double scratch[NA_MAX_BLOCKS * 2];

std::mutex g_mu;
double* g_ptr[NA_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_ptr(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NA_MAX_DEVICES) return MGAR_E_HIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MGAR_E_HIP;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return MGAR_OK;
}

__device__ inline double na_simp(double x, double k0, double kmin, double p) {
  return kmin + (k0 - kmin) * ((p == 3.0) ? x * x * x : pow(x, p));
}

// Q1 element matrix entry between local corners a and b of a cell of edge h:
// 2D 2/3, -1/6, -1/3 by Hamming distance 0..2; 3D h * (1/3, 0, -1/12, -1/12)
// by distance 0..3 (Eq 3 with the bilinear / trilinear element).
__device__ inline double na_ke(int dim, int a, int b, double h) {
  const int d = __popc((unsigned)(a ^ b));
  if (dim == 2) return d == 0 ? 2.0 / 3.0 : (d == 1 ? -1.0 / 6.0 : -1.0 / 3.0);
  return h * (d == 0 ? 1.0 / 3.0 : (d == 1 ? 0.0 : -1.0 / 12.0));
}

// Per block: partial sums of r_i^2 and q_i^2 over the free nodes it visits
// (grid-stride), r = q - K(simp(xphys)) T with T and q read as 0 on Dirichlet
// nodes.
__global__ __launch_bounds__(NA_THREADS) void k_resid_partials(Geo g, const double* __restrict__ xphys,
                                                               const double* __restrict__ q,
                                                               const double* __restrict__ T, double k0,
                                                               double kmin, double penal,
                                                               double* __restrict__ part) {
  __shared__ double sh[2 * NA_THREADS / 64];
  double rr = 0.0, qq = 0.0;
  const int nc = g.dim == 3 ? 8 : 4;
  for (long long n = blockIdx.x * (long long)NA_THREADS + threadIdx.x; n < g.nn;
       n += (long long)gridDim.x * NA_THREADS) {
    const int i = (int)(n % g.nnx);
    const int j = (int)((n / g.nnx) % g.nny);
    const int k = (int)(n / ((long long)g.nnx * g.nny));
    if (geo_fixed(g, i, j, k)) continue;
    double y = 0.0;
    for (int cz = 0; cz < (g.dim == 3 ? 2 : 1); ++cz) {
      const int ez = g.dim == 3 ? k - 1 + cz : 0;
      if (ez < 0 || ez >= g.nz) continue;
      for (int cy = 0; cy < 2; ++cy) {
        const int ey = j - 1 + cy;
        if (ey < 0 || ey >= g.ny) continue;
        for (int cx = 0; cx < 2; ++cx) {
          const int ex = i - 1 + cx;
          if (ex < 0 || ex >= g.nx) continue;
          // local corner of node n in this cell
          const int ci = (1 - cx) | ((1 - cy) << 1) | (g.dim == 3 ? (1 - cz) << 2 : 0);
          double acc = 0.0;
          for (int c = 0; c < nc; ++c) {
            const int ni = ex + (c & 1), nj = ey + ((c >> 1) & 1), nk = ez + ((c >> 2) & 1);
            const double t = geo_fixed(g, ni, nj, nk) ? 0.0 : T[geo_node(g, ni, nj, nk)];
            acc += na_ke(g.dim, ci, c, g.h) * t;
          }
          y += na_simp(xphys[geo_elem(g, ex, ey, ez)], k0, kmin, penal) * acc;
        }
      }
    }
    const double qi = q[n];
    const double r = qi - y;
    rr += r * r;
    qq += qi * qi;
  }
  // deterministic block sums (fixed wave and lane order)
  const double a = block_sum(rr, sh);
  const double b = block_sum(qq, sh + NA_THREADS / 64);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// One block: sum the partials in block order, out = sqrt(rr / qq) (0 if q = 0).
__global__ __launch_bounds__(NA_THREADS) void k_resid_final(const double* __restrict__ part, int nb,
                                                            double* __restrict__ out) {
  __shared__ double sh[2 * NA_THREADS / 64];
  double rr = 0.0, qq = 0.0;
  for (int b = threadIdx.x; b < nb; b += NA_THREADS) {
    rr += part[2 * b];
    qq += part[2 * b + 1];
  }
  const double a = block_sum(rr, sh);
  const double c = block_sum(qq, sh + NA_THREADS / 64);
  if (threadIdx.x == 0) *out = c > 0.0 ? sqrt(a / c) : 0.0;
}

}  // namespace

extern "C" int mgar_residual_noalloc(const mgar_params* p, const double* xphys, const double* q,
                                     const double* T, double* relres, void* stream) {
  if (!p || !xphys || !q || !T || !relres) return MGAR_E_ARG;
  if (p->dim != 2 && p->dim != 3) return MGAR_E_ARG;
  if (p->nelx < 1 || p->nely < 1 || (p->dim == 3 && p->nelz < 1)) return MGAR_E_ARG;
  if (!(p->k0 > 0.0) || !(p->kmin > 0.0) || !(p->penal >= 1.0)) return MGAR_E_ARG;
  mgar_params p0 = *p;
  p0.levels = 1;
  const Geo g = mgar_internal_geo(p0, 0);
  if (g.nn > NA_MAX_NODES) return MGAR_E_ARG;   // beyond the 32-bit node coordinates the kernel takes
  double* part = nullptr;
  const int rc = scratch_ptr(&part);
  if (rc != MGAR_OK) return rc;
  const long long want = (g.nn + NA_THREADS - 1) / NA_THREADS;
  const int nb = (int)(want < NA_MAX_BLOCKS ? want : NA_MAX_BLOCKS);
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_resid_partials<<<nb, NA_THREADS, 0, s>>>(g, xphys, q, T, p->k0, p->kmin, p->penal, part);
  k_resid_final<<<1, NA_THREADS, 0, s>>>(part, nb, relres);
  return hipGetLastError() == hipSuccess ? MGAR_OK : MGAR_E_HIP;
}
