// Element-level kernels of the optimisation loop: SIMP conductivity (Eq 4),
// consistent load, cone density filter and its adjoint (Eq 6-9, 11), element
// compliance sensitivity (Eq 10), and the optimality-criteria update.
#include "mgar_launch.h"
#include "zbuf.h"

namespace {

constexpr int TBX = 64, TBY = 4;
constexpr int VB = 256;
constexpr int VMAXB = 1024;
constexpr int FB = 1024;

dim3 elem_grid(const Geo& g) {
  return dim3((g.nx + TBX - 1) / TBX, (g.ny + TBY - 1) / TBY, g.nz);
}
dim3 node_grid(const Geo& g) {
  return dim3((g.nnx + TBX - 1) / TBX, (g.nny + TBY - 1) / TBY, g.nnz);
}
int nblocks(long long n) {
  long long nb = (n + VB - 1) / VB;
  return (int)(nb > VMAXB ? VMAXB : (nb < 1 ? 1 : nb));
}

__device__ inline double simp_pow(double x, double p) {
  return (p == 3.0) ? x * x * x : pow(x, p);
}

__global__ __launch_bounds__(VB) void k_simp(const double* __restrict__ xp, double* __restrict__ k,
                                             long long n, double k0, double kmin, double p) {
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    k[i] = kmin + (k0 - kmin) * simp_pow(xp[i], p);
}

// q_i = sum over cells e at node i of Qe_e |e| / 2^d; 0 on Dirichlet nodes.
template <int DIM>
__global__ __launch_bounds__(TBX* TBY) void k_load(Geo g, const double* __restrict__ Qe,
                                                   double* __restrict__ q) {
  const int i = blockIdx.x * TBX + threadIdx.x;
  const int j = blockIdx.y * TBY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nnx || j >= g.nny) return;
  double s = 0.0;
  if (!geo_fixed(g, i, j, k)) {
    for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int ex = i - 1 + a, ey = j - 1 + b, ez = (DIM == 3) ? k - 1 + c : 0;
          if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny || ez < 0 || ez >= g.nz) continue;
          s += Qe[geo_elem(g, ex, ey, ez)];
        }
    const double vol = (DIM == 3) ? g.h * g.h * g.h : g.h * g.h;
    s *= vol / (DIM == 3 ? 8.0 : 4.0);
  }
  q[geo_node(g, i, j, k)] = s;
}

// y_e = (sum_j w_ej x_j) * scale_e over the in-grid taps (scale = 1 if null).
// With scale = 1/Hs this is the forward filter; with g = dc~/Hs and no scale it
// is the adjoint (the cone weight is symmetric in e and j).
__global__ __launch_bounds__(TBX* TBY) void k_filter(Geo g, const int* __restrict__ off,
                                                     const double* __restrict__ w, int ntap,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ scale,
                                                     double* __restrict__ y) {
  const int ex = blockIdx.x * TBX + threadIdx.x;
  const int ey = blockIdx.y * TBY + threadIdx.y;
  const int ez = blockIdx.z;
  if (ex >= g.nx || ey >= g.ny) return;
  double s = 0.0;
  for (int t = 0; t < ntap; ++t) {
    const int jx = ex + off[3 * t], jy = ey + off[3 * t + 1], jz = ez + off[3 * t + 2];
    if (jx < 0 || jx >= g.nx || jy < 0 || jy >= g.ny || jz < 0 || jz >= g.nz) continue;
    s += w[t] * x[geo_elem(g, jx, jy, jz)];
  }
  const long long e = geo_elem(g, ex, ey, ez);
  y[e] = scale ? s * scale[e] : s;
}

// As k_filter with buffer loads: taps outside the grid read 0 (and so add
// w * 0 in place of being skipped), eight taps per step are loaded before the
// first is used, and the sum runs over the taps in the same order.
constexpr int FTAP = 8;
__global__ __launch_bounds__(TBX* TBY) void k_filter_b(Geo g, const int* __restrict__ off,
                                                       const double* __restrict__ w, int ntap,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ scale,
                                                       double* __restrict__ y) {
  const int ex = blockIdx.x * TBX + threadIdx.x;
  const int ey = blockIdx.y * TBY + threadIdx.y;
  const int ez = blockIdx.z;
  if (ex >= g.nx || ey >= g.ny) return;
  const __amdgpu_buffer_rsrc_t rx = zrsrc(x, g.ne * 8);
  double s = 0.0;
  for (int t0 = 0; t0 < ntap; t0 += FTAP) {
    double v[FTAP], wt[FTAP];
#pragma unroll
    for (int u = 0; u < FTAP; ++u) {
      const int t = t0 + u, tc = min(t, ntap - 1);
      const int jx = ex + off[3 * tc], jy = ey + off[3 * tc + 1], jz = ez + off[3 * tc + 2];
      const bool in = t < ntap && jx >= 0 && jx < g.nx && jy >= 0 && jy < g.ny && jz >= 0 && jz < g.nz;
      v[u] = zbload<double>(rx, in ? (unsigned)(jx + g.nx * (jy + g.ny * jz)) * 8u : ZOOB);
      wt[u] = w[tc];
    }
#pragma unroll
    for (int u = 0; u < FTAP; ++u) s += wt[u] * v[u];
  }
  const long long e = geo_elem(g, ex, ey, ez);
  y[e] = scale ? s * scale[e] : s;
}

// As k_filter_b with the inputs of a block staged in LDS first: a 64 x 4 tile
// of one element plane plus a halo of hr elements in every direction (hr =
// largest tap offset), so each input is loaded from memory about once per
// block instead of once per tap; the taps then read LDS in the same order.
// Halo positions outside the grid hold 0.
__global__ __launch_bounds__(TBX* TBY) void k_filter_lds(Geo g, const int* __restrict__ off,
                                                         const double* __restrict__ w, int ntap, int hr,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ scale,
                                                         double* __restrict__ y) {
  extern __shared__ double tile[];
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + TBX * ly;
  const int ex0 = blockIdx.x * TBX, ey0 = blockIdx.y * TBY, ez = blockIdx.z;
  const int TW = TBX + 2 * hr, TH = TBY + 2 * hr, TD = g.dim == 3 ? 2 * hr + 1 : 1;
  const int n = TW * TH * TD;
  // the taps as (LDS offset, weight), staged after the tile
  double* tw = tile + n;
  int* to = reinterpret_cast<int*>(tw + ntap);
  for (int q = tid; q < ntap; q += TBX * TBY) {
    tw[q] = w[q];
    to[q] = off[3 * q] + TW * (off[3 * q + 1] + TH * off[3 * q + 2]);
  }
  const __amdgpu_buffer_rsrc_t rx = zrsrc(x, g.ne * 8);
  for (int idx = tid; idx < n; idx += TBX * TBY) {
    const int ix = idx % TW, r = idx / TW, iy = r % TH, iz = r / TH;
    const int jx = ex0 - hr + ix, jy = ey0 - hr + iy, jz = g.dim == 3 ? ez - hr + iz : 0;
    const bool in = jx >= 0 && jx < g.nx && jy >= 0 && jy < g.ny && jz >= 0 && jz < g.nz;
    tile[idx] = zbload<double>(rx, in ? (unsigned)(jx + g.nx * (jy + g.ny * jz)) * 8u : ZOOB);
  }
  __syncthreads();
  const int ex = ex0 + lx, ey = ey0 + ly;
  if (ex >= g.nx || ey >= g.ny) return;
  const int base = (g.dim == 3 ? hr * TH * TW : 0) + (ly + hr) * TW + (lx + hr);
  double s = 0.0;
  for (int t = 0; t < ntap; ++t) s += tw[t] * tile[base + to[t]];
  const long long e = geo_elem(g, ex, ey, ez);
  y[e] = scale ? s * scale[e] : s;
}

__global__ __launch_bounds__(TBX* TBY) void k_filter_hs(Geo g, const int* __restrict__ off,
                                                        const double* __restrict__ w, int ntap,
                                                        double* __restrict__ invHs) {
  const int ex = blockIdx.x * TBX + threadIdx.x;
  const int ey = blockIdx.y * TBY + threadIdx.y;
  const int ez = blockIdx.z;
  if (ex >= g.nx || ey >= g.ny) return;
  double s = 0.0;
  for (int t = 0; t < ntap; ++t) {
    const int jx = ex + off[3 * t], jy = ey + off[3 * t + 1], jz = ez + off[3 * t + 2];
    if (jx < 0 || jx >= g.nx || jy < 0 || jy >= g.ny || jz < 0 || jz >= g.nz) continue;
    s += w[t];
  }
  invHs[geo_elem(g, ex, ey, ez)] = 1.0 / s;
}

template <int DIM>
__device__ inline double ke_unit(int ca, int cb) {
  const int hd = __popc(ca ^ cb);
  if (DIM == 2) return hd == 0 ? 2.0 / 3.0 : (hd == 1 ? -1.0 / 6.0 : -1.0 / 3.0);
  return hd == 0 ? 1.0 / 3.0 : (hd == 1 ? 0.0 : -1.0 / 12.0);
}

// g_e = -p (k0 - kmin) xphys_e^(p-1) T_e^T KE T_e / Hs_e (Eq 10 divided by the
// filter normalisation, ready for the adjoint gather of Eq 9/11).
template <int DIM>
__global__ __launch_bounds__(TBX* TBY) void k_sens(Geo g, const double* __restrict__ xphys,
                                                   const double* __restrict__ T,
                                                   const double* __restrict__ invHs, double k0,
                                                   double kmin, double p, double* __restrict__ gout) {
  const int ex = blockIdx.x * TBX + threadIdx.x;
  const int ey = blockIdx.y * TBY + threadIdx.y;
  const int ez = blockIdx.z;
  if (ex >= g.nx || ey >= g.ny) return;
  constexpr int NC = (DIM == 3) ? 8 : 4;
  double t[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int ni = ex + (c & 1), nj = ey + ((c >> 1) & 1), nk = (DIM == 3) ? ez + ((c >> 2) & 1) : 0;
    t[c] = geo_fixed(g, ni, nj, nk) ? 0.0 : T[geo_node(g, ni, nj, nk)];
  }
  double en = 0.0;
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    double ya = 0.0;
#pragma unroll
    for (int b = 0; b < NC; ++b) ya += ke_unit<DIM>(a, b) * t[b];
    en += t[a] * ya;
  }
  const long long e = geo_elem(g, ex, ey, ez);
  const double xp = xphys[e];
  const double dpow = (p == 3.0) ? xp * xp : pow(xp, p - 1.0);
  gout[e] = -p * (k0 - kmin) * dpow * en * invHs[e];
}

// ------------------------------------------------------------------- OC
// Bisection on lambda in [0, 1e9] until (l2-l1)/(l1+l2) <= tol, deciding each
// midpoint m by S(m) > target, with S(lambda) = sum_e dv_e x_new_e(lambda)
// non-increasing in lambda. Each pass evaluates S at OC_NCAND candidates in the
// still-undecided range; a single-thread walk then replays the bisection
// midpoints in order, deciding each one from the evaluated bracket, until a
// midpoint falls inside it. The midpoints, and so lam_last, are the same
// floating-point values a plain bisection computes.
//
// Placement of the next candidates for the undecided range [a, b] =
// [max(l1, lo_known), min(l2, hi_known)]: geometric while it spans more than
// 64x (or a = 0, then from b 1e-40), otherwise 7 even points and 8 around the
// secant estimate in u = lambda^-1/2 from the evaluated bracket (S is close to
// affine in u, since unclamped elements contribute dv x sqrt(B) u), spaced
// (b - a) / 128 (or / 16384 once the range is within 1 % of a).
struct OcFill {
  bool geo;
  double a, b, r, est, d;
};

__device__ inline OcFill oc_fill_params(double l1, double l2, double lo, double hi, double slo, double shi,
                                        double target) {
  OcFill f;
  f.a = fmax(l1, lo);
  f.b = fmin(l2, hi);
  f.geo = f.a <= 0.0 || f.b > 64.0 * f.a;
  f.r = 0.0;
  f.d = 0.0;
  f.est = 0.5 * (f.a + f.b);
  if (f.geo) {
    if (f.a <= 0.0) f.a = f.b * 1e-40;
    f.r = log(f.b / f.a) / (OC_NCAND + 1);
    return f;
  }
  if (lo > 0.0 && hi < INFINITY && slo > shi) {
    const double ul = 1.0 / sqrt(lo), uh = 1.0 / sqrt(hi);
    const double u = uh + (target - shi) * (ul - uh) / (slo - shi);
    if (u > 0.0) f.est = fmin(f.b, fmax(f.a, 1.0 / (u * u)));
  }
  f.d = (f.b - f.a) / ((f.b - f.a > 0.01 * f.a) ? 128.0 : 16384.0);
  return f;
}

// Candidate t of a placement.
__device__ inline double oc_candidate(int t, const OcFill& f) {
  if (f.geo) return f.a * exp(f.r * (t + 1));
  constexpr int NLIN = 7;
  if (t < NLIN) return f.a + (f.b - f.a) * (t + 1) / (NLIN + 1);
  return fmin(f.b, fmax(f.a, f.est + f.d * (t - NLIN - 3.5)));
}

__device__ void oc_fill_candidates(OcDev* oc, double target) {
  const OcFill f = oc_fill_params(oc->l1, oc->l2, oc->lo_known, oc->hi_known, oc->s_lo, oc->s_hi, target);
  for (int t = 0; t < OC_NCAND; ++t) oc->cand[t] = oc_candidate(t, f);
}

// With a previous multiplier (hint > 0, e.g. the last call's result), the first
// candidates are hint * 2^((t - 7) / 2), t = 0..14 (hint / 11 .. 11 hint): the
// bisection itself is unchanged (it still starts from [0, 1e9]), only the
// points where S is evaluated first.
__global__ void k_oc_init(OcDev* oc, double target, double hint) {
  oc->l1 = 0.0;
  oc->l2 = 1e9;
  oc->lam_last = 0.5e9;
  oc->lo_known = 0.0;
  oc->hi_known = INFINITY;
  oc->s_lo = 0.0;
  oc->s_hi = 0.0;
  oc->done = 0;
  oc->steps = 0;
  if (hint > 0.0 && hint < oc->l2) {
    for (int t = 0; t < OC_NCAND; ++t) oc->cand[t] = fmin(oc->l2, hint * exp2(0.5 * (t - OC_NCAND / 2)));
  } else {
    oc_fill_candidates(oc, target);
  }
}

__global__ __launch_bounds__(VB) void k_oc_pass(const double* __restrict__ x,
                                                const double* __restrict__ dc,
                                                const double* __restrict__ dv, long long n,
                                                double move, const OcDev* __restrict__ oc,
                                                double* __restrict__ part) {
  if (oc->done) return;
  __shared__ double rs[OC_NCAND];
  __shared__ double red[VB / MGAR_WAVE][OC_NCAND];
  if (threadIdx.x < OC_NCAND) rs[threadIdx.x] = 1.0 / sqrt(oc->cand[threadIdx.x]);
  __syncthreads();
  double s[OC_NCAND];
#pragma unroll
  for (int t = 0; t < OC_NCAND; ++t) s[t] = 0.0;
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
    const double xi = x[i], wi = dv[i];
    const double B = fmax(0.0, -dc[i]) / wi;
    const double c = xi * sqrt(B);
    const double lo = fmax(0.0, xi - move), hi = fmin(1.0, xi + move);
#pragma unroll
    for (int t = 0; t < OC_NCAND; ++t) s[t] += wi * fmax(lo, fmin(hi, c * rs[t]));
  }
  const int lane = threadIdx.x & (MGAR_WAVE - 1), wv = threadIdx.x / MGAR_WAVE;
#pragma unroll
  for (int t = 0; t < OC_NCAND; ++t) {
    const double v = wave_sum(s[t]);
    if (lane == 0) red[wv][t] = v;
  }
  __syncthreads();
  // candidate-major partials: part[t * gridDim.x + block]
  if (threadIdx.x < OC_NCAND) {
    double v = 0.0;
    for (int w = 0; w < VB / MGAR_WAVE; ++w) v += red[w][threadIdx.x];
    part[threadIdx.x * gridDim.x + blockIdx.x] = v;
  }
}

// S at the candidates from the pass's candidate-major block partials (wave t
// sums candidate t, lane l adding blocks l, l + 64, ... in order; np <= VMAXB),
// then the bisection replayed by thread 0 and the next candidates placed by
// threads 0..OC_NCAND-1.
__global__ __launch_bounds__(FB) void k_oc_walk(OcDev* oc, const double* __restrict__ part, int np,
                                                double target, double tol) {
  if (oc->done) return;
  __shared__ double S[OC_NCAND], C[OC_NCAND];
  __shared__ OcFill fill;
  __shared__ int fdone;
  const int lane = threadIdx.x & (MGAR_WAVE - 1), wv = threadIdx.x / MGAR_WAVE;
  // the state thread 0 needs, read before the partials arrive
  double lo = 0.0, hi = 0.0, slo = 0.0, shi = 0.0, l1 = 0.0, l2 = 0.0, last = 0.0;
  int steps = 0;
  if (threadIdx.x == 0) {
    lo = oc->lo_known; hi = oc->hi_known; slo = oc->s_lo; shi = oc->s_hi;
    l1 = oc->l1; l2 = oc->l2; last = oc->lam_last; steps = oc->steps;
  }
  if (threadIdx.x < OC_NCAND) C[threadIdx.x] = oc->cand[threadIdx.x];
  if (wv < OC_NCAND) {
    constexpr int PK = (VMAXB + MGAR_WAVE - 1) / MGAR_WAVE;
    const double* pt = part + (long long)wv * np;
    double pv[PK];
#pragma unroll
    for (int k = 0; k < PK; ++k) {
      const int b = lane + k * MGAR_WAVE;
      pv[k] = b < np ? pt[b] : 0.0;
    }
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < PK; ++k) v += pv[k];
    v = wave_sum(v);
    if (lane == 0) S[wv] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 0; t < OC_NCAND; ++t) {
      const double c = C[t];
      if (S[t] > target) {
        if (c > lo) { lo = c; slo = S[t]; }
      } else if (c < hi) {
        hi = c; shi = S[t];
      }
    }
    int done = 0;
    for (;;) {
      if (!((l2 - l1) / (l1 + l2) > tol)) { done = 1; break; }
      const double m = 0.5 * (l2 + l1);
      if (m <= lo) l1 = m;
      else if (m >= hi) l2 = m;
      else break;
      last = m;
      ++steps;
    }
    oc->l1 = l1; oc->l2 = l2; oc->lam_last = last; oc->steps = steps;
    oc->lo_known = lo; oc->hi_known = hi; oc->s_lo = slo; oc->s_hi = shi; oc->done = done;
    fdone = done;
    if (!done) fill = oc_fill_params(l1, l2, lo, hi, slo, shi, target);
  }
  __syncthreads();
  if (!fdone && threadIdx.x < OC_NCAND)
    oc->cand[threadIdx.x] = oc_candidate(threadIdx.x, fill);
}

__global__ __launch_bounds__(VB) void k_oc_final(const double* __restrict__ x,
                                                 const double* __restrict__ dc,
                                                 const double* __restrict__ dv, long long n,
                                                 double move, const OcDev* __restrict__ oc,
                                                 double* __restrict__ xnew) {
  const double lam = oc->lam_last;
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
    const double xi = x[i];
    const double B = fmax(0.0, -dc[i]) / dv[i];
    const double v = xi * sqrt(B / lam);
    xnew[i] = fmax(0.0, fmax(xi - move, fmin(1.0, fmin(xi + move, v))));
  }
}

}  // namespace

void launch_simp(const double* xphys, double* k, long long n, double k0, double kmin, double penal,
                 hipStream_t s) {
  k_simp<<<nblocks(n), VB, 0, s>>>(xphys, k, n, k0, kmin, penal);
}

void launch_load(const Geo& g, const double* Qe, double* q, hipStream_t s) {
  if (g.dim == 2) k_load<2><<<node_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, Qe, q);
  else k_load<3><<<node_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, Qe, q);
}

void launch_filter_fwd(const Geo& g, const int* off, const double* w, int ntap, int hr, const double* x,
                       const double* invHs, double* y, hipStream_t s) {
  const size_t lds = sizeof(double) * (TBX + 2 * hr) * (TBY + 2 * hr) * (g.dim == 3 ? 2 * hr + 1 : 1) +
                     (sizeof(double) + sizeof(int)) * (size_t)ntap;
  if (g.ne * 8 < (1LL << 31) && hr >= 0 && hr <= 3)
    k_filter_lds<<<elem_grid(g), dim3(TBX, TBY, 1), lds, s>>>(g, off, w, ntap, hr, x, invHs, y);
  else if (g.ne * 8 < (1LL << 31))
    k_filter_b<<<elem_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, off, w, ntap, x, invHs, y);
  else
    k_filter<<<elem_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, off, w, ntap, x, invHs, y);
}

void launch_filter_hs(const Geo& g, const int* off, const double* w, int ntap, double* invHs,
                      hipStream_t s) {
  k_filter_hs<<<elem_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, off, w, ntap, invHs);
}

void launch_sens_elem(const Geo& g, const double* xphys, const double* T, const double* invHs,
                      double k0, double kmin, double penal, double* gout, hipStream_t s) {
  if (g.dim == 2)
    k_sens<2><<<elem_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, xphys, T, invHs, k0, kmin, penal, gout);
  else
    k_sens<3><<<elem_grid(g), dim3(TBX, TBY, 1), 0, s>>>(g, xphys, T, invHs, k0, kmin, penal, gout);
}

void launch_oc_init(OcDev* oc, double target, double hint, hipStream_t s) {
  k_oc_init<<<1, 1, 0, s>>>(oc, target, hint);
}

int launch_oc_pass(const double* x, const double* dc, const double* dv, long long n, double move,
                   const OcDev* oc, double* part, hipStream_t s) {
  const int nb = nblocks(n);
  k_oc_pass<<<nb, VB, 0, s>>>(x, dc, dv, n, move, oc, part);
  return nb;
}

void launch_oc_walk(OcDev* oc, const double* part, int np, double target, double tol,
                    hipStream_t s) {
  k_oc_walk<<<1, FB, 0, s>>>(oc, part, np, target, tol);
}

void launch_oc_final(const double* x, const double* dc, const double* dv, long long n, double move,
                     const OcDev* oc, double* xnew, hipStream_t s) {
  k_oc_final<<<nblocks(n), VB, 0, s>>>(x, dc, dv, n, move, oc, xnew);
}
