// Vector kernels: deterministic FP64 reductions, PCG updates, Gram-Schmidt and
// the reduced (reanalysis) system.
//
// Reductions are two-stage and order-fixed: every block writes one partial per
// value (wave64 shuffle tree, then LDS across waves), and a single-block
// finalize sums the partials in index order. Reruns are bitwise identical.
#include "mgar.h"
#include "mgar_launch.h"

namespace {

constexpr int VB = 256;          // threads per block for vector kernels
constexpr int VMAXB = 1024;      // maximum blocks (so at most 1024 partials)
constexpr int FB = 1024;         // finalize block size

template <typename TA, typename TB>
__global__ __launch_bounds__(VB) void k_dot(const TA* __restrict__ a,
                                            const TB* __restrict__ b, long long n,
                                            double* __restrict__ part,
                                            const int* __restrict__ done,
                                            unsigned* __restrict__ cnt, double* __restrict__ rout) {
  if (done && *done) return;
  __shared__ double sh[VB / MGAR_WAVE];
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    s += (double)a[i] * (double)b[i];
  s = block_sum(s, sh);
  if (cnt) grid_reduce(s, blockIdx.x, gridDim.x, part, cnt, rout, sh, nullptr);
  else if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ double sum_partials(const double* __restrict__ part, int n, double* sh) {
  return block_sum(thread_partials(part, n, threadIdx.x, blockDim.x), sh);
}

__global__ __launch_bounds__(FB) void k_finalize(const double* __restrict__ part, int n,
                                                 double* __restrict__ out,
                                                 const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[FB / MGAR_WAVE];
  const double s = sum_partials(part, n, sh);
  if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(FB) void k_cg_init(CgState* st, const double* __restrict__ pq, int nq,
                                                const double* __restrict__ pr, int nr, double tol,
                                                int cg_max) {
  __shared__ double sh[FB / MGAR_WAVE];
  const double qq = sum_partials(pq, nq, sh);
  const double rr = sum_partials(pr, nr, sh);
  if (threadIdx.x == 0) {
    st->qq = qq; st->rr = rr; st->rz[0] = st->rz[1] = 0.0; st->pw = 0.0;
    st->pwh[0] = st->pwh[1] = 0.0; st->flushed = -1;
    st->done = 0; st->iters = 0; st->converged = 0; st->it = 0;
    if (sqrt(rr) <= tol * sqrt(qq)) { st->done = 1; st->converged = 1; }
    else if (cg_max <= 0) { st->done = 1; }
  }
}

// Start (fresh) or continue a PCG run on a new residual r (partials of ||r||^2):
// the stopping reference becomes qq = qscale2 ||r||^2, so the run stops once
// ||r|| has dropped by tol sqrt(qscale2). Continuing keeps the iteration
// count, the r.z and p.w history and the direction buffers (the caller has
// replaced r by a more accurate residual of the same iterate); a fresh start
// clears them as k_cg_init does.
__global__ __launch_bounds__(FB) void k_cg_start(CgState* st, const double* __restrict__ pr, int nr,
                                                 double qscale2, int fresh, double tol, int cg_max) {
  __shared__ double sh[FB / MGAR_WAVE];
  const double rr = sum_partials(pr, nr, sh);
  if (threadIdx.x == 0) {
    if (fresh) {
      st->rz[0] = st->rz[1] = 0.0; st->pw = 0.0; st->pwh[0] = st->pwh[1] = 0.0;
      st->flushed = -1; st->it = 0;
    }
    const double qq = qscale2 * rr;
    st->qq = qq; st->rr = rr;
    st->done = 0; st->converged = 0; st->iters = st->it;
    if (sqrt(rr) <= tol * sqrt(qq)) { st->done = 1; st->converged = 1; }
    else if (st->it >= cg_max) { st->done = 1; }
  }
}

// rz of the current iteration: st->rz[it & 1] = sum of the partials
__global__ __launch_bounds__(FB) void k_finalize_rz(const double* __restrict__ part, int n,
                                                    CgState* __restrict__ st) {
  if (st->done) return;
  __shared__ double sh[FB / MGAR_WAVE];
  const double s = sum_partials(part, n, sh);
  if (threadIdx.x == 0) st->rz[st->it & 1] = s;
}

// p = z + beta p, beta = rz_k / rz_{k-1} (Fletcher-Reeves); p = z at k = 0.
// With rzp set, rz_k is first summed from its np block partials, by every
// block in the same order (so all blocks hold the same value), and block 0
// stores it to st->rz[k & 1]; otherwise st->rz[k & 1] already holds it.
template <typename T>
__global__ __launch_bounds__(VB) void k_p_update(const T* __restrict__ z, T* __restrict__ p,
                                                 long long n, CgState* __restrict__ st,
                                                 const double* __restrict__ rzp, int np) {
  __shared__ double sh[VB / MGAR_WAVE];
  // the state words and this thread's partials are read in one round
  const int dn = st->done, it = st->it;
  const double h0 = st->rz[0], h1 = st->rz[1];
  const double v = rzp ? thread_partials(rzp, np, threadIdx.x, VB) : 0.0;
  if (dn) return;
  double rz = 0.0;
  if (rzp) {
    rz = block_sum(v, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rz[it & 1] = rz;
  } else {
    rz = (it & 1) ? h1 : h0;
  }
  const T beta = (T)((it == 0) ? 0.0 : rz / (((it - 1) & 1) ? h1 : h0));
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    p[i] = (it == 0) ? z[i] : z[i] + beta * p[i];
}

// x += alpha p, r -= alpha w with alpha = rz / (p . w); ||r||^2 reduced in
// the same launch, and the last block applies the stopping test that precedes
// iteration it+1 (||r|| <= tol ||q||, or it+1 == cg_max). With pwp set, p . w
// is first summed from its npw block partials by every block (same order in
// each) and block 0 stores it to st->pw; otherwise st->pw already holds it.
// With p_odd set, the direction of an odd iteration is read from p_odd, and
// the x update is deferred by one iteration: an even iteration updates r only,
// the next (odd) one applies both directions to x, x += a_(it-1) p_(it-1) +
// a_it p_it, in that order (the same two updates; one pass over x instead of
// two). k_cg_flush applies a pending update once the loop stops.
template <typename T>
__global__ __launch_bounds__(VB) void k_cg_update(T* __restrict__ x, T* __restrict__ r,
                                                  const T* __restrict__ p_even,
                                                  const T* __restrict__ w, long long n,
                                                  CgState* __restrict__ st,
                                                  double* __restrict__ part,
                                                  unsigned* __restrict__ cnt, double tol,
                                                  int cg_max, const double* __restrict__ pwp,
                                                  int npw, const T* __restrict__ p_odd) {
  // the state words and this thread's partials are read in one round
  const int dn = st->done, it = st->it, flushed = st->flushed;
  const double rz0 = st->rz[0], rz1 = st->rz[1], pws = st->pw, pwh0 = st->pwh[0],
               pwh1 = st->pwh[1], qq = st->qq;
  const double pwv = pwp ? thread_partials(pwp, npw, threadIdx.x, VB) : 0.0;
  if (dn) return;
  const T* __restrict__ p = (p_odd && (it & 1)) ? p_odd : p_even;
  if (blockIdx.x == 0 && threadIdx.x == 0) st->itn = it + 1;   // for a fused stopping test
  __shared__ double sh[VB / MGAR_WAVE];
  double pw;
  if (pwp) {
    pw = block_sum(pwv, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->pw = pw;
  } else {
    pw = pws;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->pwh[it & 1] = pw;
  const T alpha = (T)(((it & 1) ? rz1 : rz0) / pw);
  double s = 0.0;
  if (p_odd) {
    const bool odd = it & 1;
    // the pending update of the previous (even) iteration
    // (left out when k_cg_flush has already applied it)
    const T alpha0 = (odd && flushed != it - 1)
                         ? (T)((((it - 1) & 1) ? rz1 : rz0) / (((it - 1) & 1) ? pwh1 : pwh0))
                         : T(0);
    for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
      if (odd) x[i] = (x[i] + alpha0 * p_even[i]) + alpha * p_odd[i];
      const T ri = r[i] - alpha * w[i];
      r[i] = ri;
      s += (double)ri * (double)ri;
    }
  } else {
    for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
      x[i] += alpha * p[i];
      const T ri = r[i] - alpha * w[i];
      r[i] = ri;
      s += (double)ri * (double)ri;
    }
  }
  s = block_sum(s, sh);
  if (!cnt) {
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    return;
  }
  double rr = 0.0;
  if (grid_reduce(s, blockIdx.x, gridDim.x, part, cnt, nullptr, sh, &rr) && threadIdx.x == 0) {
    st->rr = rr;
    st->it = it + 1;
    if (sqrt(rr) <= tol * sqrt(qq)) {
      st->done = 1; st->converged = 1; st->iters = it + 1;
    } else if (it + 1 >= cg_max) {
      st->done = 1; st->converged = 0; st->iters = it + 1;
    }
  }
}

// End of an iteration: it += 1, then the stopping test before the next one
// from the ||r||^2 partials of the update (||r|| <= tol ||q||, or it == cg_max).
__global__ __launch_bounds__(FB) void k_cg_check(CgState* st, const double* __restrict__ part,
                                                 int np, double tol, int cg_max) {
  if (st->done) return;
  __shared__ double sh[FB / MGAR_WAVE];
  const double rr = sum_partials(part, np, sh);
  if (threadIdx.x == 0) {
    const int it = st->it + 1;
    st->it = it;
    st->rr = rr;
    if (sqrt(rr) <= tol * sqrt(st->qq)) {
      st->done = 1; st->converged = 1; st->iters = it;
    } else if (it >= cg_max) {
      st->done = 1; st->converged = 0; st->iters = it;
    }
  }
}

// After a loop with deferred x updates (k_cg_update with p_odd): the update of
// the last iteration is still pending when that iteration was even. It is
// applied once: st->flushed records it, so a second flush and the next odd
// update of a continued run leave it out.
template <typename T>
__global__ __launch_bounds__(VB) void k_cg_flush(T* __restrict__ x, const T* __restrict__ p_even, long long n,
                                                 CgState* __restrict__ st) {
  const int k = st->it - 1;   // last completed iteration
  if (k < 0 || (k & 1) || st->flushed == k) return;
  const T alpha = (T)(st->rz[k & 1] / st->pwh[k & 1]);
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    x[i] += alpha * p_even[i];
  // no block of this launch reads st->flushed after its entry test above
  if (blockIdx.x == 0 && threadIdx.x == 0) st->flushed = k;
}

__global__ __launch_bounds__(VB) void k_copy(const double* __restrict__ a, double* __restrict__ b,
                                             long long n) {
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    b[i] = a[i];
}

// a[i] = v0 + dv * (i mod 97): deterministic non-constant fill for timing runs.
template <typename T>
__global__ __launch_bounds__(VB) void k_fill(T* __restrict__ a, long long n, float v0, float dv) {
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    a[i] = (T)(v0 + dv * (float)(i % 97));
}

__global__ __launch_bounds__(VB) void k_fill_bf16(uint16_t* __restrict__ a, long long n) {
  // BF16 values 0.25 .. 0.98 (exponent field of 0.5, varied mantissa)
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    a[i] = (uint16_t)(0x3E80u + (unsigned)(i % 97));
}

__global__ __launch_bounds__(VB) void k_scale_into(const double* __restrict__ a,
                                                   double* __restrict__ b, double alpha,
                                                   long long n) {
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    b[i] = alpha * a[i];
}

// ---- Gram-Schmidt in three passes per column (single design; FP64 columns in
// both precision forms). Column j (j >= 1) of R: pass 1 sums R_c . R_j (c < j)
// and R_j . R_j (and R_0 . R_0 for j = 1); pass 2 subtracts the projection
// onto the earlier columns and sums the same products of the result; pass 3
// subtracts the second (re-orthogonalisation) projection. Earlier columns stay
// unnormalised (with their squared norms nn[c]) until the last column's pass
// 3, which also normalises every column. The squared norm after the second
// projection is ||R_j'||^2 - sum_c c2_c^2 nn_c: exact for orthogonal R_c, and
// accurate since c2 is of round-off size. Drop rule: a column whose norm after
// projection is below 1e-10 of its norm before (or zero) is zeroed and left
// out.

// The nv (<= NVM) sums over np block partials laid out part[b * nv + v],
// formed the same way in every block of a launch (so every block holds the
// same values): thread t adds blocks t, t + nt, ... in order (the first U of
// them loaded together), each value is summed over the wave, then over the
// waves in order. out[v] (shared) for v < nv, valid in every thread on return.
// shm: (blockDim / 64) * NVM doubles of shared memory.
template <int NVM, int U>
__device__ inline void partial_sums(const double* __restrict__ part, int np, int nv, double* out, double* shm) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int nw = (nt + MGAR_WAVE - 1) / MGAR_WAVE;
  double acc[NVM], a[U][NVM];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int b = t + u * nt;
#pragma unroll
    for (int v = 0; v < NVM; ++v) a[u][v] = (b < np && v < nv) ? part[(long long)b * nv + v] : 0.0;
  }
#pragma unroll
  for (int v = 0; v < NVM; ++v) {
    acc[v] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) acc[v] += a[u][v];
  }
  for (int b = t + U * nt; b < np; b += nt)
#pragma unroll
    for (int v = 0; v < NVM; ++v)
      if (v < nv) acc[v] += part[(long long)b * nv + v];
#pragma unroll
  for (int v = 0; v < NVM; ++v) {
    const double w = wave_sum(acc[v]);
    if ((t & (MGAR_WAVE - 1)) == 0) shm[(t / MGAR_WAVE) * NVM + v] = w;
  }
  __syncthreads();
  if (t < nv) {
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += shm[w * NVM + t];
    out[t] = r;
  }
  __syncthreads();
}

// part[b * NV + v]: v < J: R_v . R_J; v = J: R_J . R_J; v = J + 1 (J = 1): R_0 . R_0
template <int J>
__global__ __launch_bounds__(VB) void k_gs_dots(const double* __restrict__ R, long long ld, long long n,
                                                double* __restrict__ part) {
  __shared__ double sh[VB / MGAR_WAVE];
  constexpr int NV = J + 1 + (J == 1 ? 1 : 0);
  double s[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) s[v] = 0.0;
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
    const double rj = R[J * ld + i];
#pragma unroll
    for (int c = 0; c < J; ++c) s[c] += R[c * ld + i] * rj;
    s[J] += rj * rj;
    if (J == 1) {
      const double r0 = R[i];
      s[NV - 1] += r0 * r0;
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double t = block_sum(s[v], sh);
    if (threadIdx.x == 0) part[blockIdx.x * NV + v] = t;
  }
}

// Pass 2: every block first forms pass 1's results from its partials (dpart,
// np blocks): n0[J]; for J = 1 also column 0's norms; c[q] = R_q . R_J / nn[q]
// (block 0 records them in md). Then R_J -= sum_q c[q] R_q, and partials of
// R_q . R_J' (q < J) and R_J' . R_J' into part.
template <int J>
__global__ __launch_bounds__(VB) void k_gs_proj(double* __restrict__ R, long long ld, long long n,
                                                MgarDev* md, const double* __restrict__ dpart, int np,
                                                double* __restrict__ part) {
  constexpr int NV1 = J + 1 + (J == 1 ? 1 : 0);
  __shared__ double sh[VB / MGAR_WAVE];
  __shared__ double shm[(VB / MGAR_WAVE) * NV1];
  __shared__ double v1[NV1];
  partial_sums<NV1, 4>(dpart, np, NV1, v1, shm);
  double nn[J], c[J];
  int act[J];
#pragma unroll
  for (int q = 0; q < J; ++q) {
    nn[q] = (J == 1) ? v1[NV1 - 1] : md->nn[q];
    act[q] = (J == 1) ? (nn[q] > 0.0 ? 1 : 0) : md->active[q];
    c[q] = act[q] ? v1[q] / nn[q] : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (J == 1) {
      md->n0[0] = nn[0];
      md->nn[0] = nn[0];
      md->active[0] = act[0];
    }
    md->n0[J] = v1[J];
    for (int q = 0; q < J; ++q) md->c[q] = c[q];
  }
  double s[J + 1];
#pragma unroll
  for (int q = 0; q <= J; ++q) s[q] = 0.0;
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
    double rc[J];
    double v = R[J * ld + i];
#pragma unroll
    for (int q = 0; q < J; ++q) {
      rc[q] = R[q * ld + i];
      v -= c[q] * rc[q];
    }
    R[J * ld + i] = v;
#pragma unroll
    for (int q = 0; q < J; ++q) s[q] += rc[q] * v;
    s[J] += v * v;
  }
#pragma unroll
  for (int q = 0; q <= J; ++q) {
    const double t = block_sum(s[q], sh);
    if (threadIdx.x == 0) part[blockIdx.x * (J + 1) + q] = t;
  }
}

// Pass 3: every block first forms pass 2's results from its partials (ppart,
// np blocks): c2[q] = R_q . R_J' / nn[q], nn[J] = ||R_J'||^2 - sum_q c2_q^2
// nn[q] and the drop decision; for J = 0 (a single column, ppart holding the
// partials of ||R_0||^2) column 0's norms. Block 0 records them in md. Then
// R_J -= sum_q c2[q] R_q (J >= 1); with LAST, every column q <= J is scaled
// by 1 / sqrt(nn[q]) (0 for dropped columns).
template <int J, bool LAST>
__global__ __launch_bounds__(VB) void k_gs_fix(double* __restrict__ R, long long ld, long long n,
                                               MgarDev* md, const double* __restrict__ ppart, int np) {
  __shared__ double shm[(VB / MGAR_WAVE) * (J + 1)];
  __shared__ double v2[J + 1];
  partial_sums<J + 1, 4>(ppart, np, J + 1, v2, shm);
  double c2[J > 0 ? J : 1], sc[J + 1];
  double nnJ;
  int actJ;
  if (J == 0) {
    nnJ = v2[0];
    actJ = nnJ > 0.0 ? 1 : 0;
  } else {
    nnJ = v2[J];
#pragma unroll
    for (int q = 0; q < J; ++q) {
      const double nq = md->nn[q];
      c2[q] = md->active[q] ? v2[q] / nq : 0.0;
      nnJ -= c2[q] * c2[q] * nq;
    }
    nnJ = nnJ > 0.0 ? nnJ : 0.0;
    const double n0 = md->n0[J];
    actJ = (n0 > 0.0 && nnJ >= 1e-20 * n0) ? 1 : 0;
    if (!actJ) nnJ = 0.0;
  }
#pragma unroll
  for (int q = 0; q < J; ++q) sc[q] = (md->active[q] && md->nn[q] > 0.0) ? 1.0 / sqrt(md->nn[q]) : 0.0;
  sc[J] = (actJ && nnJ > 0.0) ? 1.0 / sqrt(nnJ) : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (J == 0) md->n0[0] = nnJ;
    for (int q = 0; q < J; ++q) md->c2[q] = c2[q];
    md->nn[J] = nnJ;
    md->active[J] = actJ;
  }
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
    double rc[J > 0 ? J : 1];
    double v = R[J * ld + i];
#pragma unroll
    for (int q = 0; q < J; ++q) {
      rc[q] = R[q * ld + i];
      v -= c2[q] * rc[q];
    }
    if (LAST) {
#pragma unroll
      for (int q = 0; q < J; ++q) R[q * ld + i] = rc[q] * sc[q];
      R[J * ld + i] = v * sc[J];
    } else {
      R[J * ld + i] = v;
    }
  }
}

// Gram products of the reduced system (Eq 19-20), K_R[a][b] = Q_a . W_b
// (a <= b), q_R[a] = Q_a . q, and ||q||^2, on the matrix cores. With
// A = [Q_0 .. Q_{M-1}, q] and B = [W_0 .. W_{M-1}, q] (N x (M+1) each),
// G = A^T B is a product whose inner dimension is the node index. One
// v_mfma_f64_16x16x4f64 takes a 16 x 4 operand from each side: lane l
// supplies row l % 16 at inner index l / 16 (lane layout checked on gfx950).
// Its 16 rows carry NG = 16 / (M + 1) node groups side by side: row
// g (M + 1) + a is column a of A (or B) over the nodes 4 g .. 4 g + 3 of the
// instruction's span of 4 NG nodes (rows past NG (M + 1) are zero). The
// diagonal blocks of the 16 x 16 result, D[g (M+1) + a][g (M+1) + b], are the
// products over group g's nodes; the off-diagonal blocks pair different nodes
// and are not used. Lane l holds D rows 4 r + l / 16, r = 0..3, of column
// l % 16. Per block G[a][b] = sum over waves, then groups, of the diagonal
// blocks, written as M(M+1)/2 + M + 1 values: the upper triangle of K_R row by
// row, then q_R, then ||q||^2 (summed over the blocks by k_combine).
typedef double mgar_d4 __attribute__((ext_vector_type(4)));
constexpr int GRAM_GROUP = 4;   // instructions whose loads are issued together

template <int M>
__global__ __launch_bounds__(VB) void k_gram_mfma(const double* __restrict__ Q, const double* __restrict__ W,
                                                  const double* __restrict__ q, long long ld, long long n,
                                                  double* __restrict__ part) {
  constexpr int NW = VB / MGAR_WAVE;
  constexpr int NV = M * (M + 1) / 2 + M + 1;
  constexpr int NG = 16 / (M + 1);
  constexpr int SPAN = 4 * NG;
  __shared__ double G[NW][16][17];
  const int lane = threadIdx.x & (MGAR_WAVE - 1), wid = threadIdx.x / MGAR_WAVE;
  const int row = lane & 15, kk = lane >> 4;
  const int col = row % (M + 1), grp = row / (M + 1);
  const bool live = grp < NG;
  const double* pa = live ? (col < M ? Q + col * ld : q) : nullptr;
  const double* pb = live ? (col < M ? W + col * ld : q) : nullptr;
  const int off = 4 * grp + kk;
  mgar_d4 d = {0.0, 0.0, 0.0, 0.0};
  const long long nstep = (n + SPAN - 1) / SPAN;
  const long long waves = (long long)gridDim.x * NW;
  // a wave's instructions (steps c, c + waves, ...) in the plain grid-stride
  // order, the loads of GRAM_GROUP of them issued together
  for (long long c0 = (long long)blockIdx.x * NW + wid; c0 < nstep; c0 += GRAM_GROUP * waves) {
    double av[GRAM_GROUP], bv[GRAM_GROUP];
#pragma unroll
    for (int u = 0; u < GRAM_GROUP; ++u) {
      const long long node = (c0 + u * waves) * SPAN + off;
      const bool in = live && node < n;
      av[u] = in ? pa[node] : 0.0;
      bv[u] = in ? pb[node] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < GRAM_GROUP; ++u) d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], d, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) G[wid][4 * r + kk][row] = d[r];
  __syncthreads();
  if (threadIdx.x < NV) {
    const int v = threadIdx.x;
    int a = 0, b = 0;
    if (v < M * (M + 1) / 2) {          // upper triangle, row by row
      int rem = v;
      while (rem >= M - a) { rem -= M - a; ++a; }
      b = a + rem;
    } else if (v < NV - 1) {            // q_R
      a = v - M * (M + 1) / 2;
      b = M;
    } else {                            // ||q||^2
      a = M;
      b = M;
    }
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
      for (int g = 0; g < NG; ++g) s += G[w][g * (M + 1) + a][g * (M + 1) + b];
    part[blockIdx.x * NV + v] = s;
  }
}

// Solve K_R y = q_R over the active columns by Cholesky (m <= 8, one thread);
// KR is row-major with leading dimension MGAR_MAXB.
__device__ void reduced_solve(const int* active, const double* KR, const double* qR, int m, double* y,
                              int* fail) {
  double L[MGAR_MAXB][MGAR_MAXB];
  double rhs[MGAR_MAXB];
  int idx[MGAR_MAXB];
  int na = 0;
  for (int a = 0; a < m; ++a)
    if (active[a]) idx[na++] = a;
  for (int a = 0; a < m; ++a) y[a] = 0.0;
  *fail = 0;
  for (int a = 0; a < na; ++a) {
    rhs[a] = qR[idx[a]];
    for (int b = 0; b < na; ++b) L[a][b] = KR[idx[a] * MGAR_MAXB + idx[b]];
  }
  for (int j = 0; j < na; ++j) {
    double d = L[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) { *fail = 1; return; }
    d = sqrt(d);
    L[j][j] = d;
    for (int i = j + 1; i < na; ++i) {
      double s = L[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = s / d;
    }
  }
  double z[MGAR_MAXB];
  for (int i = 0; i < na; ++i) {
    double s = rhs[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
    z[i] = s / L[i][i];
  }
  for (int i = na - 1; i >= 0; --i) {
    double s = z[i];
    for (int k = i + 1; k < na; ++k) s -= L[k][i] * y[idx[k]];
    y[idx[i]] = s / L[i][i];
  }
}

__device__ void reduced_solve(const MgarDev* md, int m, double* y, int* fail) {
  reduced_solve(md->active, md->KR, md->qR, m, y, fail);
}

// Every block first sums the Gram partials (gpart, gnp blocks; layout of
// k_gram_mfma) into K_R, q_R and ||q||^2 and solves the reduced system
// (redundantly per block, the same values in each; block 0 records them in
// md); then t = Q y, res = W y - q, partial ||res||^2.
template <int M>
__global__ __launch_bounds__(VB) void k_combine(const double* __restrict__ Q,
                                                const double* __restrict__ W,
                                                const double* __restrict__ q, long long ld,
                                                long long n, MgarDev* md, double* __restrict__ t,
                                                double* __restrict__ part, double* __restrict__ rq,
                                                const double* __restrict__ gpart, int gnp) {
  constexpr int NV = M * (M + 1) / 2 + M + 1;
  __shared__ double sh[VB / MGAR_WAVE];
  __shared__ double shm[(VB / MGAR_WAVE) * NV];
  __shared__ double gv[NV];
  __shared__ double ys[MGAR_MAXB];
  __shared__ double KR[MGAR_MAXB * MGAR_MAXB], qR[MGAR_MAXB];
  __shared__ int act[MGAR_MAXB];
  partial_sums<NV, (NV <= 16 ? 4 : 1)>(gpart, gnp, NV, gv, shm);
  if (threadIdx.x < M * M) {
    // entry (a, b) of K_R from the packed upper triangle
    const int a = threadIdx.x / M, b = threadIdx.x % M;
    const int r = a < b ? a : b, c = a < b ? b : a;
    KR[a * MGAR_MAXB + b] = gv[r * M - r * (r - 1) / 2 + (c - r)];
  }
  if (threadIdx.x < M) {
    qR[threadIdx.x] = gv[M * (M + 1) / 2 + threadIdx.x];
    act[threadIdx.x] = md->active[threadIdx.x];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double y[MGAR_MAXB];
    int fail;
    reduced_solve(act, KR, qR, M, y, &fail);
    for (int a = 0; a < MGAR_MAXB; ++a) ys[a] = (a < M) ? y[a] : 0.0;
    if (blockIdx.x == 0) {
      for (int a = 0; a < M; ++a) {
        for (int b = 0; b < M; ++b) md->KR[a * MGAR_MAXB + b] = KR[a * MGAR_MAXB + b];
        md->qR[a] = qR[a];
        md->y[a] = y[a];
      }
      md->qq = gv[NV - 1];
      md->spd_fail = fail;
    }
  }
  __syncthreads();
  double y[M];
#pragma unroll
  for (int a = 0; a < M; ++a) y[a] = ys[a];
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
    double ti = 0.0, wi = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      ti += y[a] * Q[a * ld + i];
      wi += y[a] * W[a * ld + i];
    }
    t[i] = ti;
    const double ri = wi - q[i];
    if (rq) rq[i] = -ri;
    s += ri * ri;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Round to BF16 with round-to-nearest-even, going through FP32 exactly as a
// float -> bfloat16 conversion of an FP32 value does (NaN kept quiet).
__device__ inline uint16_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7fffu + lsb) >> 16);
}

__global__ __launch_bounds__(VB) void k_cast_bf16(const double* __restrict__ a, uint16_t* __restrict__ b,
                                                  long long n) {
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    b[i] = f32_to_bf16_rne((float)a[i]);
}

__global__ __launch_bounds__(VB) void k_cast_f32(const double* __restrict__ a, float* __restrict__ b,
                                                 long long n) {
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    b[i] = (float)a[i];
}

// x += d with d in FP32 and x in FP64 (a segment's correction folded into x).
__global__ __launch_bounds__(VB) void k_add_f32(double* __restrict__ x, const float* __restrict__ d,
                                                long long n) {
  for (long long i = blockIdx.x * (long long)VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB)
    x[i] += (double)d[i];
}

// ---------------------------------------------------------------------------
// Batched vector kernels over several designs: one work item per design (its
// finest grid), the design's nodes at item.off of the concatenated vectors,
// and its partials in blocks item.first .. item.first + item.nblk - 1.
__device__ inline int vb_find(const BItem* __restrict__ items, int nit, int blk) {
  int lo = 0, hi = nit - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ inline bool vb_skip(const int* skip, int sstride, int design) {
  return skip && skip[(long long)design * sstride] != 0;
}

template <typename T>
__global__ __launch_bounds__(VB) void kb_dot(const BItem* __restrict__ items, int nit,
                                             const T* __restrict__ a, const T* __restrict__ b,
                                             double* __restrict__ part, const int* __restrict__ skip,
                                             int sstride) {
  __shared__ double sh[VB / MGAR_WAVE];
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  if (vb_skip(skip, sstride, it.design)) return;
  const long long n = it.g.nn;
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  const double s = block_sum(i < n ? (double)a[it.off + i] * (double)b[it.off + i] : 0.0, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// one block per item: out[d * ostride + v (+ (itsel[d*sstride] & 1))] = sum of
// the item's partials of value v
__global__ __launch_bounds__(FB) void kb_finalize(const BItem* __restrict__ items,
                                                  const double* __restrict__ part, int nv,
                                                  double* __restrict__ out, int ostride,
                                                  const int* __restrict__ itsel,
                                                  const int* __restrict__ skip, int sstride) {
  __shared__ double sh[FB / MGAR_WAVE];
  const BItem& it = items[blockIdx.x];
  if (vb_skip(skip, sstride, it.design)) return;
  const int shift = itsel ? (itsel[(long long)it.design * sstride] & 1) : 0;
  for (int v = 0; v < nv; ++v) {
    double s = 0.0;
    for (int b = threadIdx.x; b < it.nblk; b += FB) s += part[(long long)(it.first + b) * nv + v];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[(long long)it.design * ostride + v + shift] = s;
  }
}

// Stopping test before iteration 0 (same rule as k_cg_init); designs with
// keep_done[d] != 0 stay done (their reduced solution was accepted).
__global__ __launch_bounds__(FB) void kb_cg_init(const BItem* __restrict__ items, BCgState* st,
                                                 const double* __restrict__ pq,
                                                 const double* __restrict__ pr, double tol, int cg_max,
                                                 const int* __restrict__ keep_done) {
  __shared__ double sh[FB / MGAR_WAVE];
  const BItem& it = items[blockIdx.x];
  const int d = it.design;
  double qq = 0.0, rr = 0.0;
  for (int b = threadIdx.x; b < it.nblk; b += FB) {
    qq += pq[it.first + b];
    rr += pr[it.first + b];
  }
  qq = block_sum(qq, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    BCgState& s = st[d];
    s.qq = qq; s.rr = rr; s.rz[0] = s.rz[1] = 0.0; s.pw = 0.0;
    s.it = 0; s.done = 0; s.conv = 0;
    if (keep_done && keep_done[d]) { s.done = 1; s.conv = 1; }
    else if (sqrt(rr) <= tol * sqrt(qq)) { s.done = 1; s.conv = 1; }
    else if (cg_max <= 0) { s.done = 1; }
  }
}

template <typename T>
__global__ __launch_bounds__(VB) void kb_p_update(const BItem* __restrict__ items, int nit,
                                                  const T* __restrict__ z, T* __restrict__ p,
                                                  const BCgState* __restrict__ st) {
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  const BCgState& s = st[it.design];
  if (s.done) return;
  const int k = s.it;
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  if (i >= it.g.nn) return;
  const long long n = it.off + i;
  if (k == 0) p[n] = z[n];
  else p[n] = z[n] + (T)(s.rz[k & 1] / s.rz[(k - 1) & 1]) * p[n];
}

template <typename T>
__global__ __launch_bounds__(VB) void kb_cg_update(const BItem* __restrict__ items, int nit,
                                                   T* __restrict__ x, T* __restrict__ r,
                                                   const T* __restrict__ p, const T* __restrict__ w,
                                                   const BCgState* __restrict__ st,
                                                   double* __restrict__ part) {
  __shared__ double sh[VB / MGAR_WAVE];
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  const BCgState& s = st[it.design];
  if (s.done) return;
  const T alpha = (T)(s.rz[s.it & 1] / s.pw);
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < it.g.nn) {
    const long long n = it.off + i;
    x[n] += alpha * p[n];
    const T ri = r[n] - alpha * w[n];
    r[n] = ri;
    v = (double)ri * (double)ri;
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// one block per item: ||r||^2 from the update's partials, then the stopping
// test that precedes the next iteration
__global__ __launch_bounds__(FB) void kb_cg_check(const BItem* __restrict__ items, BCgState* st,
                                                  const double* __restrict__ part, double tol,
                                                  int cg_max) {
  __shared__ double sh[FB / MGAR_WAVE];
  const BItem& it = items[blockIdx.x];
  BCgState& s = st[it.design];
  if (s.done) return;
  double rr = 0.0;
  for (int b = threadIdx.x; b < it.nblk; b += FB) rr += part[it.first + b];
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    s.rr = rr;
    s.it += 1;
    if (sqrt(rr) <= tol * sqrt(s.qq)) { s.done = 1; s.conv = 1; }
    else if (s.it >= cg_max) { s.done = 1; s.conv = 0; }
  }
}

template <int NC>
__global__ __launch_bounds__(VB) void kb_multidot(const BItem* __restrict__ items, int nit,
                                                  const double* __restrict__ Q, long long ld,
                                                  const double* __restrict__ v,
                                                  double* __restrict__ part) {
  __shared__ double sh[VB / MGAR_WAVE];
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  const bool in = i < it.g.nn;
  const long long n = it.off + i;
  const double vi = in ? v[n] : 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double s = block_sum(in ? Q[c * ld + n] * vi : 0.0, sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * NC + c] = s;
  }
}

template <int NC>
__global__ __launch_bounds__(VB) void kb_gs_update(const BItem* __restrict__ items, int nit,
                                                   double* __restrict__ v, const double* __restrict__ Q,
                                                   long long ld, const MgarDev* __restrict__ md) {
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  if (i >= it.g.nn) return;
  const long long n = it.off + i;
  const double* c = md[it.design].c;
  double s = v[n];
#pragma unroll
  for (int j = 0; j < NC; ++j) s -= c[j] * Q[j * ld + n];
  v[n] = s;
}

__global__ __launch_bounds__(VB) void kb_gs_normalize(const BItem* __restrict__ items, int nit,
                                                      double* __restrict__ v, MgarDev* md, int col,
                                                      const double* __restrict__ nrm2, int nstride) {
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  MgarDev& m = md[it.design];
  const double n0 = sqrt(m.n0[col]);
  const double n1 = sqrt(nrm2[(long long)it.design * nstride]);
  const bool keep = (n0 > 0.0) && (n1 >= 1e-10 * n0);
  const double sc = keep ? 1.0 / n1 : 0.0;
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  if (i < it.g.nn) {
    const long long n = it.off + i;
    v[n] = keep ? v[n] * sc : 0.0;
  }
  if (blockIdx.x == it.first && threadIdx.x == 0) m.active[col] = keep ? 1 : 0;
}

template <int M>
__global__ __launch_bounds__(VB) void kb_gram(const BItem* __restrict__ items, int nit,
                                              const double* __restrict__ Q, const double* __restrict__ W,
                                              const double* __restrict__ q, long long ld,
                                              double* __restrict__ part) {
  __shared__ double sh[VB / MGAR_WAVE];
  constexpr int NV = M * (M + 1) / 2 + M;
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  const bool in = i < it.g.nn;
  const long long n = it.off + i;
  double qa[M], wa[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    qa[a] = in ? Q[a * ld + n] : 0.0;
    wa[a] = in ? W[a * ld + n] : 0.0;
  }
  const double qi = in ? q[n] : 0.0;
  double s[NV];
  int idx = 0;
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int b = a; b < M; ++b) s[idx++] = qa[a] * wa[b];
#pragma unroll
  for (int a = 0; a < M; ++a) s[idx + a] = qa[a] * qi;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double t = block_sum(s[c], sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * NV + c] = t;
  }
}

__global__ __launch_bounds__(FB) void kb_gram_finalize(const BItem* __restrict__ items,
                                                       const double* __restrict__ part, int m,
                                                       MgarDev* md) {
  __shared__ double sh[FB / MGAR_WAVE];
  const BItem& it = items[blockIdx.x];
  MgarDev& g = md[it.design];
  const int nv = m * (m + 1) / 2 + m;
  int idx = 0;
  for (int a = 0; a < m; ++a)
    for (int b = a; b < m; ++b, ++idx) {
      double s = 0.0;
      for (int k = threadIdx.x; k < it.nblk; k += FB) s += part[(long long)(it.first + k) * nv + idx];
      s = block_sum(s, sh);
      if (threadIdx.x == 0) {
        g.KR[a * MGAR_MAXB + b] = s;
        g.KR[b * MGAR_MAXB + a] = s;
      }
    }
  for (int a = 0; a < m; ++a) {
    double s = 0.0;
    for (int k = threadIdx.x; k < it.nblk; k += FB) s += part[(long long)(it.first + k) * nv + idx + a];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) g.qR[a] = s;
  }
}

template <int M>
__global__ __launch_bounds__(VB) void kb_combine(const BItem* __restrict__ items, int nit,
                                                 const double* __restrict__ Q,
                                                 const double* __restrict__ W,
                                                 const double* __restrict__ q, long long ld,
                                                 MgarDev* md, double* __restrict__ t,
                                                 double* __restrict__ part) {
  __shared__ double sh[VB / MGAR_WAVE];
  __shared__ double ys[MGAR_MAXB];
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  MgarDev& g = md[it.design];
  if (threadIdx.x == 0) {
    double y[MGAR_MAXB];
    int fail;
    reduced_solve(&g, M, y, &fail);
    for (int a = 0; a < MGAR_MAXB; ++a) ys[a] = (a < M) ? y[a] : 0.0;
    if (blockIdx.x == it.first) {
      for (int a = 0; a < M; ++a) g.y[a] = y[a];
      g.spd_fail = fail;
    }
  }
  __syncthreads();
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < it.g.nn) {
    const long long n = it.off + i;
    double ti = 0.0, wi = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      ti += ys[a] * Q[a * ld + n];
      wi += ys[a] * W[a * ld + n];
    }
    t[n] = ti;
    const double ri = wi - q[n];
    s = ri * ri;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void kb_decide(const BItem* __restrict__ items, int nit, MgarDev* md, BCgState* st,
                          double eps, int* __restrict__ keep, int* __restrict__ path,
                          double* __restrict__ res_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nit) return;
  const int d = items[k].design;
  const MgarDev& g = md[d];
  const double res = (g.qq > 0.0) ? sqrt(g.res2 / g.qq) : 0.0;
  res_out[d] = res;
  const bool acc = !g.spd_fail && res <= eps;
  keep[d] = acc ? 1 : 0;
  path[d] = acc ? MGAR_PATH_ACCEPT : MGAR_PATH_FALLBACK;
  if (acc) { st[d].done = 1; st[d].conv = 1; st[d].it = 0; }
}

template <typename T>
__global__ __launch_bounds__(VB) void kb_copy_cells(const BItem* __restrict__ items, int nit,
                                                    const T* __restrict__ a, T* __restrict__ b,
                                                    const int* __restrict__ skip, int sstride) {
  const BItem& it = items[vb_find(items, nit, blockIdx.x)];
  if (vb_skip(skip, sstride, it.design)) return;
  const long long i = (long long)(blockIdx.x - it.first) * blockDim.x + threadIdx.x;
  if (i < it.g.ne) b[it.eoff + i] = a[it.eoff + i];
}

#define MGAR_DISPATCH_M(m, CALL)                                    \
  switch (m) {                                                      \
    case 1: CALL(1); break; case 2: CALL(2); break;                 \
    case 3: CALL(3); break; case 4: CALL(4); break;                 \
    case 5: CALL(5); break; case 6: CALL(6); break;                 \
    case 7: CALL(7); break; default: CALL(8); break;                \
  }

}  // namespace

int vec_num_blocks(long long n) {
  long long nb = (n + VB - 1) / VB;
  if (nb > VMAXB) nb = VMAXB;
  if (nb < 1) nb = 1;
  return (int)nb;
}

template <typename TA, typename TB>
int launch_dot_t(const TA* a, const TB* b, long long n, double* part, const int* done, hipStream_t s,
                 unsigned* cnt, double* rout) {
  const int nb = vec_num_blocks(n);
  k_dot<TA, TB><<<nb, VB, 0, s>>>(a, b, n, part, done, cnt, rout);
  return nb;
}
template int launch_dot_t<double, double>(const double*, const double*, long long, double*, const int*,
                                          hipStream_t, unsigned*, double*);
template int launch_dot_t<float, float>(const float*, const float*, long long, double*, const int*,
                                        hipStream_t, unsigned*, double*);

int launch_dot(const double* a, const double* b, long long n, double* part, const int* done,
               hipStream_t s, unsigned* cnt, double* rout) {
  return launch_dot_t<double, double>(a, b, n, part, done, s, cnt, rout);
}

void launch_finalize(const double* part, int n, double* out, const int* done, hipStream_t s) {
  k_finalize<<<1, FB, 0, s>>>(part, n, out, done);
}

void launch_finalize_rz(const double* part, int n, CgState* st, hipStream_t s) {
  k_finalize_rz<<<1, FB, 0, s>>>(part, n, st);
}

void launch_cg_check(CgState* st, const double* part, int np, double tol, int cg_max, hipStream_t s) {
  k_cg_check<<<1, FB, 0, s>>>(st, part, np, tol, cg_max);
}

void launch_cg_init(CgState* st, const double* part_qq, int nq, const double* part_rr, int nr,
                    double tol, int cg_max, hipStream_t s) {
  k_cg_init<<<1, FB, 0, s>>>(st, part_qq, nq, part_rr, nr, tol, cg_max);
}

void launch_cg_start(CgState* st, const double* part_rr, int nr, double qscale2, bool fresh, double tol,
                     int cg_max, hipStream_t s) {
  k_cg_start<<<1, FB, 0, s>>>(st, part_rr, nr, qscale2, fresh ? 1 : 0, tol, cg_max);
}

template <typename T>
void launch_p_update_t(const T* z, T* p, long long n, CgState* st, hipStream_t s, const double* rzp,
                       int np) {
  k_p_update<T><<<vec_num_blocks(n), VB, 0, s>>>(z, p, n, st, rzp, np);
}
template void launch_p_update_t<double>(const double*, double*, long long, CgState*, hipStream_t,
                                        const double*, int);
template void launch_p_update_t<float>(const float*, float*, long long, CgState*, hipStream_t,
                                       const double*, int);

void launch_p_update(const double* z, double* p, long long n, CgState* st, hipStream_t s,
                     const double* rzp, int np) {
  launch_p_update_t<double>(z, p, n, st, s, rzp, np);
}

template <typename T>
int launch_cg_update_t(T* x, T* r, const T* p, const T* w, long long n, CgState* st, double* part,
                       unsigned* cnt, double tol, int cg_max, hipStream_t s, const double* pwp, int npw,
                       const T* p_odd) {
  const int nb = vec_num_blocks(n);
  k_cg_update<T><<<nb, VB, 0, s>>>(x, r, p, w, n, st, part, cnt, tol, cg_max, pwp, npw, p_odd);
  return nb;
}
template int launch_cg_update_t<double>(double*, double*, const double*, const double*, long long,
                                        CgState*, double*, unsigned*, double, int, hipStream_t,
                                        const double*, int, const double*);
template int launch_cg_update_t<float>(float*, float*, const float*, const float*, long long,
                                       CgState*, double*, unsigned*, double, int, hipStream_t,
                                       const double*, int, const float*);

template <typename T>
void launch_cg_flush_t(T* x, const T* p_even, long long n, CgState* st, hipStream_t s) {
  k_cg_flush<T><<<vec_num_blocks(n), VB, 0, s>>>(x, p_even, n, st);
}
template void launch_cg_flush_t<double>(double*, const double*, long long, CgState*, hipStream_t);
template void launch_cg_flush_t<float>(float*, const float*, long long, CgState*, hipStream_t);

int launch_cg_update(double* x, double* r, const double* p, const double* w, long long n,
                     CgState* st, double* part, unsigned* cnt, double tol, int cg_max, hipStream_t s,
                     const double* pwp, int npw, const double* p_odd) {
  return launch_cg_update_t<double>(x, r, p, w, n, st, part, cnt, tol, cg_max, s, pwp, npw, p_odd);
}

void launch_copy(const double* a, double* b, long long n, hipStream_t s) {
  k_copy<<<vec_num_blocks(n), VB, 0, s>>>(a, b, n);
}

template <typename T>
void launch_fill_t(T* a, long long n, float v0, float dv, hipStream_t s) {
  k_fill<T><<<vec_num_blocks(n), VB, 0, s>>>(a, n, v0, dv);
}
template void launch_fill_t<double>(double*, long long, float, float, hipStream_t);
template void launch_fill_t<float>(float*, long long, float, float, hipStream_t);

void launch_fill_bf16(uint16_t* a, long long n, hipStream_t s) {
  k_fill_bf16<<<vec_num_blocks(n), VB, 0, s>>>(a, n);
}

void launch_scale_into(const double* a, double* b, double alpha, long long n, hipStream_t s) {
  k_scale_into<<<vec_num_blocks(n), VB, 0, s>>>(a, b, alpha, n);
}

int launch_gram(const double* Q, const double* W, const double* q, int m, long long ld,
                long long n, double* part, hipStream_t s) {
  const int nb = vec_num_blocks(n);
#define CALL_G(M) k_gram_mfma<M><<<nb, VB, 0, s>>>(Q, W, q, ld, n, part)
  MGAR_DISPATCH_M(m, CALL_G)
#undef CALL_G
  return nb;
}

void launch_gs_fused(double* R, int m, long long ld, long long n, MgarDev* md, double* part, double* part2,
                     hipStream_t s) {
  const int nb = vec_num_blocks(n);
  if (m == 1) {
    k_gs_dots<0><<<nb, VB, 0, s>>>(R, ld, n, part);
    k_gs_fix<0, true><<<nb, VB, 0, s>>>(R, ld, n, md, part, nb);
    return;
  }
  // pass 1 partials in part, pass 2 partials in part2 (pass 2 reads part)
  for (int j = 1; j < m; ++j) {
    const bool last = j == m - 1;
#define GS_J(J)                                                                  \
  case J:                                                                        \
    k_gs_dots<J><<<nb, VB, 0, s>>>(R, ld, n, part);                              \
    k_gs_proj<J><<<nb, VB, 0, s>>>(R, ld, n, md, part, nb, part2);               \
    if (last) k_gs_fix<J, true><<<nb, VB, 0, s>>>(R, ld, n, md, part2, nb);      \
    else k_gs_fix<J, false><<<nb, VB, 0, s>>>(R, ld, n, md, part2, nb);          \
    break;
    switch (j) { GS_J(1) GS_J(2) GS_J(3) GS_J(4) GS_J(5) GS_J(6) default: GS_J(7) }
#undef GS_J
  }
}

int launch_combine(const double* Q, const double* W, const double* q, int m, long long ld,
                   long long n, MgarDev* md, double* t, double* part, hipStream_t s, double* rq,
                   const double* gpart, int gnp) {
  const int nb = vec_num_blocks(n);
#define CALL_C(M) k_combine<M><<<nb, VB, 0, s>>>(Q, W, q, ld, n, md, t, part, rq, gpart, gnp)
  MGAR_DISPATCH_M(m, CALL_C)
#undef CALL_C
  return nb;
}

void launch_cast_bf16(const double* a, uint16_t* b, long long n, hipStream_t s) {
  k_cast_bf16<<<vec_num_blocks(n), VB, 0, s>>>(a, b, n);
}

void launch_cast_f32(const double* a, float* b, long long n, hipStream_t s) {
  k_cast_f32<<<vec_num_blocks(n), VB, 0, s>>>(a, b, n);
}

void launch_add_f32(double* x, const float* d, long long n, hipStream_t s) {
  k_add_f32<<<vec_num_blocks(n), VB, 0, s>>>(x, d, n);
}

void launch_copy_u16(const uint16_t* a, uint16_t* b, long long n, hipStream_t s) {
  (void)hipMemcpyAsync(b, a, sizeof(uint16_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
}

// ---------------------------------------------------------------- batched launchers

template <typename T>
void launch_bdot_t(const BItem* items, int nit, int nblk, int bs, const T* a, const T* b, double* part,
                   const int* skip, int sstride, hipStream_t s) {
  if (nblk > 0) kb_dot<T><<<nblk, bs, 0, s>>>(items, nit, a, b, part, skip, sstride);
}
template void launch_bdot_t<float>(const BItem*, int, int, int, const float*, const float*, double*, const int*,
                                   int, hipStream_t);
void launch_bdot(const BItem* items, int nit, int nblk, int bs, const double* a, const double* b,
                 double* part, const int* skip, int sstride, hipStream_t s) {
  launch_bdot_t<double>(items, nit, nblk, bs, a, b, part, skip, sstride, s);
}
void launch_bfinalize(const BItem* items, int nit, const double* part, int nv, double* out,
                      int ostride, const int* itsel, const int* skip, int sstride, hipStream_t s) {
  if (nit > 0) kb_finalize<<<nit, FB, 0, s>>>(items, part, nv, out, ostride, itsel, skip, sstride);
}
void launch_bcg_init(const BItem* items, int nit, BCgState* st, const double* part_qq,
                     const double* part_rr, double tol, int cg_max, const int* keep_done,
                     hipStream_t s) {
  if (nit > 0) kb_cg_init<<<nit, FB, 0, s>>>(items, st, part_qq, part_rr, tol, cg_max, keep_done);
}
template <typename T>
void launch_bp_update_t(const BItem* items, int nit, int nblk, int bs, const T* z, T* p, const BCgState* st,
                        hipStream_t s) {
  if (nblk > 0) kb_p_update<T><<<nblk, bs, 0, s>>>(items, nit, z, p, st);
}
template void launch_bp_update_t<float>(const BItem*, int, int, int, const float*, float*, const BCgState*,
                                        hipStream_t);
template <typename T>
void launch_bcg_update_t(const BItem* items, int nit, int nblk, int bs, T* x, T* r, const T* p, const T* w,
                         const BCgState* st, double* part, hipStream_t s) {
  if (nblk > 0) kb_cg_update<T><<<nblk, bs, 0, s>>>(items, nit, x, r, p, w, st, part);
}
template void launch_bcg_update_t<float>(const BItem*, int, int, int, float*, float*, const float*, const float*,
                                         const BCgState*, double*, hipStream_t);
void launch_bp_update(const BItem* items, int nit, int nblk, int bs, const double* z, double* p,
                      const BCgState* st, hipStream_t s) {
  launch_bp_update_t<double>(items, nit, nblk, bs, z, p, st, s);
}
void launch_bcg_update(const BItem* items, int nit, int nblk, int bs, double* x, double* r, const double* p,
                       const double* w, const BCgState* st, double* part, hipStream_t s) {
  launch_bcg_update_t<double>(items, nit, nblk, bs, x, r, p, w, st, part, s);
}
void launch_bcg_check(const BItem* items, int nit, BCgState* st, const double* part, double tol,
                      int cg_max, hipStream_t s) {
  if (nit > 0) kb_cg_check<<<nit, FB, 0, s>>>(items, st, part, tol, cg_max);
}
void launch_bmultidot(const BItem* items, int nit, int nblk, int bs, const double* Q, long long ld, int nc,
                      const double* v, double* part, hipStream_t s) {
  if (nblk <= 0 || nc <= 0) return;
#define CALL(M) kb_multidot<M><<<nblk, bs, 0, s>>>(items, nit, Q, ld, v, part)
  MGAR_DISPATCH_M(nc, CALL)
#undef CALL
}
void launch_bgs_update(const BItem* items, int nit, int nblk, int bs, double* v, const double* Q, long long ld,
                       int nc, const MgarDev* md, hipStream_t s) {
  if (nblk <= 0 || nc <= 0) return;
#define CALL(M) kb_gs_update<M><<<nblk, bs, 0, s>>>(items, nit, v, Q, ld, md)
  MGAR_DISPATCH_M(nc, CALL)
#undef CALL
}
void launch_bgs_normalize(const BItem* items, int nit, int nblk, int bs, double* v, MgarDev* md, int col,
                          const double* nrm2, int nstride, hipStream_t s) {
  if (nblk > 0) kb_gs_normalize<<<nblk, bs, 0, s>>>(items, nit, v, md, col, nrm2, nstride);
}
void launch_bgram(const BItem* items, int nit, int nblk, int bs, const double* Q, const double* W,
                  const double* q, long long ld, int m, double* part, hipStream_t s) {
  if (nblk <= 0) return;
#define CALL(M) kb_gram<M><<<nblk, bs, 0, s>>>(items, nit, Q, W, q, ld, part)
  MGAR_DISPATCH_M(m, CALL)
#undef CALL
}
void launch_bgram_finalize(const BItem* items, int nit, const double* part, int m, MgarDev* md,
                           hipStream_t s) {
  if (nit > 0) kb_gram_finalize<<<nit, FB, 0, s>>>(items, part, m, md);
}
void launch_bcombine(const BItem* items, int nit, int nblk, int bs, const double* Q, const double* W,
                     const double* q, long long ld, int m, MgarDev* md, double* t, double* part,
                     hipStream_t s) {
  if (nblk <= 0) return;
#define CALL(M) kb_combine<M><<<nblk, bs, 0, s>>>(items, nit, Q, W, q, ld, md, t, part)
  MGAR_DISPATCH_M(m, CALL)
#undef CALL
}
void launch_bdecide(const BItem* items, int nit, MgarDev* md, BCgState* st, double eps, int* keep,
                    int* path, double* res_out, hipStream_t s) {
  if (nit > 0) kb_decide<<<(nit + 63) / 64, 64, 0, s>>>(items, nit, md, st, eps, keep, path, res_out);
}
template <typename T>
void launch_bcopy_cells_t(const BItem* items, int nit, int nblk, int bs, const T* a, T* b, const int* skip,
                          int sstride, hipStream_t s) {
  if (nblk > 0) kb_copy_cells<T><<<nblk, bs, 0, s>>>(items, nit, a, b, skip, sstride);
}
template void launch_bcopy_cells_t<uint16_t>(const BItem*, int, int, int, const uint16_t*, uint16_t*, const int*,
                                             int, hipStream_t);
void launch_bcopy_cells(const BItem* items, int nit, int nblk, int bs, const double* a, double* b,
                        const int* skip, int sstride, hipStream_t s) {
  launch_bcopy_cells_t<double>(items, nit, nblk, bs, a, b, skip, sstride, s);
}
