// Learned initial guess: a 3D convolutional U-Net on the element grid, trained
// online on the (density, temperature) pairs of the optimisation loop by the
// kernels of this file (forward, backward, Adam).
//
// Network, L levels with C[l] channels (level l has n / 2^l elements per
// axis): input (3 channels per element: physical density, fraction of the
// element's Dirichlet corner nodes, heat source over its max-norm) ->
// per level two 3x3x3 convolutions with ReLU, 2x average pooling between
// levels -> decoder from level L-2 to 0: trilinear 2x upsampling
// (cell-centred), concatenation [upsampled, skip of the level], two
// convolutions with ReLU -> 1x1x1 head to one output u per element. Node
// prediction: scale * mean of u over the elements touching the node, 0 on
// Dirichlet nodes. Loss over the free nodes: mean (prediction/scale -
// T/scale)^2.
//
// Storage and arithmetic. Parameters, Adam moments and the head are FP32.
// Activations and their gradients are stored channels-last in BF16 (round to
// nearest even from FP32). The 3x3x3 convolutions are implicit GEMMs on the
// matrix cores (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32 sums): output
// voxels x output channels, K = 27 taps x input channels; a 16 x 4 x 4 voxel
// tile and its halo are staged in LDS per chunk of 16 input channels (one
// chunk of 4 for the 3 input channels, four taps per K step). The data
// gradient is the same kernel with the taps mirrored and the weights
// transposed; it stages the output gradient masked by the ReLU of the layer's
// stored output. The weight gradient is a GEMM over voxels on the matrix
// cores with FP32 block partials summed over blocks in a fixed order in
// FP64. Pooling, upsampling and their adjoints sum in FP32. Every long sum
// has a fixed order, so results do not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mgar.h"
#include "mgar_launch.h"

namespace {

#define NHIP(x)                                   \
  do {                                            \
    hipError_t err_ = (x);                        \
    if (err_ != hipSuccess) return MGAR_E_HIP;    \
  } while (0)
#define NACK(x)                                   \
  do {                                            \
    int rc_ = (x);                                \
    if (rc_ != MGAR_OK) return rc_;               \
  } while (0)
#define NLAUNCH() NHIP(hipGetLastError())

constexpr int NB = 256;
constexpr int MAXL = 6;
constexpr int TX = 16, TY = 4, TZ = 4;                 // voxel tile of the convolutions
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;   // halo tile
constexpr int HV = HX * HY * HZ;                       // 648 halo voxels

typedef unsigned short u16;
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned long long u64;

__device__ inline u16 f2bf(float f) {   // round to nearest even (finite values)
  unsigned u = __builtin_bit_cast(unsigned, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ inline float bf2f(u16 b) { return __builtin_bit_cast(float, (unsigned)b << 16); }
__device__ inline bool bfpos(u16 b) { return !(b & 0x8000u) && (b & 0x7FFFu); }

inline int nblk(long long n) { return (int)std::min<long long>((n + NB - 1) / NB, 65535LL * 16); }

// ---------------------------------------------------------------- input and output on the grids

// Input channels of element e: density, fraction of Dirichlet corners, source.
__global__ __launch_bounds__(NB) void k_net_input(Geo g, const double* __restrict__ xphys,
                                                  const float* __restrict__ src, u16* __restrict__ in) {
  const long long e = blockIdx.x * (long long)NB + threadIdx.x;
  if (e >= g.ne) return;
  const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long long)g.nx * g.ny));
  int cnt = 0;
  for (int c = 0; c < 8; ++c) cnt += geo_fixed(g, i + (c & 1), j + ((c >> 1) & 1), k + (c >> 2)) ? 1 : 0;
  const u64 v = (u64)f2bf((float)xphys[e]) | ((u64)f2bf((float)cnt / 8.0f) << 16) |
                ((u64)f2bf(src[e]) << 32);
  reinterpret_cast<u64*>(in)[e] = v;
}

// Sum of u over the elements touching node n, corners in the order c = 0..7
// (c = bx + 2 by + 4 bz, element (i - bx, j - by, k - bz)); cnt returns their number.
__device__ inline double node_sum(const Geo& g, const float* __restrict__ u, int i, int j, int k, int& cnt) {
  double s = 0.0;
  cnt = 0;
  for (int c = 0; c < 8; ++c) {
    const int ex = i - (c & 1), ey = j - ((c >> 1) & 1), ez = k - (c >> 2);
    if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nx || ey >= g.ny || ez >= g.nz) continue;
    s += (double)u[geo_elem(g, ex, ey, ez)];
    ++cnt;
  }
  return s;
}

__global__ __launch_bounds__(NB) void k_to_nodes(Geo g, const float* __restrict__ u, double scale,
                                                 double* __restrict__ T) {
  const long long n = blockIdx.x * (long long)NB + threadIdx.x;
  if (n >= g.nn) return;
  const int i = (int)(n % g.nnx), j = (int)((n / g.nnx) % g.nny), k = (int)(n / ((long long)g.nnx * g.nny));
  int cnt;
  const double s = node_sum(g, u, i, j, k, cnt);
  T[n] = geo_fixed(g, i, j, k) ? 0.0 : scale * s / (double)cnt;
}

// Loss terms per node: r = mean(u) - T/scale on free nodes; gn = 2 r / nf / cnt
// (the share of each touching element's output gradient); r^2 block partials.
__global__ __launch_bounds__(NB) void k_node_resid(Geo g, const float* __restrict__ u,
                                                   const double* __restrict__ T, double scale, double nf,
                                                   double* __restrict__ gn, double* __restrict__ part) {
  __shared__ double sh[NB / MGAR_WAVE];
  const long long n = blockIdx.x * (long long)NB + threadIdx.x;
  double rr = 0.0;
  if (n < g.nn) {
    const int i = (int)(n % g.nnx), j = (int)((n / g.nnx) % g.nny), k = (int)(n / ((long long)g.nnx * g.nny));
    double gv = 0.0;
    if (!geo_fixed(g, i, j, k)) {
      int cnt;
      const double s = node_sum(g, u, i, j, k, cnt);
      const double r = 1.0 * s / (double)cnt - T[n] / scale;
      rr = r * r;
      gv = 2.0 * r / nf / (double)cnt;
    }
    gn[n] = gv;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = rr;
}

__global__ __launch_bounds__(NB) void k_elem_du(Geo g, const double* __restrict__ gn, float* __restrict__ du) {
  const long long e = blockIdx.x * (long long)NB + threadIdx.x;
  if (e >= g.ne) return;
  const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((long long)g.nx * g.ny));
  double s = 0.0;
  for (int c = 0; c < 8; ++c) s += gn[geo_node(g, i + (c & 1), j + ((c >> 1) & 1), k + (c >> 2))];
  du[e] = (float)s;
}

__global__ __launch_bounds__(NB) void k_sum_parts(const double* __restrict__ part, int n, double scale,
                                                  double* __restrict__ out) {
  __shared__ double sh[NB / MGAR_WAVE];
  const double s = block_sum(thread_partials(part, n, threadIdx.x, NB), sh);
  if (threadIdx.x == 0) *out = s * scale;
}

// ---------------------------------------------------------------- head (1x1x1, one output channel)

__global__ __launch_bounds__(NB) void k_head_fwd(long long V, int C, const u16* __restrict__ d0,
                                                 const float* __restrict__ w, float* __restrict__ u) {
  const long long e = blockIdx.x * (long long)NB + threadIdx.x;
  if (e >= V) return;
  // four channels per 8-byte load (C is a multiple of 16), summed in channel order
  const u64* dq = reinterpret_cast<const u64*>(d0) + e * (C / 4);
  float s = 0.0f;
  for (int c4 = 0; c4 < C / 4; ++c4) {
    const u64 v = dq[c4];
#pragma unroll
    for (int a = 0; a < 4; ++a) s += bf2f((u16)(v >> (16 * a))) * w[4 * c4 + a];
  }
  u[e] = s + w[C];
}

// Data gradient of the head and block partials of its weight and bias
// gradients ([block][C + 1]: sum_e d0[e][c] du[e], sum_e du[e]); wave sums,
// then the waves of the block in order.
constexpr int HMAXC = 128;
__global__ __launch_bounds__(NB) void k_head_bwd(long long V, int C, const u16* __restrict__ d0,
                                                 const float* __restrict__ w, const float* __restrict__ du,
                                                 u16* __restrict__ gd0, double* __restrict__ part) {
  __shared__ double sh[NB / MGAR_WAVE][HMAXC + 1];
  const long long e = blockIdx.x * (long long)NB + threadIdx.x;
  const bool in = e < V;
  const float g = in ? du[e] : 0.0f;
  const int wv = threadIdx.x / MGAR_WAVE, lane = threadIdx.x % MGAR_WAVE;
  // four channels per 8-byte load and store (C is a multiple of 16)
  const u64* dq = reinterpret_cast<const u64*>(d0) + (in ? e : 0) * (C / 4);
  u64* gq = reinterpret_cast<u64*>(gd0) + (in ? e : 0) * (C / 4);
  for (int c4 = 0; c4 < C / 4; ++c4) {
    const u64 dv = in ? dq[c4] : 0;
    u64 go = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int c = 4 * c4 + a;
      double v = in ? (double)bf2f((u16)(dv >> (16 * a))) * (double)g : 0.0;
      go |= (u64)f2bf(g * w[c]) << (16 * a);
      v = wave_sum(v);
      if (lane == 0) sh[wv][c] = v;
    }
    if (in) gq[c4] = go;
  }
  {
    double v = in ? (double)g : 0.0;
    v = wave_sum(v);
    if (lane == 0) sh[wv][C] = v;
  }
  __syncthreads();
  for (int c = threadIdx.x; c <= C; c += NB) {
    double s = 0.0;
    for (int k = 0; k < NB / MGAR_WAVE; ++k) s += sh[k][c];
    part[(long long)blockIdx.x * (C + 1) + c] = s;
  }
}

// grad[c] = sum over the nb blocks of part[b][c] (block c of the grid; every
// thread sums its blocks in order, then a fixed-order block sum)
__global__ __launch_bounds__(NB) void k_head_reduce(const double* __restrict__ part, int nb, int C,
                                                    double* __restrict__ grad) {
  __shared__ double sh[NB / MGAR_WAVE];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += NB) s += part[(long long)b * (C + 1) + c];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) grad[c] = s;
}

// ---------------------------------------------------------------- pooling and upsampling (channels-last)

struct Dims { int nx, ny, nz; };

// Voxel v = t / Q, channel quad q = t % Q and the voxel's (i, j, k) on an
// nx x ny x .. grid, in 32-bit arithmetic (the network's sizes keep every
// voxel x quad count below 2^28, checked at creation).
struct VQ { unsigned v; int q, i, j, k; };
__device__ inline VQ split_vq(unsigned t, int Q, int nx, int ny) {
  VQ r;
  r.v = t / (unsigned)Q;
  r.q = (int)(t - r.v * (unsigned)Q);
  const unsigned jk = r.v / (unsigned)nx;
  r.i = (int)(r.v - jk * (unsigned)nx);
  r.k = (int)(jk / (unsigned)ny);
  r.j = (int)(jk - (unsigned)r.k * (unsigned)ny);
  return r;
}

// coarse (nx, ny, nz) = fine / 2; one thread per (coarse voxel, channel quad)
__global__ __launch_bounds__(NB) void k_pool(Dims c, int C, const u16* __restrict__ fine, u16* __restrict__ out) {
  const int Q = C / 4;
  const unsigned t = blockIdx.x * NB + threadIdx.x;
  if (t >= (unsigned)c.nx * c.ny * c.nz * Q) return;
  const VQ x = split_vq(t, Q, c.nx, c.ny);
  const unsigned v = x.v;
  const int q = x.q, i = x.i, j = x.j, k = x.k;
  const int fx = 2 * c.nx, fy = 2 * c.ny;
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  for (int b = 0; b < 8; ++b) {
    const unsigned fv = (2 * i + (b & 1)) + (unsigned)fx * ((2 * j + ((b >> 1) & 1)) + (unsigned)fy * (2 * k + (b >> 2)));
    const u64 w = reinterpret_cast<const u64*>(fine)[fv * Q + q];
    for (int a = 0; a < 4; ++a) s[a] += bf2f((u16)(w >> (16 * a)));
  }
  u64 o = 0;
  for (int a = 0; a < 4; ++a) o |= (u64)f2bf(s[a] * 0.125f) << (16 * a);
  reinterpret_cast<u64*>(out)[v * (unsigned)Q + q] = o;
}

// 1D linear 2x upsampling of cell-centred values: fine cell f lies at coarse
// coordinate (f + 1/2)/2 - 1/2, clamped to [0, n-1]; weights on i0 and i1.
__device__ inline void up_axis(int f, int n, int& i0, int& i1, float& w0, float& w1) {
  float c = (f + 0.5f) * 0.5f - 0.5f;
  c = fminf(fmaxf(c, 0.0f), (float)(n - 1));
  i0 = (int)floorf(c);
  i1 = min(i0 + 1, n - 1);
  w1 = c - (float)i0;
  w0 = 1.0f - w1;
}

// weight of coarse cell m in fine cell f (the transpose of up_axis)
__device__ inline float up_weight(int f, int m, int n) {
  int i0, i1;
  float w0, w1;
  up_axis(f, n, i0, i1, w0, w1);
  return (i0 == m ? w0 : 0.0f) + (i1 == m ? w1 : 0.0f);
}

// fine = up(coarse); c: coarse dims; one thread per (fine voxel, channel quad)
__global__ __launch_bounds__(NB) void k_up(Dims c, int C, const u16* __restrict__ crs, u16* __restrict__ out) {
  const int Q = C / 4;
  const int fx = 2 * c.nx, fy = 2 * c.ny, fz = 2 * c.nz;
  const unsigned t = blockIdx.x * NB + threadIdx.x;
  if (t >= (unsigned)fx * fy * fz * Q) return;
  const VQ vq = split_vq(t, Q, fx, fy);
  const unsigned v = vq.v;
  const int q = vq.q, i = vq.i, j = vq.j, k = vq.k;
  int x0, x1, y0, y1, z0, z1;
  float wx0, wx1, wy0, wy1, wz0, wz1;
  up_axis(i, c.nx, x0, x1, wx0, wx1);
  up_axis(j, c.ny, y0, y1, wy0, wy1);
  up_axis(k, c.nz, z0, z1, wz0, wz1);
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  for (int b = 0; b < 8; ++b) {
    const int xi = (b & 1) ? x1 : x0, yi = (b & 2) ? y1 : y0, zi = (b & 4) ? z1 : z0;
    const float wt = ((b & 1) ? wx1 : wx0) * ((b & 2) ? wy1 : wy0) * ((b & 4) ? wz1 : wz0);
    const u64 w = reinterpret_cast<const u64*>(crs)[(xi + (unsigned)c.nx * (yi + (unsigned)c.ny * zi)) * Q + q];
    for (int a = 0; a < 4; ++a) s[a] += wt * bf2f((u16)(w >> (16 * a)));
  }
  u64 o = 0;
  for (int a = 0; a < 4; ++a) o |= (u64)f2bf(s[a]) << (16 * a);
  reinterpret_cast<u64*>(out)[v * (unsigned)Q + q] = o;
}

// coarse = up^T(fine); one thread per (coarse voxel, channel quad): gathers the
// fine cells 2m-1 .. 2m+2 of every axis with their upsampling weights
__global__ __launch_bounds__(NB) void k_up_adj(Dims c, int C, const u16* __restrict__ fine, u16* __restrict__ out) {
  const int Q = C / 4;
  const int fx = 2 * c.nx, fy = 2 * c.ny, fz = 2 * c.nz;
  const unsigned t = blockIdx.x * NB + threadIdx.x;
  if (t >= (unsigned)c.nx * c.ny * c.nz * Q) return;
  const VQ vq = split_vq(t, Q, c.nx, c.ny);
  const unsigned v = vq.v;
  const int q = vq.q, i = vq.i, j = vq.j, k = vq.k;
  // per axis, the weights of the fine cells 2m - 1 .. 2m + 2 (0 outside the
  // grid); the terms are taken in the same order and skipped where a weight is 0
  float wx[4], wy[4], wz[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int fi = 2 * i + d - 1, fj = 2 * j + d - 1, fk = 2 * k + d - 1;
    wx[d] = (fi >= 0 && fi < fx) ? up_weight(fi, i, c.nx) : 0.0f;
    wy[d] = (fj >= 0 && fj < fy) ? up_weight(fj, j, c.ny) : 0.0f;
    wz[d] = (fk >= 0 && fk < fz) ? up_weight(fk, k, c.nz) : 0.0f;
  }
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  for (int dz = 0; dz < 4; ++dz) {
    if (wz[dz] == 0.0f) continue;
    const int fk = 2 * k + dz - 1;
#pragma unroll
    for (int dy = 0; dy < 4; ++dy) {
      if (wy[dy] == 0.0f) continue;
      const int fj = 2 * j + dy - 1;
      u64 w4[4];
#pragma unroll
      for (int dx = 0; dx < 4; ++dx) {
        const int fi = 2 * i + dx - 1;
        w4[dx] = wx[dx] != 0.0f
                     ? reinterpret_cast<const u64*>(fine)[(fi + (unsigned)fx * (fj + (unsigned)fy * fk)) * Q + q]
                     : 0;
      }
#pragma unroll
      for (int dx = 0; dx < 4; ++dx) {
        if (wx[dx] == 0.0f) continue;
        const float wt = wx[dx] * wy[dy] * wz[dz];
        for (int a = 0; a < 4; ++a) s[a] += wt * bf2f((u16)(w4[dx] >> (16 * a)));
      }
    }
  }
  u64 o = 0;
  for (int a = 0; a < 4; ++a) o |= (u64)f2bf(s[a]) << (16 * a);
  reinterpret_cast<u64*>(out)[v * Q + q] = o;
}

// skip gradient = skip part of the decoder's data gradient + pooling adjoint of
// the gradient of the pooled tensor (its coarse value / 8); f: fine dims
__global__ __launch_bounds__(NB) void k_skip_add(Dims f, int C, const u16* __restrict__ gsk,
                                                 const u16* __restrict__ gp, u16* __restrict__ out) {
  const int Q = C / 4;
  const unsigned t = blockIdx.x * NB + threadIdx.x;
  if (t >= (unsigned)f.nx * f.ny * f.nz * Q) return;
  const VQ vq = split_vq(t, Q, f.nx, f.ny);
  const unsigned v = vq.v;
  const int q = vq.q, i = vq.i, j = vq.j, k = vq.k;
  const unsigned cv = (i / 2) + (unsigned)(f.nx / 2) * ((j / 2) + (unsigned)(f.ny / 2) * (k / 2));
  const u64 a = reinterpret_cast<const u64*>(gsk)[v * Q + q];
  const u64 b = reinterpret_cast<const u64*>(gp)[cv * Q + q];
  u64 o = 0;
  for (int s = 0; s < 4; ++s)
    o |= (u64)f2bf(bf2f((u16)(a >> (16 * s))) + bf2f((u16)(b >> (16 * s))) * 0.125f) << (16 * s);
  reinterpret_cast<u64*>(out)[v * Q + q] = o;
}

// ---------------------------------------------------------------- 3x3x3 convolution on the matrix cores

struct ConvArgs {
  int nx, ny, nz;        // grid of the level (voxels)
  const u16* s0;         // input channels [0, c0), channels-last
  const u16* s1;         // input channels [c0, c0 + c1) (c1 = 0: none)
  const u16* m0;         // data gradient: the layer's output (ReLU mask of s0); else null
  const u16* w;          // BF16 weights [27][cout][cin], cin = c0 + c1
  const float* bias;     // forward: cout biases (ReLU applied); data gradient: null
  u16* o0;               // output channels [0, d0) (d0 channels per voxel)
  u16* o1;               // output channels [d0, cout)
  int c0, c1, cout, d0;
  int ntx, nty;          // tiles per axis
};

// One block: a 16 x 4 x 4 voxel tile (wave w: z-slice w, M-tiles = its 4 rows
// of 16 voxels) and NT 16-channel output tiles (blockIdx.y selects which).
// Chunks of CC input channels are staged with their halo in LDS
// [halo voxel][CC]; K step kb covers K = 16 kb .. 16 kb + 15 of (tap, channel)
// = (k / CC, k % CC), lane group g taking four consecutive channels of one tap.
template <int NT, int CC, bool DG>
__global__ __launch_bounds__(NB) void k_conv(ConvArgs a) {
  // halo voxel stride in LDS: 16 channels padded to 24 values (12 dwords), so
  // the 16 rows x 4 channel groups of an operand read fall in distinct banks
  constexpr int SV = CC == 16 ? 24 : CC;
  __shared__ __attribute__((aligned(16))) u16 S[HV * SV];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, gq = l >> 4, r = l & 15;
  const int tx = blockIdx.x % a.ntx, ty = (blockIdx.x / a.ntx) % a.nty, tz = blockIdx.x / (a.ntx * a.nty);
  const int x0 = TX * tx, y0 = TY * ty, z0 = TZ * tz;
  const int nt0 = blockIdx.y * NT;   // first 16-channel output tile
  const int cin = a.c0 + a.c1;
  f4 acc[4][NT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n] = f4{0.f, 0.f, 0.f, 0.f};
  for (int cb = 0; cb < cin; cb += CC) {
    const bool first = cb < a.c0;
    const u16* __restrict__ src = first ? a.s0 : a.s1;
    const int cs = first ? a.c0 : a.c1, cl = first ? cb : cb - a.c0;
    // the chunk with its halo. Forward: every load of a thread issued before
    // the first LDS store (one memory round trip per chunk); data gradient
    // (twice the loads, the ReLU mask too): one load pair per step, which
    // measured faster there (fewer registers)
    if constexpr (!DG) {
      constexpr int NQ = (HV * (CC / 4) + NB - 1) / NB;
      u64 vals[NQ];
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const int q = tid + u * NB;
        const int hv = q / (CC / 4), qq = q % (CC / 4);
        const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
        vals[u] = 0;
        if (q < HV * (CC / 4) && gx >= 0 && gy >= 0 && gz >= 0 && gx < a.nx && gy < a.ny && gz < a.nz) {
          const long long off = ((gx + (long long)a.nx * (gy + (long long)a.ny * gz)) * cs + cl) / 4 + qq;
          vals[u] = reinterpret_cast<const u64*>(src)[off];
        }
      }
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const int q = tid + u * NB;
        if (q < HV * (CC / 4)) reinterpret_cast<u64*>(S)[(q / (CC / 4)) * (SV / 4) + q % (CC / 4)] = vals[u];
      }
    } else {
      for (int q = tid; q < HV * (CC / 4); q += NB) {
        const int hv = q / (CC / 4), qq = q % (CC / 4);
        const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
        u64 val = 0;
        if (gx >= 0 && gy >= 0 && gz >= 0 && gx < a.nx && gy < a.ny && gz < a.nz) {
          const long long off = ((gx + (long long)a.nx * (gy + (long long)a.ny * gz)) * cs + cl) / 4 + qq;
          val = reinterpret_cast<const u64*>(src)[off];
          const u64 mk = reinterpret_cast<const u64*>(a.m0)[off];
          u64 keep = 0;
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (bfpos((u16)(mk >> (16 * s)))) keep |= 0xFFFFull << (16 * s);
          val &= keep;
        }
        reinterpret_cast<u64*>(S)[hv * (SV / 4) + qq] = val;
      }
    }
    __syncthreads();
    constexpr int NKB = (27 * CC + 15) / 16;
    // operands of K step kb (A from LDS, B from the weights in global memory);
    // those of the next step are loaded before the matrix products of this one
    auto load = [&](int kb, bf4 (&A)[4], bf4 (&B)[NT]) {
      const int k = 16 * kb + 4 * gq;
      const int tap = k / CC, ci0 = k % CC;
      const bool valid = tap < 27;
      const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int hv = (r + dx) + HX * ((m + dy) + HY * (w + dz));
        A[m] = valid ? *reinterpret_cast<const bf4*>(&S[hv * SV + ci0]) : bf4{0, 0, 0, 0};
      }
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int co = (nt0 + n) * 16 + r;
        B[n] = valid ? *reinterpret_cast<const bf4*>(&a.w[((long long)tap * a.cout + co) * cin + cb + ci0])
                     : bf4{0, 0, 0, 0};
      }
    };
    bf4 A[4], B[NT];
    load(0, A, B);
    for (int kb = 0; kb < NKB; ++kb) {
      bf4 An[4], Bn[NT];
      if (kb + 1 < NKB) load(kb + 1, An, Bn);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[m], B[n], acc[m][n], 0, 0, 0);
      if (kb + 1 < NKB) {
#pragma unroll
        for (int m = 0; m < 4; ++m) A[m] = An[m];
#pragma unroll
        for (int n = 0; n < NT; ++n) B[n] = Bn[n];
      }
    }
    __syncthreads();
  }
  const int z = z0 + w;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int y = y0 + m;
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int co = (nt0 + n) * 16 + r;
      const float bco = DG ? 0.0f : a.bias[co];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = x0 + 4 * gq + j;
        if (x >= a.nx || y >= a.ny || z >= a.nz) continue;
        float v = acc[m][n][j] + bco;
        if (!DG) v = fmaxf(v, 0.0f);
        const long long vox = x + (long long)a.nx * (y + (long long)a.ny * z);
        if (co < a.d0) a.o0[vox * a.d0 + co] = f2bf(v);
        else a.o1[vox * (a.cout - a.d0) + (co - a.d0)] = f2bf(v);
      }
    }
  }
}

struct WgArgs {
  int nx, ny, nz;
  const u16* a0;         // layer input channels [0, c0)
  const u16* a1;         // layer input channels [c0, c0 + c1)
  const u16* gA;         // gradient of the layer's output
  const u16* A;          // the layer's output (ReLU mask)
  float* part;           // [block][27][cout][cin16] FP32 partials
  double* bpart;         // [block][cout] bias partials
  int c0, c1, cout, cin16;
  int ntx, nty, ntiles, tpb;
};

constexpr int WRW = 20;            // LDS row of the weight gradient's input tile: 18 halo voxels + 2 zeros
constexpr int WROWS = HY * HZ;     // 36 halo rows per channel
// LDS strides of the weight gradient (BF16 values): per input channel 776 >=
// 36 x 20 (388 dwords), per output-gradient channel 264 >= 256 (132 dwords);
// both are 4 dwords modulo the 64 banks, so the 16 channels x 4 voxel groups
// of an operand read fall in distinct banks
constexpr int WCS = 776, WDS = 264;

// 4 x 4 transpose of BF16 values: in[s] holds 4 channels of voxel s; out[j]
// holds channel j of the 4 voxels
__device__ inline void tr4(const u64 (&in)[4], u64 (&out)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    u64 v = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) v |= ((in[s] >> (16 * j)) & 0xFFFFull) << (16 * s);
    out[j] = v;
  }
}

// Weight gradient dW[tap][co][ci] = sum over voxels of gZ[v][co] * in[v + tap][ci],
// gZ = gA * (A > 0). Grid: x = block (a range of tpb tiles), y = 16-channel
// input chunk, z = group of NTC 16-channel output tiles. Per tile the input
// chunk with its halo is staged in LDS as [channel][halo row][20] and gZ as
// [channel][voxel] (each thread loads 4 voxels x 4 channels and writes them
// transposed); wave w accumulates the taps w, w + 4, ... over K = the 256
// voxels of the tile (16 steps of one 16-voxel row), the input operand of a
// tap shifted by dx from two aligned 8-byte reads.
template <int NTC>
__global__ __launch_bounds__(NB) void k_wgrad(WgArgs a) {
  __shared__ __attribute__((aligned(16))) u16 As[16 * WCS];
  __shared__ __attribute__((aligned(16))) u16 Ds[NTC * 16 * WDS];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, gq = l >> 4, r = l & 15;
  const int t0 = blockIdx.x * a.tpb, t1 = min(t0 + a.tpb, a.ntiles);
  const int cg = blockIdx.y, ng0 = blockIdx.z * NTC;
  const int cin = a.c0 + a.c1, cbase = 16 * cg;
  constexpr int TV = TX * TY * TZ;
  f4 acc[7][NTC];
#pragma unroll
  for (int i = 0; i < 7; ++i)
#pragma unroll
    for (int n = 0; n < NTC; ++n) acc[i][n] = f4{0.f, 0.f, 0.f, 0.f};
  // bias partials (first input chunk only): thread tid sums output channel
  // 16 ng0 + tid % (16 NTC) over the voxels v = tid / (16 NTC) + k nbg of every
  // tile, in order; the nbg partials of a channel are added in order at the end
  constexpr int NBC = 16 * NTC, NBG = NB / NBC;
  __shared__ double bsh[NBG * NBC];
  const int bco = tid % NBC, bgr = tid / NBC;
  double bsum = 0.0;
  // input chunk (channels cbase .. cbase + 15 of the concatenated input) of
  // tile t into registers: the next tile's loads are issued before the
  // current tile's matrix products, and stored to LDS after them
  constexpr int NIT = (WROWS * (WRW / 4) * 4 + NB - 1) / NB;
  u64 vin[NIT][4];
  auto load_in = [&](int t) {
    const int tx = t % a.ntx, ty = (t / a.ntx) % a.nty, tz = t / (a.ntx * a.nty);
    const int x0 = TX * tx, y0 = TY * ty, z0 = TZ * tz;
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int it = tid + u * NB;
      const int cq = it % 4, xg = (it / 4) % (WRW / 4), row = it / (4 * (WRW / 4));
      const int hy = row % HY, hz = row / HY;
      const int gy = y0 - 1 + hy, gz = z0 - 1 + hz, c = cbase + 4 * cq;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int hx = 4 * xg + q, gx = x0 - 1 + hx;
        vin[u][q] = 0;
        if (it < WROWS * (WRW / 4) * 4 && hx < HX && c < cin && gx >= 0 && gy >= 0 && gz >= 0 && gx < a.nx &&
            gy < a.ny && gz < a.nz) {
          const long long vox = gx + (long long)a.nx * (gy + (long long)a.ny * gz);
          vin[u][q] = c < a.c0 ? reinterpret_cast<const u64*>(a.a0)[(vox * a.c0 + c) / 4]
                               : reinterpret_cast<const u64*>(a.a1)[(vox * a.c1 + (c - a.c0)) / 4];
        }
      }
    }
  };
  if (t0 < t1) load_in(t0);
  for (int t = t0; t < t1; ++t) {
    const int tx = t % a.ntx, ty = (t / a.ntx) % a.nty, tz = t / (a.ntx * a.nty);
    const int x0 = TX * tx, y0 = TY * ty, z0 = TZ * tz;
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      const int it = tid + u * NB;
      if (it >= WROWS * (WRW / 4) * 4) continue;
      const int cq = it % 4, xg = (it / 4) % (WRW / 4), row = it / (4 * (WRW / 4));
      u64 o[4];
      tr4(vin[u], o);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        *reinterpret_cast<u64*>(&As[(4 * cq + j) * WCS + row * WRW + 4 * xg]) = o[j];
    }
    // masked output gradient (channels 16 ng0 .. 16 (ng0 + NTC) - 1)
    for (int it = tid; it < (TV / 4) * 4 * NTC; it += NB) {
      const int cq = it % (4 * NTC), xg = (it / (4 * NTC)) % (TX / 4), vrow = it / (4 * NTC * (TX / 4));
      const int gy = y0 + (vrow & 3), gz = z0 + (vrow >> 2);
      u64 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gx = x0 + 4 * xg + q;
        v[q] = 0;
        if (gx < a.nx && gy < a.ny && gz < a.nz) {
          const long long off = ((gx + (long long)a.nx * (gy + (long long)a.ny * gz)) * a.cout + 16 * ng0) / 4 + cq;
          const u64 mk = reinterpret_cast<const u64*>(a.A)[off];
          u64 keep = 0;
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if (bfpos((u16)(mk >> (16 * s)))) keep |= 0xFFFFull << (16 * s);
          v[q] = reinterpret_cast<const u64*>(a.gA)[off] & keep;
        }
      }
      u64 o[4];
      tr4(v, o);
#pragma unroll
      for (int j = 0; j < 4; ++j) *reinterpret_cast<u64*>(&Ds[(4 * cq + j) * WDS + vrow * TX + 4 * xg]) = o[j];
    }
    __syncthreads();
    if (t + 1 < t1) load_in(t + 1);
    if (cg == 0 && bgr < NBG) {
      double s = 0.0;
      for (int v = bgr; v < TV; v += NBG) s += (double)bf2f(Ds[bco * WDS + v]);
      bsum += s;
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const int tap = w + 4 * i;
      if (tap < 27) {
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
#pragma unroll 4
        for (int kb = 0; kb < 16; ++kb) {
          const int row = ((kb >> 2) + dz) * HY + ((kb & 3) + dy);
          const u64* pb = reinterpret_cast<const u64*>(&As[r * WCS + row * WRW + 4 * gq]);
          const u64 lo = pb[0], hi = pb[1];
          const u64 bw = dx == 0 ? lo : (lo >> (16 * dx)) | (hi << (64 - 16 * dx));
          const bf4 B = __builtin_bit_cast(bf4, bw);
#pragma unroll
          for (int n = 0; n < NTC; ++n) {
            const bf4 A = *reinterpret_cast<const bf4*>(&Ds[(n * 16 + r) * WDS + kb * TX + 4 * gq]);
            acc[i][n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[i][n], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const int tap = w + 4 * i;
    if (tap < 27) {
#pragma unroll
      for (int n = 0; n < NTC; ++n)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int co = 16 * (ng0 + n) + 4 * gq + j, ci = cbase + r;
          a.part[(((long long)blockIdx.x * 27 + tap) * a.cout + co) * a.cin16 + ci] = acc[i][n][j];
        }
    }
  }
  if (cg == 0) {
    if (bgr < NBG) bsh[bgr * NBC + bco] = bsum;
    __syncthreads();
    if (tid < NBC) {
      double s = 0.0;
      for (int q = 0; q < NBG; ++q) s += bsh[q * NBC + tid];
      a.bpart[(long long)blockIdx.x * a.cout + 16 * ng0 + tid] = s;
    }
  }
}

// grad[woff + (co ci + c) 27 + tap] = sum over blocks of part[b][tap][co][c]
// (c < ci), and grad[boff + co] = sum over blocks of bpart[b][co]. Sixteen
// threads per parameter: thread q sums the blocks q, q + 16, ... in order and
// the sixteen sums are added in order of q. A block holds WRT consecutive
// parameters (one per lane, so a wave's loads of one block row are contiguous)
// times the WRQ threads of each.
constexpr int WRQ = 16, WRT = 64;
__global__ __launch_bounds__(WRT * WRQ) void k_wreduce(const float* __restrict__ part,
                                                       const double* __restrict__ bpart, int nb, int cout,
                                                       int ci, int cin16, double* __restrict__ gw,
                                                       double* __restrict__ gb) {
  __shared__ double sh[WRQ][WRT];
  const int tl = threadIdx.x % WRT, q = threadIdx.x / WRT;
  const long long t = blockIdx.x * (long long)WRT + tl;
  const long long nw = 27LL * cout * cin16;
  double s = 0.0;
  if (t < nw) {
#pragma unroll 8
    for (int b = q; b < nb; b += WRQ) s += (double)part[(long long)b * nw + t];
  } else if (t < nw + cout) {
#pragma unroll 8
    for (int b = q; b < nb; b += WRQ) s += bpart[(long long)b * cout + (t - nw)];
  }
  sh[q][tl] = s;
  __syncthreads();
  if (q == 0 && t < nw + cout) {
    double v = 0.0;
    for (int k = 0; k < WRQ; ++k) v += sh[k][tl];
    if (t < nw) {
      const int c = (int)(t % cin16), co = (int)((t / cin16) % cout), tap = (int)(t / ((long long)cin16 * cout));
      if (c < ci) gw[((long long)co * ci + c) * 27 + tap] = v;
    } else {
      gb[t - nw] = v;
    }
  }
}

// ---------------------------------------------------------------- parameters

// BF16 copies of a convolution's weights: forward wf[tap][co][cip] (input
// channels padded to cip with zeros) and data gradient wd[tap][ci][co] with
// the taps mirrored (tap' = 26 - tap).
__global__ __launch_bounds__(NB) void k_pack_w(const float* __restrict__ w, int co, int ci, int cip,
                                               u16* __restrict__ wf, u16* __restrict__ wd) {
  const long long t = blockIdx.x * (long long)NB + threadIdx.x;
  if (t >= 27LL * co * cip) return;
  const int c = (int)(t % cip), o = (int)((t / cip) % co), tap = (int)(t / ((long long)cip * co));
  const u16 b = c < ci ? f2bf(w[((long long)o * ci + c) * 27 + tap]) : (u16)0;
  wf[t] = b;
  if (c < ci) wd[((long long)(26 - tap) * ci + c) * co + o] = b;
}

__global__ __launch_bounds__(NB) void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                             const double* __restrict__ g, long long n, double lr, double c1,
                                             double c2) {
  const long long i = blockIdx.x * (long long)NB + threadIdx.x;
  if (i >= n) return;
  const double gi = g[i];
  const float mi = (float)(0.9 * (double)m[i] + (1.0 - 0.9) * gi);
  const float vi = (float)(0.999 * (double)v[i] + (1.0 - 0.999) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  const double mh = (double)mi / c1, vh = (double)vi / c2;
  th[i] = (float)((double)th[i] - lr * mh / (sqrt(vh) + 1e-8));
}

}  // namespace

// ---------------------------------------------------------------- handle

struct mgar_net {
  hipStream_t s = nullptr;
  Geo g{};
  int L = 0;
  int C[MAXL] = {};
  Dims lv[MAXL] = {};
  long long V[MAXL] = {};
  long long np = 0;
  int t = 0;
  float *theta = nullptr, *m = nullptr, *v = nullptr;
  double* grad = nullptr;
  float* src = nullptr;
  u16* in = nullptr;
  u16 *e[MAXL] = {}, *s_[MAXL] = {}, *p[MAXL] = {}, *up[MAXL] = {}, *h[MAXL] = {}, *d[MAXL] = {};
  u16 *g1[MAXL] = {}, *g2[MAXL] = {}, *gup[MAXL] = {}, *gsk[MAXL] = {}, *gpool[MAXL] = {};
  float *u = nullptr, *du = nullptr;
  double *gn = nullptr, *lpart = nullptr, *loss = nullptr, *hpart = nullptr;
  float* wpart = nullptr;
  double* bpart = nullptr;
  long long wpart_cap = 0, bpart_cap = 0;
  struct Layer { int co, ci, cip, k, lev; long long woff, boff; u16* wf; u16* wd; };
  std::vector<Layer> layers;
  std::vector<void*> allocs;
};

namespace {

template <typename T>
int nalloc(mgar_net* n, T** p, long long count) {
  *p = nullptr;
  if (count <= 0) return MGAR_OK;
  NHIP(hipMalloc((void**)p, sizeof(T) * (size_t)count));
  n->allocs.push_back((void*)*p);
  return MGAR_OK;
}

int layer_index(const mgar_net* n, char kind, int l, char ab) {
  if (kind == 'e') return 2 * l + (ab == 'b');
  if (kind == 'd') return 2 * n->L + 2 * (n->L - 2 - l) + (ab == 'b');
  return 4 * n->L - 2;   // head
}

inline int tiles(const Dims& d, int* ntx, int* nty) {
  *ntx = (d.nx + TX - 1) / TX;
  *nty = (d.ny + TY - 1) / TY;
  return *ntx * *nty * ((d.nz + TZ - 1) / TZ);
}

// out = conv(in) (forward, ReLU) or the data gradient (DG) of a layer.
int conv(mgar_net* n, const Dims& d, const u16* s0, int c0, const u16* s1, int c1, const u16* m0,
         const u16* wts, const float* bias, int cout, u16* o0, int d0, u16* o1, bool dg) {
  ConvArgs a;
  a.nx = d.nx; a.ny = d.ny; a.nz = d.nz;
  a.s0 = s0; a.s1 = s1; a.m0 = m0; a.w = wts; a.bias = bias;
  a.o0 = o0; a.o1 = o1; a.c0 = c0; a.c1 = c1; a.cout = cout; a.d0 = d0;
  if (cout % 16 || (c0 + c1) % 4) return MGAR_E_ARG;
  const int nt = tiles(d, &a.ntx, &a.nty);
  const int T16 = cout / 16;
  // output tiles per block: as many as divide the count, fewer when the grid
  // has few voxel tiles (each block then stages the same input for fewer
  // output channels, and more blocks share the work)
  int NTc = (T16 % 4 == 0) ? 4 : (T16 % 3 == 0) ? 3 : (T16 % 2 == 0) ? 2 : 1;
  while (NTc > 1 && (long long)nt * (T16 / NTc) < 1024) {
    int nx = NTc - 1;
    while (nx > 1 && T16 % nx) --nx;
    NTc = nx;
  }
  const dim3 grid(nt, T16 / NTc);
  const bool small = (c0 + c1) < 16;
  if (small && (dg || c1 || c0 != 4)) return MGAR_E_ARG;
#define KCONV(NTV, CCV, DGV) hipLaunchKernelGGL((k_conv<NTV, CCV, DGV>), grid, dim3(NB), 0, n->s, a)
  if (small) {
    switch (NTc) {
      case 1: KCONV(1, 4, false); break;
      case 2: KCONV(2, 4, false); break;
      case 3: KCONV(3, 4, false); break;
      default: KCONV(4, 4, false); break;
    }
  } else if (dg) {
    if (c0 % 16 || c1 % 16) return MGAR_E_ARG;
    switch (NTc) {
      case 1: KCONV(1, 16, true); break;
      case 2: KCONV(2, 16, true); break;
      case 3: KCONV(3, 16, true); break;
      default: KCONV(4, 16, true); break;
    }
  } else {
    if (c0 % 16 || c1 % 16) return MGAR_E_ARG;
    switch (NTc) {
      case 1: KCONV(1, 16, false); break;
      case 2: KCONV(2, 16, false); break;
      case 3: KCONV(3, 16, false); break;
      default: KCONV(4, 16, false); break;
    }
  }
#undef KCONV
  NLAUNCH();
  return MGAR_OK;
}

// weight and bias gradients of layer li into n->grad
int wgrad(mgar_net* n, int li, const Dims& d, const u16* a0, int c0, const u16* a1, int c1, const u16* gA,
          const u16* A) {
  const auto& Ly = n->layers[li];
  WgArgs a;
  a.nx = d.nx; a.ny = d.ny; a.nz = d.nz;
  a.a0 = a0; a.a1 = a1; a.gA = gA; a.A = A;
  a.c0 = c0; a.c1 = c1; a.cout = Ly.co;
  a.cin16 = ((c0 + c1) + 15) / 16 * 16;
  a.ntiles = tiles(d, &a.ntx, &a.nty);
  const long long per = 27LL * a.cout * a.cin16;
  long long nb = std::min<long long>(a.ntiles, 512);
  nb = std::min<long long>(nb, std::max<long long>(1, n->wpart_cap / per));
  a.tpb = (int)((a.ntiles + nb - 1) / nb);
  nb = (a.ntiles + a.tpb - 1) / a.tpb;
  if (nb * per > n->wpart_cap || nb * a.cout > n->bpart_cap) return MGAR_E_ARG;
  a.part = n->wpart;
  a.bpart = n->bpart;
  const int nco = a.cout / 16;
  const int NTC = (nco % 4 == 0) ? 4 : (nco % 3 == 0) ? 3 : (nco % 2 == 0) ? 2 : 1;
  const dim3 grid((unsigned)nb, (unsigned)(a.cin16 / 16), (unsigned)(nco / NTC));
  switch (NTC) {
    case 1: hipLaunchKernelGGL(k_wgrad<1>, grid, dim3(NB), 0, n->s, a); break;
    case 2: hipLaunchKernelGGL(k_wgrad<2>, grid, dim3(NB), 0, n->s, a); break;
    case 3: hipLaunchKernelGGL(k_wgrad<3>, grid, dim3(NB), 0, n->s, a); break;
    default: hipLaunchKernelGGL(k_wgrad<4>, grid, dim3(NB), 0, n->s, a); break;
  }
  NLAUNCH();
  hipLaunchKernelGGL(k_wreduce, dim3((unsigned)((per + a.cout + WRT - 1) / WRT)), dim3(WRT * WRQ), 0, n->s,
                     (const float*)n->wpart,
                     (const double*)n->bpart, (int)nb, a.cout, Ly.ci, a.cin16, n->grad + Ly.woff,
                     n->grad + Ly.boff);
  NLAUNCH();
  return MGAR_OK;
}

int pack_weights(mgar_net* n) {
  for (auto& Ly : n->layers) {
    if (Ly.k != 3) continue;
    hipLaunchKernelGGL(k_pack_w, dim3(nblk(27LL * Ly.co * Ly.cip)), dim3(NB), 0, n->s,
                       (const float*)(n->theta + Ly.woff), Ly.co, Ly.ci, Ly.cip, Ly.wf, Ly.wd);
    NLAUNCH();
  }
  return MGAR_OK;
}

int forward(mgar_net* n, const double* xphys) {
  const int L = n->L;
  hipLaunchKernelGGL(k_net_input, dim3(nblk(n->g.ne)), dim3(NB), 0, n->s, n->g, xphys, (const float*)n->src, n->in);
  NLAUNCH();
  for (int l = 0; l < L; ++l) {
    const auto& La = n->layers[layer_index(n, 'e', l, 'a')];
    const auto& Lb = n->layers[layer_index(n, 'e', l, 'b')];
    const u16* x = n->in;
    int cx = 4;
    if (l > 0) {
      hipLaunchKernelGGL(k_pool, dim3(nblk(n->V[l] * n->C[l - 1] / 4)), dim3(NB), 0, n->s, n->lv[l], n->C[l - 1],
                         (const u16*)n->s_[l - 1], n->p[l]);
      NLAUNCH();
      x = n->p[l];
      cx = n->C[l - 1];
    }
    NACK(conv(n, n->lv[l], x, cx, nullptr, 0, nullptr, La.wf, n->theta + La.boff, La.co, n->e[l], La.co, nullptr,
              false));
    NACK(conv(n, n->lv[l], n->e[l], n->C[l], nullptr, 0, nullptr, Lb.wf, n->theta + Lb.boff, Lb.co, n->s_[l],
              Lb.co, nullptr, false));
  }
  for (int l = L - 2; l >= 0; --l) {
    const u16* below = (l + 1 == L - 1) ? n->s_[L - 1] : n->d[l + 1];
    hipLaunchKernelGGL(k_up, dim3(nblk(n->V[l] * n->C[l + 1] / 4)), dim3(NB), 0, n->s, n->lv[l + 1], n->C[l + 1],
                       below, n->up[l]);
    NLAUNCH();
    const auto& La = n->layers[layer_index(n, 'd', l, 'a')];
    const auto& Lb = n->layers[layer_index(n, 'd', l, 'b')];
    NACK(conv(n, n->lv[l], n->up[l], n->C[l + 1], n->s_[l], n->C[l], nullptr, La.wf, n->theta + La.boff, La.co,
              n->h[l], La.co, nullptr, false));
    NACK(conv(n, n->lv[l], n->h[l], n->C[l], nullptr, 0, nullptr, Lb.wf, n->theta + Lb.boff, Lb.co, n->d[l],
              Lb.co, nullptr, false));
  }
  const auto& Lh = n->layers[layer_index(n, 'h', 0, 'a')];
  hipLaunchKernelGGL(k_head_fwd, dim3(nblk(n->V[0])), dim3(NB), 0, n->s, n->V[0], n->C[0], (const u16*)n->d[0],
                     (const float*)(n->theta + Lh.woff), n->u);
  NLAUNCH();
  return MGAR_OK;
}

// loss (device, n->loss) and the gradient of every parameter (n->grad)
int loss_grad(mgar_net* n, const double* xphys, const double* T, double scale) {
  const int L = n->L;
  NACK(forward(n, xphys));
  const Geo& g = n->g;
  long long nfree = g.nn;
  {
    const long long fx = std::max(0, g.f1x - g.f0x + 1), fy = std::max(0, g.f1y - g.f0y + 1),
                    fz = std::max(0, g.f1z - g.f0z + 1);
    nfree -= fx * fy * fz;
  }
  const int nbn = nblk(g.nn);
  hipLaunchKernelGGL(k_node_resid, dim3(nbn), dim3(NB), 0, n->s, g, (const float*)n->u, T, scale, (double)nfree,
                     n->gn, n->lpart);
  NLAUNCH();
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(NB), 0, n->s, (const double*)n->lpart, nbn, 1.0 / (double)nfree,
                     n->loss);
  NLAUNCH();
  hipLaunchKernelGGL(k_elem_du, dim3(nblk(g.ne)), dim3(NB), 0, n->s, g, (const double*)n->gn, n->du);
  NLAUNCH();
  // head
  const auto& Lh = n->layers[layer_index(n, 'h', 0, 'a')];
  const int nbv = nblk(n->V[0]);
  hipLaunchKernelGGL(k_head_bwd, dim3(nbv), dim3(NB), 0, n->s, n->V[0], n->C[0], (const u16*)n->d[0],
                     (const float*)(n->theta + Lh.woff), (const float*)n->du, n->g1[0], n->hpart);
  NLAUNCH();
  hipLaunchKernelGGL(k_head_reduce, dim3(n->C[0] + 1), dim3(NB), 0, n->s, (const double*)n->hpart, nbv, n->C[0],
                     n->grad + Lh.woff);
  NLAUNCH();
  // decoder, level 0 up to L-2; g1[l] holds the gradient of d_l (of s_(L-1) at l = L-1)
  for (int l = 0; l <= L - 2; ++l) {
    const int ia = layer_index(n, 'd', l, 'a'), ib = layer_index(n, 'd', l, 'b');
    const auto& La = n->layers[ia];
    const auto& Lb = n->layers[ib];
    NACK(wgrad(n, ib, n->lv[l], n->h[l], n->C[l], nullptr, 0, n->g1[l], n->d[l]));
    NACK(conv(n, n->lv[l], n->g1[l], n->C[l], nullptr, 0, n->d[l], Lb.wd, nullptr, Lb.ci, n->g2[l], Lb.ci,
              nullptr, true));
    NACK(wgrad(n, ia, n->lv[l], n->up[l], n->C[l + 1], n->s_[l], n->C[l], n->g2[l], n->h[l]));
    NACK(conv(n, n->lv[l], n->g2[l], n->C[l], nullptr, 0, n->h[l], La.wd, nullptr, La.ci, n->gup[l], n->C[l + 1],
              n->gsk[l], true));
    hipLaunchKernelGGL(k_up_adj, dim3(nblk(n->V[l + 1] * n->C[l + 1] / 4)), dim3(NB), 0, n->s, n->lv[l + 1],
                       n->C[l + 1], (const u16*)n->gup[l], n->g1[l + 1]);
    NLAUNCH();
  }
  // encoder, level L-1 down to 0
  for (int l = L - 1; l >= 0; --l) {
    const int ia = layer_index(n, 'e', l, 'a'), ib = layer_index(n, 'e', l, 'b');
    const auto& Lb = n->layers[ib];
    if (l < L - 1) {
      hipLaunchKernelGGL(k_skip_add, dim3(nblk(n->V[l] * n->C[l] / 4)), dim3(NB), 0, n->s, n->lv[l], n->C[l],
                         (const u16*)n->gsk[l], (const u16*)n->gpool[l + 1], n->g1[l]);
      NLAUNCH();
    }
    NACK(wgrad(n, ib, n->lv[l], n->e[l], n->C[l], nullptr, 0, n->g1[l], n->s_[l]));
    NACK(conv(n, n->lv[l], n->g1[l], n->C[l], nullptr, 0, n->s_[l], Lb.wd, nullptr, Lb.ci, n->g2[l], Lb.ci,
              nullptr, true));
    if (l == 0) {
      NACK(wgrad(n, ia, n->lv[0], n->in, 4, nullptr, 0, n->g2[0], n->e[0]));
    } else {
      const auto& La = n->layers[ia];
      NACK(wgrad(n, ia, n->lv[l], n->p[l], n->C[l - 1], nullptr, 0, n->g2[l], n->e[l]));
      NACK(conv(n, n->lv[l], n->g2[l], n->C[l], nullptr, 0, n->e[l], La.wd, nullptr, La.ci, n->gpool[l], La.ci,
                nullptr, true));
    }
  }
  return MGAR_OK;
}

int create_impl(mgar_net* N, const mgar_params* p, int levels, const int* channels, void* stream) {
  NACK(mgar_internal_validate(p));
  if (p->dim != 3 || levels < 2 || levels > MAXL || !channels) return MGAR_E_ARG;
  const int f = 1 << (levels - 1);
  if (p->nelx % f || p->nely % f || p->nelz % f) return MGAR_E_DIMS;
  for (int l = 0; l < levels; ++l)
    if (channels[l] < 16 || channels[l] > 128 || channels[l] % 16) return MGAR_E_ARG;
  N->s = (hipStream_t)stream;
  N->g = mgar_internal_geo(*p, 0);
  N->L = levels;
  for (int l = 0; l < levels; ++l) {
    N->C[l] = channels[l];
    N->lv[l] = Dims{p->nelx >> l, p->nely >> l, p->nelz >> l};
    N->V[l] = (long long)N->lv[l].nx * N->lv[l].ny * N->lv[l].nz;
  }
  // the pooling, upsampling and skip kernels take one thread per (voxel,
  // channel quad) of a grid, with 32-bit indices and at most nblk's block cap
  for (int l = 0; l < levels; ++l) {
    const int cm = std::max({N->C[std::max(l - 1, 0)], N->C[l], N->C[std::min(l + 1, levels - 1)]});
    if (N->V[l] * (cm / 4) > 65535LL * 16 * NB) return MGAR_E_DIMS;
  }
  const int L = levels;
  // layers in parameter order: encoder, decoder, head
  long long off = 0;
  auto add = [&](int co, int ci, int k, int lev) {
    mgar_net::Layer Ly{co, ci, ci < 4 ? 4 : ci, k, lev, off, off + (long long)co * ci * k * k * k, nullptr, nullptr};
    off = Ly.boff + co;
    N->layers.push_back(Ly);
  };
  for (int l = 0; l < L; ++l) {
    add(N->C[l], l == 0 ? 3 : N->C[l - 1], 3, l);
    add(N->C[l], N->C[l], 3, l);
  }
  for (int l = L - 2; l >= 0; --l) {
    add(N->C[l], N->C[l + 1] + N->C[l], 3, l);
    add(N->C[l], N->C[l], 3, l);
  }
  add(1, N->C[0], 1, 0);
  N->np = off;
  NACK(nalloc(N, &N->theta, off));
  NACK(nalloc(N, &N->m, off));
  NACK(nalloc(N, &N->v, off));
  NACK(nalloc(N, &N->grad, off));
  NHIP(hipMemset(N->theta, 0, sizeof(float) * off));
  NHIP(hipMemset(N->m, 0, sizeof(float) * off));
  NHIP(hipMemset(N->v, 0, sizeof(float) * off));
  NHIP(hipMemset(N->grad, 0, sizeof(double) * off));
  long long wmax = 0;
  for (auto& Ly : N->layers) {
    if (Ly.k != 3) continue;
    NACK(nalloc(N, &Ly.wf, 27LL * Ly.co * Ly.cip));
    NACK(nalloc(N, &Ly.wd, 27LL * Ly.co * Ly.ci));
    wmax = std::max(wmax, 27LL * Ly.co * ((Ly.ci + 15) / 16 * 16));
  }
  const long long E = N->V[0];
  NACK(nalloc(N, &N->src, E));
  {
    std::vector<float> one((size_t)E, 1.0f);
    NHIP(hipMemcpy(N->src, one.data(), sizeof(float) * (size_t)E, hipMemcpyHostToDevice));
  }
  NACK(nalloc(N, &N->in, 4 * E));
  for (int l = 0; l < L; ++l) {
    const long long Vl = N->V[l];
    NACK(nalloc(N, &N->e[l], Vl * N->C[l]));
    NACK(nalloc(N, &N->s_[l], Vl * N->C[l]));
    NACK(nalloc(N, &N->g1[l], Vl * N->C[l]));
    NACK(nalloc(N, &N->g2[l], Vl * N->C[l]));
    if (l > 0) {
      NACK(nalloc(N, &N->p[l], Vl * N->C[l - 1]));
      NACK(nalloc(N, &N->gpool[l], Vl * N->C[l - 1]));
    }
    if (l <= L - 2) {
      NACK(nalloc(N, &N->up[l], Vl * N->C[l + 1]));
      NACK(nalloc(N, &N->h[l], Vl * N->C[l]));
      NACK(nalloc(N, &N->d[l], Vl * N->C[l]));
      NACK(nalloc(N, &N->gup[l], Vl * N->C[l + 1]));
      NACK(nalloc(N, &N->gsk[l], Vl * N->C[l]));
    }
  }
  NACK(nalloc(N, &N->u, E));
  NACK(nalloc(N, &N->du, E));
  NACK(nalloc(N, &N->gn, N->g.nn));
  NACK(nalloc(N, &N->lpart, nblk(N->g.nn)));
  NACK(nalloc(N, &N->loss, 1));
  NACK(nalloc(N, &N->hpart, (long long)nblk(E) * (N->C[0] + 1)));
  // weight-gradient partials: at least one block of the largest layer, at
  // most 16 Mi floats
  N->wpart_cap = std::max<long long>(wmax, 16LL << 20);
  NACK(nalloc(N, &N->wpart, N->wpart_cap));
  N->bpart_cap = 512LL * 128;
  NACK(nalloc(N, &N->bpart, N->bpart_cap));
  NACK(pack_weights(N));
  NHIP(hipStreamSynchronize(N->s));
  return MGAR_OK;
}

}  // namespace

extern "C" {

void mgar_net_destroy(mgar_net* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->s);   // work still queued on the network's stream reads these buffers
  for (void* p : n->allocs) (void)hipFree(p);
  delete n;
}

int mgar_net_create(const mgar_params* p, int levels, const int* channels, void* stream, mgar_net** out) {
  if (!p || !out) return MGAR_E_ARG;
  *out = nullptr;
  mgar_net* N = new mgar_net();
  const int rc = create_impl(N, p, levels, channels, stream);
  if (rc != MGAR_OK) {
    mgar_net_destroy(N);
    return rc;
  }
  *out = N;
  return MGAR_OK;
}

int mgar_net_sizes(const mgar_net* n, long long* nparams) {
  if (!n || !nparams) return MGAR_E_ARG;
  *nparams = n->np;
  return MGAR_OK;
}

int mgar_net_set_source(mgar_net* n, const double* qe) {
  if (!n || !qe) return MGAR_E_ARG;
  const long long E = n->V[0];
  std::vector<double> h((size_t)E);
  NHIP(hipMemcpyAsync(h.data(), qe, sizeof(double) * (size_t)E, hipMemcpyDeviceToHost, n->s));
  NHIP(hipStreamSynchronize(n->s));
  double mx = 0.0;
  for (double v : h) mx = std::max(mx, std::fabs(v));
  std::vector<float> f((size_t)E);
  for (long long e = 0; e < E; ++e) f[(size_t)e] = mx > 0.0 ? (float)(h[(size_t)e] / mx) : 0.0f;
  NHIP(hipMemcpyAsync(n->src, f.data(), sizeof(float) * (size_t)E, hipMemcpyHostToDevice, n->s));
  NHIP(hipStreamSynchronize(n->s));
  return MGAR_OK;
}

int mgar_net_set_params(mgar_net* n, const float* theta) {
  if (!n || !theta) return MGAR_E_ARG;
  NHIP(hipMemcpyAsync(n->theta, theta, sizeof(float) * (size_t)n->np, hipMemcpyHostToDevice, n->s));
  NHIP(hipMemsetAsync(n->m, 0, sizeof(float) * (size_t)n->np, n->s));
  NHIP(hipMemsetAsync(n->v, 0, sizeof(float) * (size_t)n->np, n->s));
  NACK(pack_weights(n));
  NHIP(hipStreamSynchronize(n->s));
  n->t = 0;
  return MGAR_OK;
}

int mgar_net_get_params(const mgar_net* n, float* theta) {
  if (!n || !theta) return MGAR_E_ARG;
  NHIP(hipMemcpyAsync(theta, n->theta, sizeof(float) * (size_t)n->np, hipMemcpyDeviceToHost, n->s));
  NHIP(hipStreamSynchronize(n->s));
  return MGAR_OK;
}

int mgar_net_infer(mgar_net* n, const double* xphys, double scale, double* T) {
  if (!n || !xphys || !T) return MGAR_E_ARG;
  NACK(forward(n, xphys));
  hipLaunchKernelGGL(k_to_nodes, dim3(nblk(n->g.nn)), dim3(NB), 0, n->s, n->g, (const float*)n->u, scale, T);
  NLAUNCH();
  return MGAR_OK;
}

int mgar_net_output(const mgar_net* n, float* u) {
  if (!n || !u) return MGAR_E_ARG;
  NHIP(hipMemcpyAsync(u, n->u, sizeof(float) * (size_t)n->V[0], hipMemcpyDeviceToHost, n->s));
  NHIP(hipStreamSynchronize(n->s));
  return MGAR_OK;
}

int mgar_net_grad(mgar_net* n, const double* xphys, const double* T, double scale, double* grad, double* loss) {
  if (!n || !xphys || !T || !(scale > 0.0)) return MGAR_E_ARG;
  NACK(loss_grad(n, xphys, T, scale));
  if (grad) NHIP(hipMemcpyAsync(grad, n->grad, sizeof(double) * (size_t)n->np, hipMemcpyDeviceToHost, n->s));
  if (loss) NHIP(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->s));
  NHIP(hipStreamSynchronize(n->s));
  return MGAR_OK;
}

int mgar_net_train_step(mgar_net* n, const double* xphys, const double* T, double scale, double lr,
                        double* loss) {
  if (!n || !xphys || !T || !(scale > 0.0) || !(lr > 0.0)) return MGAR_E_ARG;
  NACK(loss_grad(n, xphys, T, scale));
  n->t += 1;
  const double c1 = 1.0 - std::pow(0.9, n->t), c2 = 1.0 - std::pow(0.999, n->t);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n->np)), dim3(NB), 0, n->s, n->theta, n->m, n->v, (const double*)n->grad,
                     n->np, lr, c1, c2);
  NLAUNCH();
  NACK(pack_weights(n));
  if (loss) {
    NHIP(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->s));
    NHIP(hipStreamSynchronize(n->s));
  }
  return MGAR_OK;
}

}  // extern "C"
