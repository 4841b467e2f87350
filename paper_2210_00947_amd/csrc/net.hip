// Learned initial guess: a small 3D convolutional U-Net on a coarse cell grid
// (blocks of f^3 finest elements), trained online on the (density,
// temperature) pairs of the optimisation loop, by the kernels of this file:
// forward, backward and Adam. FP32 storage; the 27 taps of one source
// channel (and, for weight gradients, a thread's few voxels) are summed in
// FP32, every longer sum in FP64.
//
// Network: in(2) -> conv+ReLU (C1) -> conv+ReLU (C1) = skip -> 2x avg pool ->
// conv+ReLU (C2) -> conv+ReLU (C2) -> 2x nearest up -> concat [up, skip] ->
// conv+ReLU (C1) -> conv (1) = u. Convolutions: 3x3x3 cross-correlation, zero
// padding 1, weights [co][ci][dz][dy][dx] then biases per layer in one flat
// FP32 vector (layers in the order above). Activations are [channel][z][y][x].
// Input channels: mean physical density of the block; fraction of the
// block's 8 corner nodes that are Dirichlet nodes. Prediction on the finest
// nodes: scale * trilinear interpolation of u between coarse cell centres
// (finest nodes f*i + f/2), clamped at the outermost centres, Dirichlet 0.
// Training target: y = T at the centre nodes / scale; loss = mean (u - y)^2.
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
constexpr int NBC = 64;   // voxels per block of the forward and data-gradient convolutions

__device__ inline int cidx(int c, int z, int y, int x, int D, int H, int W) {
  return ((c * D + z) * H + y) * W + x;
}

// ---------------------------------------------------------------- grid <-> net

__global__ __launch_bounds__(NB) void k_net_input(Geo g, const double* __restrict__ xphys, int f, int D,
                                                  int H, int W, float* __restrict__ in) {
  const int v = blockIdx.x * NB + threadIdx.x;
  const int V = D * H * W;
  if (v >= V) return;
  const int i = v % W, j = (v / W) % H, k = v / (W * H);
  double s = 0.0;
  for (int c = 0; c < f; ++c)
    for (int b = 0; b < f; ++b)
      for (int a = 0; a < f; ++a) s += xphys[geo_elem(g, f * i + a, f * j + b, f * k + c)];
  int cnt = 0;
  for (int c = 0; c < 8; ++c)
    cnt += geo_fixed(g, f * (i + (c & 1)), f * (j + ((c >> 1) & 1)), f * (k + ((c >> 2) & 1))) ? 1 : 0;
  in[v] = (float)(s / (double)(f * f * f));
  in[V + v] = (float)(cnt / 8.0);
}

__global__ __launch_bounds__(NB) void k_net_target(Geo g, const double* __restrict__ T, int f, int D,
                                                   int H, int W, double inv_scale, float* __restrict__ y) {
  const int v = blockIdx.x * NB + threadIdx.x;
  if (v >= D * H * W) return;
  const int i = v % W, j = (v / W) % H, k = v / (W * H);
  const int h = f / 2;
  y[v] = (float)(T[geo_node(g, f * i + h, f * j + h, f * k + h)] * inv_scale);
}

__device__ inline void axis_w(int n, int f, int ncell, int& i0, int& i1, double& w) {
  double p = ((double)n - 0.5 * f) / (double)f;
  p = fmin(fmax(p, 0.0), (double)(ncell - 1));
  i0 = min((int)floor(p), ncell - 1);
  i1 = min(i0 + 1, ncell - 1);
  w = p - (double)i0;
}

__global__ __launch_bounds__(NB) void k_net_to_nodes(Geo g, const float* __restrict__ u, int f, int D,
                                                     int H, int W, double scale, double* __restrict__ T) {
  const long long n = blockIdx.x * (long long)NB + threadIdx.x;
  if (n >= g.nn) return;
  const int i = (int)(n % g.nnx);
  const long long r = n / g.nnx;
  const int j = (int)(r % g.nny), k = (int)(r / g.nny);
  if (geo_fixed(g, i, j, k)) {
    T[n] = 0.0;
    return;
  }
  int x0, x1, y0, y1, z0, z1;
  double wx, wy, wz;
  axis_w(i, f, W, x0, x1, wx);
  axis_w(j, f, H, y0, y1, wy);
  axis_w(k, f, D, z0, z1, wz);
  auto U = [&](int z, int y, int x) { return (double)u[(z * H + y) * W + x]; };
  const double s = (1 - wz) * ((1 - wy) * ((1 - wx) * U(z0, y0, x0) + wx * U(z0, y0, x1)) +
                               wy * ((1 - wx) * U(z0, y1, x0) + wx * U(z0, y1, x1))) +
                   wz * ((1 - wy) * ((1 - wx) * U(z1, y0, x0) + wx * U(z1, y0, x1)) +
                         wy * ((1 - wx) * U(z1, y1, x0) + wx * U(z1, y1, x1)));
  T[n] = scale * s;
}

// ---------------------------------------------------------------- layers

// Forward and data-gradient convolutions share one kernel: dst[d][v] =
// bias[d] + sum_s sum_taps wt(d, s, t) src[s][v + sgn (t - 1)], with
//   forward:        src = in,   d = co, s = ci, wt = w[co][ci][t],      sgn = +1;
//   data gradient:  src = gout, d = ci, s = co, wt = w[co][ci][t],      sgn = -1
// (zero padding; the bias only in the forward, optional ReLU). One thread per
// voxel and group of CT destination channels (blockIdx.y); the 27 taps of a
// source channel are summed in FP32, the source channels in FP64. Taps
// outside the grid load a clamped neighbour weighted 0 (no branch between the
// loads).
constexpr int CT = 4;

template <bool FWD, bool RELU>
__global__ __launch_bounds__(NBC) void k_conv(const float* __restrict__ src, int Cs,
                                              const float* __restrict__ w, const float* __restrict__ bias,
                                              float* __restrict__ dst, int Cd, int D, int H, int W) {
  const int V = D * H * W;
  const int v = blockIdx.x * NBC + threadIdx.x;
  if (v >= V) return;
  const int c0 = blockIdx.y * CT;
  const int x = v % W, y = (v / W) % H, z = v / (W * H);
  constexpr int sg = FWD ? 1 : -1;
  double s[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) s[c] = FWD ? (double)bias[min(c0 + c, Cd - 1)] : 0.0;
  for (int sc = 0; sc < Cs; ++sc) {
    float xin[27];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int zz = z + sg * (dz - 1), yy = y + sg * (dy - 1), xx = x + sg * (dx - 1);
          const bool ok = zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
          const float val = src[cidx(sc, min(max(zz, 0), D - 1), min(max(yy, 0), H - 1), min(max(xx, 0), W - 1),
                                     D, H, W)];
          xin[(dz * 3 + dy) * 3 + dx] = val * (ok ? 1.0f : 0.0f);
        }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int d = min(c0 + c, Cd - 1);
      const float* wp = w + (FWD ? (d * Cs + sc) : (sc * Cd + d)) * 27;
      float t = 0.0f;
#pragma unroll
      for (int q = 0; q < 27; ++q) t += wp[q] * xin[q];
      s[c] += (double)t;
    }
  }
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (c0 + c >= Cd) break;
    const float f = (float)s[c];
    dst[(c0 + c) * V + v] = RELU ? fmaxf(f, 0.0f) : f;
  }
}

// gw[co][ci][t] = sum_v gout[co][v] in[ci][v + t - 1]; gb[co] = sum_v gout[co][v],
// in two stages. Block (ci, group of WCT output channels, slab s) stages input
// channel ci over its slab (wz planes x hy rows x all W columns) plus a one-voxel
// zero halo in LDS, so the 27 taps of a voxel are plain LDS reads shared by the
// WCT channels. Each thread sums the products of its voxels (at most a few
// dozen) in FP32; from there on the sums are FP64, in a fixed order (see the
// block sums below), and part holds 28 sums (27 taps, then the bias term) per
// (co, ci, s). k_conv_bwd_weight_sum adds the
// slabs in order.
constexpr int WCT = 2;          // output channels per block
constexpr int WLDS = 12288;     // floats of the staged slab (48 KiB)

// Slab shape for a D x H x W grid and a layer of ci -> co channels: wz planes
// (at most 8; thinner while the launch would have fewer than 512 blocks, down
// to 2) and hy rows, whose haloed tile fits WLDS floats. Returns the number of
// slabs, or 0 if even a 1 x 1 slab does not fit (W too large).
int weight_slabs(int D, int H, int W, int ci, int co, int* wz, int* hy) {
  const long long cg = (co + WCT - 1) / WCT;
  int z = std::min(D, 8), y = H;
  auto slabs = [&]() { return (long long)((D + z - 1) / z) * ((H + y - 1) / y); };
  while (z > 2 && ci * cg * slabs() < 512) z = (z + 1) / 2;
  while ((long long)(z + 2) * (y + 2) * (W + 2) > WLDS) {
    if (z > 1) z = (z + 1) / 2;
    else if (y > 1) y = (y + 1) / 2;
    else return 0;
  }
  *wz = z;
  *hy = y;
  return (int)slabs();
}

__global__ __launch_bounds__(NB) void k_conv_bwd_weight_lds(const float* __restrict__ in, int Ci,
                                                            const float* __restrict__ gout, int Co,
                                                            double* __restrict__ part, int D, int H, int W,
                                                            int wz, int hy) {
  __shared__ float tile[WLDS];
  static_assert(28 * (NB + NB / 32) <= WLDS, "the block sums reuse the tile");
  const int ci = blockIdx.x, co0 = blockIdx.y * WCT, sl = blockIdx.z, S = gridDim.z;
  const int nys = (H + hy - 1) / hy;
  const int z0 = (sl / nys) * wz, y0 = (sl % nys) * hy;
  const int nz = min(wz, D - z0), ny = min(hy, H - y0);
  const int PW = W + 2, PH = ny + 2, PP = PW * PH;
  const int V = D * H * W;
  // planes z0-1 .. z0+nz, rows y0-1 .. y0+ny, columns -1 .. W; zero outside the
  // grid. Sixteen loads per thread are issued before their stores.
  const int nt = (nz + 2) * PP;
  for (int t0 = threadIdx.x; t0 < nt; t0 += 16 * NB) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = t0 + u * NB;
      const int lz = t / PP, rem = t - lz * PP, ly = rem / PW, lx = rem - ly * PW;
      const int z = z0 - 1 + lz, y = y0 - 1 + ly, x = lx - 1;
      const bool ok = t < nt && z >= 0 && z < D && y >= 0 && y < H && x >= 0 && x < W;
      v[u] = ok ? in[cidx(ci, z, y, x, D, H, W)] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (t0 + u * NB < nt) tile[t0 + u * NB] = v[u];
  }
  __syncthreads();
  float acc[WCT][28];
#pragma unroll
  for (int c = 0; c < WCT; ++c)
#pragma unroll
    for (int q = 0; q < 28; ++q) acc[c][q] = 0.0f;
  const int nv = nz * ny * W;
#pragma unroll 2
  for (int t = threadIdx.x; t < nv; t += NB) {
    const int x = t % W, r = t / W, ly = r % ny, lz = r / ny;
    const int v = ((z0 + lz) * H + (y0 + ly)) * W + x;
    const int c = ((lz + 1) * PH + (ly + 1)) * PW + (x + 1);   // the voxel in the tile
    float g[WCT];
#pragma unroll
    for (int k = 0; k < WCT; ++k) g[k] = (co0 + k < Co) ? gout[(co0 + k) * V + v] : 0.0f;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const float tv = tile[c + (dz - 1) * PP + (dy - 1) * PW + (dx - 1)];
#pragma unroll
          for (int k = 0; k < WCT; ++k) acc[k][(dz * 3 + dy) * 3 + dx] += g[k] * tv;
        }
#pragma unroll
    for (int k = 0; k < WCT; ++k) acc[k][27] += g[k];
  }
  // block sums through LDS (the tile is no longer read): per output channel,
  // thread t stores its 28 partials at red[q * RS + t + t / 32]; then thread
  // r < 224 sums, in FP64 and in order, the 32 partials of threads
  // 32 (r % 8) .. 32 (r % 8) + 31 for output q = r / 8, and the eight lanes of
  // each q add their sums by three shuffles (the same total in each lane)
  constexpr int RS = NB + NB / 32;
  float* red = tile;
  const int r = threadIdx.x, q = r >> 3, sg = r & 7;
#pragma unroll
  for (int k = 0; k < WCT; ++k) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 28; ++j) red[j * RS + r + (r >> 5)] = acc[k][j];
    __syncthreads();
    double sum = 0.0;
    if (q < 28) {
      const float* src = red + q * RS + sg * 33;
      for (int i = 0; i < 32; ++i) sum += (double)src[i];
    }
    sum += __shfl_xor(sum, 4, 8);
    sum += __shfl_xor(sum, 2, 8);
    sum += __shfl_xor(sum, 1, 8);
    if (q < 28 && sg == 0 && co0 + k < Co) part[(((co0 + k) * Ci + ci) * S + sl) * 28 + q] = sum;
  }
}

__global__ __launch_bounds__(NB) void k_conv_bwd_weight_sum(const double* __restrict__ part, int Ci, int Co,
                                                            int S, float* __restrict__ gw,
                                                            float* __restrict__ gb) {
  const int q = blockIdx.x * NB + threadIdx.x;   // (co * Ci + ci) * 28 + t
  if (q >= Co * Ci * 28) return;
  const int t = q % 28, cc = q / 28, ci = cc % Ci, co = cc / Ci;
  double s = 0.0;
  for (int sl = 0; sl < S; ++sl) s += part[(cc * S + sl) * 28 + t];
  if (t < 27) gw[cc * 27 + t] = (float)s;
  else if (ci == 0) gb[co] = (float)s;
}

__global__ __launch_bounds__(NB) void k_relu_bwd(float* __restrict__ g, const float* __restrict__ act, int n) {
  const int i = blockIdx.x * NB + threadIdx.x;
  if (i < n && !(act[i] > 0.0f)) g[i] = 0.0f;
}

// out[c][Z][Y][X] = mean of the 2x2x2 children (C channels, fine D x H x W)
__global__ __launch_bounds__(NB) void k_pool2(const float* __restrict__ in, float* __restrict__ out, int C,
                                              int D, int H, int W) {
  const int d = D / 2, h = H / 2, w = W / 2;
  const int v = blockIdx.x * NB + threadIdx.x;
  if (v >= C * d * h * w) return;
  const int X = v % w, Y = (v / w) % h, Z = (v / (w * h)) % d, c = v / (w * h * d);
  double s = 0.0;
  for (int a = 0; a < 8; ++a)
    s += (double)in[cidx(c, 2 * Z + ((a >> 2) & 1), 2 * Y + ((a >> 1) & 1), 2 * X + (a & 1), D, H, W)];
  out[v] = (float)(s * 0.125);
}

// g_fine[c][z][y][x] = g_coarse[c][z/2][y/2][x/2] / 8 + add[c][z][y][x]
__global__ __launch_bounds__(NB) void k_pool2_bwd(const float* __restrict__ gc, const float* __restrict__ add,
                                                  float* __restrict__ gf, int C, int D, int H, int W) {
  const int v = blockIdx.x * NB + threadIdx.x;
  if (v >= C * D * H * W) return;
  const int x = v % W, y = (v / W) % H, z = (v / (W * H)) % D, c = v / (W * H * D);
  gf[v] = (float)((double)gc[cidx(c, z / 2, y / 2, x / 2, D / 2, H / 2, W / 2)] * 0.125 + (double)add[v]);
}

// out[c][z][y][x] = in[c][z/2][y/2][x/2] (fine D x H x W)
__global__ __launch_bounds__(NB) void k_up2(const float* __restrict__ in, float* __restrict__ out, int C,
                                            int D, int H, int W) {
  const int v = blockIdx.x * NB + threadIdx.x;
  if (v >= C * D * H * W) return;
  const int x = v % W, y = (v / W) % H, z = (v / (W * H)) % D, c = v / (W * H * D);
  out[v] = in[cidx(c, z / 2, y / 2, x / 2, D / 2, H / 2, W / 2)];
}

// g_coarse = sum of the 8 children of the fine gradient
__global__ __launch_bounds__(NB) void k_up2_bwd(const float* __restrict__ gf, float* __restrict__ gc, int C,
                                                int D, int H, int W) {
  const int d = D / 2, h = H / 2, w = W / 2;
  const int v = blockIdx.x * NB + threadIdx.x;
  if (v >= C * d * h * w) return;
  const int X = v % w, Y = (v / w) % h, Z = (v / (w * h)) % d, c = v / (w * h * d);
  double s = 0.0;
  for (int a = 0; a < 8; ++a)
    s += (double)gf[cidx(c, 2 * Z + ((a >> 2) & 1), 2 * Y + ((a >> 1) & 1), 2 * X + (a & 1), D, H, W)];
  gc[v] = (float)s;
}

// g = 2 (u - y) / V; partial sums of (u - y)^2 per block
__global__ __launch_bounds__(NB) void k_mse(const float* __restrict__ u, const float* __restrict__ y, int V,
                                            float* __restrict__ g, double* __restrict__ part) {
  __shared__ double sh[NB / MGAR_WAVE];
  const int v = blockIdx.x * NB + threadIdx.x;
  double e = 0.0;
  if (v < V) {
    const double d = (double)u[v] - (double)y[v];
    g[v] = (float)(2.0 * d / (double)V);
    e = d * d;
  }
  const double s = block_sum(e, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_sum_to(const double* __restrict__ part, int n, double scale,
                                                 double* __restrict__ out) {
  __shared__ double sh[1024 / MGAR_WAVE];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = s * scale;
}

__global__ __launch_bounds__(NB) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                             const float* __restrict__ g, long long n, double lr, double c1,
                                             double c2) {
  const long long i = blockIdx.x * (long long)NB + threadIdx.x;
  if (i >= n) return;
  const double gi = (double)g[i];
  const double mi = 0.9 * (double)m[i] + 0.1 * gi;
  const double vi = 0.999 * (double)v[i] + 0.001 * gi * gi;
  m[i] = (float)mi;
  v[i] = (float)vi;
  p[i] = (float)((double)p[i] - lr * (mi / c1) / (sqrt(vi / c2) + 1e-8));
}

int nblk(long long n) { return (int)((n + NB - 1) / NB); }

}  // namespace

struct mgar_net {
  hipStream_t s = nullptr;
  Geo g;
  int f = 4, D = 0, H = 0, W = 0, c1 = 0, c2 = 0;
  long long np = 0;
  long long woff[6], boff[6];
  int co[6], ci[6];
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  float *in = nullptr, *a1 = nullptr, *a2 = nullptr, *pool = nullptr, *a3 = nullptr, *a4 = nullptr,
        *cat = nullptr, *a5 = nullptr, *u = nullptr, *y = nullptr;
  float *gU = nullptr, *gA5 = nullptr, *gCat = nullptr, *gA4 = nullptr, *gA3 = nullptr, *gPool = nullptr,
        *gA2 = nullptr, *gA1 = nullptr;
  double *part = nullptr, *loss = nullptr;
  double* wpart = nullptr;   // per-slab partial sums of the weight gradients
  int t = 0;   // Adam steps taken
};

namespace {

int conv(mgar_net* N, int layer, const float* in, float* out, bool relu, int D, int H, int W) {
  const dim3 grid((unsigned)((D * H * W + NBC - 1) / NBC), (N->co[layer] + CT - 1) / CT);
  const dim3 blk(NBC);
  const float* w = N->theta + N->woff[layer];
  const float* b = N->theta + N->boff[layer];
  if (relu) k_conv<true, true><<<grid, blk, 0, N->s>>>(in, N->ci[layer], w, b, out, N->co[layer], D, H, W);
  else k_conv<true, false><<<grid, blk, 0, N->s>>>(in, N->ci[layer], w, b, out, N->co[layer], D, H, W);
  NLAUNCH();
  return MGAR_OK;
}

// weight and bias gradients of `layer`, and (gin != null) its input gradient
int conv_bwd(mgar_net* N, int layer, const float* in, const float* gout, float* gin, int D, int H, int W) {
  int wz = 0, hy = 0;
  const int S = weight_slabs(D, H, W, N->ci[layer], N->co[layer], &wz, &hy);
  if (S <= 0) return MGAR_E_ARG;
  const dim3 gw(N->ci[layer], (N->co[layer] + WCT - 1) / WCT, S);
  k_conv_bwd_weight_lds<<<gw, NB, 0, N->s>>>(in, N->ci[layer], gout, N->co[layer], N->wpart, D, H, W, wz, hy);
  k_conv_bwd_weight_sum<<<nblk((long long)N->co[layer] * N->ci[layer] * 28), NB, 0, N->s>>>(
      N->wpart, N->ci[layer], N->co[layer], S, N->grad + N->woff[layer], N->grad + N->boff[layer]);
  if (gin) {
    const dim3 gd((unsigned)((D * H * W + NBC - 1) / NBC), (N->ci[layer] + CT - 1) / CT);
    k_conv<false, false><<<gd, NBC, 0, N->s>>>(gout, N->co[layer], N->theta + N->woff[layer], nullptr,
                                                         gin, N->ci[layer], D,
                                         H, W);
  }
  NLAUNCH();
  return MGAR_OK;
}

int forward(mgar_net* N, const double* xphys) {
  const int D = N->D, H = N->H, W = N->W, V = D * H * W;
  const int d = D / 2, h = H / 2, w = W / 2;
  k_net_input<<<nblk(V), NB, 0, N->s>>>(N->g, xphys, N->f, D, H, W, N->in);
  NACK(conv(N, 0, N->in, N->a1, true, D, H, W));
  NACK(conv(N, 1, N->a1, N->a2, true, D, H, W));
  k_pool2<<<nblk((long long)N->c1 * d * h * w), NB, 0, N->s>>>(N->a2, N->pool, N->c1, D, H, W);
  NACK(conv(N, 2, N->pool, N->a3, true, d, h, w));
  NACK(conv(N, 3, N->a3, N->a4, true, d, h, w));
  k_up2<<<nblk((long long)N->c2 * V), NB, 0, N->s>>>(N->a4, N->cat, N->c2, D, H, W);
  NHIP(hipMemcpyAsync(N->cat + (long long)N->c2 * V, N->a2, sizeof(float) * (size_t)N->c1 * V,
                      hipMemcpyDeviceToDevice, N->s));
  NACK(conv(N, 4, N->cat, N->a5, true, D, H, W));
  NACK(conv(N, 5, N->a5, N->u, false, D, H, W));
  NLAUNCH();
  return MGAR_OK;
}

// loss and parameter gradient for the pair (xphys, T / scale)
int loss_grad(mgar_net* N, const double* xphys, const double* T, double scale) {
  const int D = N->D, H = N->H, W = N->W, V = D * H * W;
  const int d = D / 2, h = H / 2, w = W / 2, V8 = d * h * w;
  NACK(forward(N, xphys));
  k_net_target<<<nblk(V), NB, 0, N->s>>>(N->g, T, N->f, D, H, W, 1.0 / scale, N->y);
  k_mse<<<nblk(V), NB, 0, N->s>>>(N->u, N->y, V, N->gU, N->part);
  k_sum_to<<<1, 1024, 0, N->s>>>(N->part, nblk(V), 1.0 / (double)V, N->loss);
  NACK(conv_bwd(N, 5, N->a5, N->gU, N->gA5, D, H, W));
  k_relu_bwd<<<nblk((long long)N->c1 * V), NB, 0, N->s>>>(N->gA5, N->a5, N->c1 * V);
  NACK(conv_bwd(N, 4, N->cat, N->gA5, N->gCat, D, H, W));
  k_up2_bwd<<<nblk((long long)N->c2 * V8), NB, 0, N->s>>>(N->gCat, N->gA4, N->c2, D, H, W);
  k_relu_bwd<<<nblk((long long)N->c2 * V8), NB, 0, N->s>>>(N->gA4, N->a4, N->c2 * V8);
  NACK(conv_bwd(N, 3, N->a3, N->gA4, N->gA3, d, h, w));
  k_relu_bwd<<<nblk((long long)N->c2 * V8), NB, 0, N->s>>>(N->gA3, N->a3, N->c2 * V8);
  NACK(conv_bwd(N, 2, N->pool, N->gA3, N->gPool, d, h, w));
  k_pool2_bwd<<<nblk((long long)N->c1 * V), NB, 0, N->s>>>(N->gPool, N->gCat + (long long)N->c2 * V, N->gA2,
                                                            N->c1, D, H, W);
  k_relu_bwd<<<nblk((long long)N->c1 * V), NB, 0, N->s>>>(N->gA2, N->a2, N->c1 * V);
  NACK(conv_bwd(N, 1, N->a1, N->gA2, N->gA1, D, H, W));
  k_relu_bwd<<<nblk((long long)N->c1 * V), NB, 0, N->s>>>(N->gA1, N->a1, N->c1 * V);
  NACK(conv_bwd(N, 0, N->in, N->gA1, nullptr, D, H, W));
  NLAUNCH();
  return MGAR_OK;
}

template <typename T>
int nalloc(T** p, long long n) {
  *p = nullptr;
  NHIP(hipMalloc((void**)p, sizeof(T) * (size_t)(n > 0 ? n : 1)));
  return MGAR_OK;
}

}  // namespace

extern "C" {

void mgar_net_destroy(mgar_net* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->s);   // work still queued on the network's stream reads these buffers
  for (void* p : {(void*)n->theta, (void*)n->grad, (void*)n->m, (void*)n->v, (void*)n->in, (void*)n->a1,
                  (void*)n->a2, (void*)n->pool, (void*)n->a3, (void*)n->a4, (void*)n->cat, (void*)n->a5,
                  (void*)n->u, (void*)n->y, (void*)n->gU, (void*)n->gA5, (void*)n->gCat, (void*)n->gA4,
                  (void*)n->gA3, (void*)n->gPool, (void*)n->gA2, (void*)n->gA1, (void*)n->part,
                  (void*)n->loss, (void*)n->wpart})
    if (p) (void)hipFree(p);
  delete n;
}

static int net_create_impl(const mgar_params* p, int pool, int c1, int c2, void* stream, mgar_net* N) {
  NACK(mgar_internal_validate(p));
  if (p->dim != 3) return MGAR_E_ARG;
  if (pool < 2 || (pool & 1) || c1 < 1 || c2 < 1 || c1 > 256 || c2 > 256) return MGAR_E_ARG;
  if (p->nelx % (2 * pool) || p->nely % (2 * pool) || p->nelz % (2 * pool)) return MGAR_E_DIMS;
  N->s = (hipStream_t)stream;
  N->g = mgar_internal_geo(*p, 0);
  N->f = pool;
  N->W = p->nelx / pool;
  N->H = p->nely / pool;
  N->D = p->nelz / pool;
  N->c1 = c1;
  N->c2 = c2;
  const int cos[6] = {c1, c1, c2, c2, c1, 1}, cis[6] = {2, c1, c1, c2, c2 + c1, c1};
  long long off = 0;
  for (int l = 0; l < 6; ++l) {
    N->co[l] = cos[l];
    N->ci[l] = cis[l];
    N->woff[l] = off;
    off += (long long)cos[l] * cis[l] * 27;
    N->boff[l] = off;
    off += cos[l];
  }
  N->np = off;
  const long long V = (long long)N->D * N->H * N->W, V8 = V / 8;
  NACK(nalloc(&N->theta, off));
  NACK(nalloc(&N->grad, off));
  NACK(nalloc(&N->m, off));
  NACK(nalloc(&N->v, off));
  NHIP(hipMemset(N->theta, 0, sizeof(float) * off));
  NHIP(hipMemset(N->m, 0, sizeof(float) * off));
  NHIP(hipMemset(N->v, 0, sizeof(float) * off));
  NACK(nalloc(&N->in, 2 * V));
  NACK(nalloc(&N->a1, c1 * V));
  NACK(nalloc(&N->a2, c1 * V));
  NACK(nalloc(&N->pool, c1 * V8));
  NACK(nalloc(&N->a3, c2 * V8));
  NACK(nalloc(&N->a4, c2 * V8));
  NACK(nalloc(&N->cat, (c2 + c1) * V));
  NACK(nalloc(&N->a5, c1 * V));
  NACK(nalloc(&N->u, V));
  NACK(nalloc(&N->y, V));
  NACK(nalloc(&N->gU, V));
  NACK(nalloc(&N->gA5, c1 * V));
  NACK(nalloc(&N->gCat, (c2 + c1) * V));
  NACK(nalloc(&N->gA4, c2 * V8));
  NACK(nalloc(&N->gA3, c2 * V8));
  NACK(nalloc(&N->gPool, c1 * V8));
  NACK(nalloc(&N->gA2, c1 * V));
  NACK(nalloc(&N->gA1, c1 * V));
  NACK(nalloc(&N->part, nblk(V)));
  NACK(nalloc(&N->loss, 1));
  {
    // layers 2 and 3 run on the pooled grid, the others on the cell grid
    long long mx = 0;
    for (int l = 0; l < 6; ++l) {
      const bool half = l == 2 || l == 3;
      int wz = 0, hy = 0;
      const int S = half ? weight_slabs(N->D / 2, N->H / 2, N->W / 2, N->ci[l], N->co[l], &wz, &hy)
                         : weight_slabs(N->D, N->H, N->W, N->ci[l], N->co[l], &wz, &hy);
      if (S <= 0) return MGAR_E_ARG;   // cell grid too wide for the staged slab
      mx = std::max(mx, (long long)N->co[l] * N->ci[l] * S);
    }
    NACK(nalloc(&N->wpart, mx * 28));
  }
  return MGAR_OK;
}

int mgar_net_create(const mgar_params* p, int pool, int c1, int c2, void* stream, mgar_net** out) {
  if (!p || !out) return MGAR_E_ARG;
  *out = nullptr;
  mgar_net* N = new mgar_net();
  const int rc = net_create_impl(p, pool, c1, c2, stream, N);
  if (rc != MGAR_OK) {
    mgar_net_destroy(N);
    return rc;
  }
  *out = N;
  return MGAR_OK;
}

int mgar_net_sizes(const mgar_net* n, long long* nparams, int* cells) {
  if (!n || !nparams || !cells) return MGAR_E_ARG;
  *nparams = n->np;
  cells[0] = n->D;
  cells[1] = n->H;
  cells[2] = n->W;
  return MGAR_OK;
}

int mgar_net_set_params(mgar_net* n, const float* theta) {
  if (!n || !theta) return MGAR_E_ARG;
  NHIP(hipMemcpyAsync(n->theta, theta, sizeof(float) * (size_t)n->np, hipMemcpyHostToDevice, n->s));
  NHIP(hipMemsetAsync(n->m, 0, sizeof(float) * (size_t)n->np, n->s));
  NHIP(hipMemsetAsync(n->v, 0, sizeof(float) * (size_t)n->np, n->s));
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
  k_net_to_nodes<<<nblk(n->g.nn), NB, 0, n->s>>>(n->g, n->u, n->f, n->D, n->H, n->W, scale, T);
  NLAUNCH();
  return MGAR_OK;
}

int mgar_net_output(const mgar_net* n, float* u) {
  if (!n || !u) return MGAR_E_ARG;
  NHIP(hipMemcpyAsync(u, n->u, sizeof(float) * (size_t)n->D * n->H * n->W, hipMemcpyDeviceToHost, n->s));
  NHIP(hipStreamSynchronize(n->s));
  return MGAR_OK;
}

int mgar_net_grad(mgar_net* n, const double* xphys, const double* T, double scale, float* grad,
                  double* loss) {
  if (!n || !xphys || !T || !(scale > 0.0)) return MGAR_E_ARG;
  NACK(loss_grad(n, xphys, T, scale));
  if (grad) NHIP(hipMemcpyAsync(grad, n->grad, sizeof(float) * (size_t)n->np, hipMemcpyDeviceToHost, n->s));
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
  k_adam<<<nblk(n->np), NB, 0, n->s>>>(n->theta, n->m, n->v, n->grad, n->np, lr, c1, c2);
  NLAUNCH();
  if (loss) {
    NHIP(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->s));
    NHIP(hipStreamSynchronize(n->s));
  }
  return MGAR_OK;
}

}  // extern "C"
