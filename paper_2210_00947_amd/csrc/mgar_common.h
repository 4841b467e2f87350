// Internal definitions shared by the libmgar translation units: grid geometry
// of one MG level, device-side solver state, and wave64 reduction helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#define MGAR_WAVE 64
#define MGAR_MAXB 8

// Geometry of one grid level. In 2D nz = nnz = 1 so that E = nx*ny and
// N = nnx*nny under the same indexing formulas as 3D.
struct Geo {
  int dim;
  int nx, ny, nz;            // elements per axis
  int nnx, nny, nnz;         // nodes per axis
  int f0x, f1x, f0y, f1y, f0z, f1z;  // Dirichlet node box, inclusive (empty if f0 > f1)
  double h;                  // cell edge of this level (2^l)
  long long nn, ne;          // node and element counts
};

__host__ __device__ inline bool geo_fixed(const Geo& g, int i, int j, int k) {
  return i >= g.f0x && i <= g.f1x && j >= g.f0y && j <= g.f1y && k >= g.f0z && k <= g.f1z;
}

__host__ __device__ inline long long geo_node(const Geo& g, int i, int j, int k) {
  return (long long)i + (long long)g.nnx * ((long long)j + (long long)g.nny * k);
}

__host__ __device__ inline long long geo_elem(const Geo& g, int ex, int ey, int ez) {
  return (long long)ex + (long long)g.nx * ((long long)ey + (long long)g.ny * ez);
}

// Cell-conductivity loaders. Kernels read cell conductivities through one of
// these: an FP64 array, an FP32 array, or BF16-stored physical densities with
// the SIMP law (Eq 4, p = 3) applied in FP32 on load.
// Each loader also says how to turn one raw stored element (type E) into a
// conductivity, for kernels that fetch the raw elements themselves.
struct CellD {
  using E = double;
  const double* p;
  __device__ double operator()(long long e) const { return p[e]; }
  __device__ double value(double v) const { return v; }
};
struct CellF {
  using E = float;
  const float* p;
  __device__ float operator()(long long e) const { return p[e]; }
  __device__ float value(float v) const { return v; }
};
__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
  union { uint32_t u; float f; } v;
  v.u = (uint32_t)b << 16;
  return v.f;
}
struct CellB {
  using E = uint16_t;
  const uint16_t* p;
  float kmin, kdiff;
  __device__ float value(uint16_t h) const {
    const float r = bf16_bits_to_f32(h);
    return kmin + kdiff * (r * r * r);
  }
  __device__ float operator()(long long e) const { return value(p[e]); }
};

// PCG state in device memory. Every field has a single writer per kernel.
struct CgState {
  double qq;                 // ||q||^2 over free nodes
  double rr;                 // latest ||r||^2
  double rz[2];              // r.z by iteration parity
  double pw;                 // p.(K p)
  double pwh[2];             // p.(K p) by iteration parity (deferred x updates)
  int done;                  // set once the stopping test fires
  int iters;                 // iterations performed at exit
  int converged;             // 1 = tolerance met, 0 = cg_max reached
  int it;                    // iterations done so far (device counter: the launches
                             // of an iteration carry no host iteration index, so a
                             // captured iteration can be replayed)
  int itn;                   // it + 1, stored by the x/r update for a stopping test
                             // fused into a later kernel (whose blocks must not read
                             // it while its block 0 advances it)
  int flushed;               // iteration whose deferred x update k_cg_flush applied
                             // (-1: none); the next odd update leaves it out
};

// PCG state of one design of a batch. The iteration counter lives on the
// device, so one captured iteration can be replayed any number of times.
struct BCgState {
  double qq, rr;             // ||q||^2, latest ||r||^2
  double rz[2];              // r.z by iteration parity
  double pw;                 // p.(K p)
  int it;                    // iterations done
  int done;                  // stopping test fired (or design excluded from this solve)
  int conv;                  // 1 = tolerance met
  int pad;
};

// Reanalysis (reduced-basis) state in device memory.
struct MgarDev {
  double n0[MGAR_MAXB];      // squared column norm before projection
  double c[MGAR_MAXB];       // projection coefficients
  int active[MGAR_MAXB];     // 1 = column kept
  double KR[MGAR_MAXB * MGAR_MAXB];
  double qR[MGAR_MAXB];
  double y[MGAR_MAXB];
  double res2;               // ||K Q y - q||^2
  double qq;                 // ||q||^2
  int spd_fail;
  int pad;
  double nn[MGAR_MAXB];      // squared norm of each column after projection (fused Gram-Schmidt)
  double c2[MGAR_MAXB];      // coefficients of the second projection pass
};

// OC bisection state in device memory. The filtered volume S(lambda) is
// non-increasing in lambda, so evaluating it at candidate values brackets the
// root: lo_known is the largest evaluated lambda with S > target, hi_known the
// smallest with S <= target. Every bisection midpoint outside (lo_known,
// hi_known) is then decided without another evaluation.
#define OC_NCAND 15
struct OcDev {
  double l1, l2;             // current bisection bracket
  double lam_last;           // last midpoint the bisection evaluated
  double lo_known, hi_known; // evaluated bracket of the root
  double s_lo, s_hi;         // S at lo_known and hi_known (when evaluated)
  double cand[OC_NCAND];     // candidates for the next pass
  int done;
  int steps;                 // bisection steps replayed so far
  int pad[2];
};

// Bisection state of the boundary-smoothing level (Eq 24-27).
struct SmoothDev {
  double lo, hi;             // bracket: volume(lo) >= target > volume(hi)
  double width0;             // initial bracket width
  double vol;                // volume at lo after the final pass
  int steps, done;
};

// ---------------------------------------------------------------- reductions

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = MGAR_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, MGAR_WAVE);
  return v;
}

// This thread's share of a partial-sum vector: p[t] + p[t + nt] + ... in
// that order (starting from +0.0), with the first four loads issued together
// so that a short vector costs one memory round trip. Terms past n add +0.0,
// which leaves the sum bitwise unchanged.
__device__ inline double thread_partials(const double* __restrict__ p, int n, int t, int nt) {
  double a[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = t + u * nt;
    a[u] = i < n ? p[i] : 0.0;
  }
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) v += a[u];
  for (int i = t + 4 * nt; i < n; i += nt) v += p[i];
  return v;
}

// Deterministic block sum; result valid in every thread. `sh` needs
// blockDim/64 doubles of LDS. Contains __syncthreads (call from all threads).
__device__ inline double block_sum(double v, double* sh) {
  const int nt = blockDim.x * blockDim.y * blockDim.z;
  const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nw = (nt + MGAR_WAVE - 1) / MGAR_WAVE;
  v = wave_sum(v);
  __syncthreads();
  if ((t & (MGAR_WAVE - 1)) == 0) sh[t / MGAR_WAVE] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += sh[w];
  return s;
}

// Grid-level reduction without a second launch: every block stores its
// partial, then one thread per block bumps a device-scope counter; the block
// that sees the count reach nb sums all partials in index order (so the
// result is the same whichever block finishes last), writes *out and resets
// the counter. Returns true in the threads of that last block. Call from
// all threads; `s` must be valid in thread 0.
__device__ inline bool grid_reduce(double s, int bid, int nb, double* __restrict__ part,
                                   unsigned* __restrict__ cnt, double* __restrict__ out,
                                   double* sh, double* total) {
  __shared__ int last;
  const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nt = blockDim.x * blockDim.y * blockDim.z;
  if (t == 0) {
    part[bid] = s;
    __threadfence();
    last = (atomicAdd(cnt, 1u) == (unsigned)(nb - 1));
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double v = 0.0;
  for (int i = t; i < nb; i += nt) v += __builtin_nontemporal_load(part + i);
  v = block_sum(v, sh);
  if (t == 0) {
    if (out) *out = v;
    *cnt = 0u;
  }
  if (total) *total = v;
  return true;
}

__device__ inline int flat_tid() {
  return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
}

__device__ inline int flat_bid() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
