// Boundary-smoothing post-process (Sec. 2.3, Eq 24-27): element sensitivities
// projected onto the nodes with cone weights, then the level-set reading of
// Eq 24 with the intermediate density of Eq 25-27 counted on a lattice of
// sub-points, and the level found by bisection on the volume it keeps.
// Runs once after the optimisation loop; every step is on the device.
#include "mgar_launch.h"

namespace {

constexpr int TBX = 64, TBY = 4;
constexpr int VB = 256;
constexpr int VMAXB = 1024;

int nblocks(long long n) {
  long long nb = (n + VB - 1) / VB;
  return (int)(nb > VMAXB ? VMAXB : (nb < 1 ? 1 : nb));
}

// ns_i = sum_e w_ie (-dc_e) / sum_e w_ie, w_ie = max(0, r - |x_i - c_e|), over
// the elements e of the grid whose centroid c_e = (ex + 1/2, ...) is within r
// of node i = (i, j, k) (unit cells): the nodal sensitivity, large where
// material pays most.
template <int DIM>
__global__ __launch_bounds__(TBX* TBY) void k_node_project(Geo g, const double* __restrict__ dc, double r, int R,
                                                           double* __restrict__ ns) {
  const int i = blockIdx.x * TBX + threadIdx.x;
  const int j = blockIdx.y * TBY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nnx || j >= g.nny) return;
  double acc = 0.0, ws = 0.0;
  const int z0 = DIM == 3 ? max(k - R, 0) : 0, z1 = DIM == 3 ? min(k + R, g.nz) : 1;
  for (int ez = z0; ez < z1; ++ez) {
    const double dz = DIM == 3 ? (ez + 0.5 - k) : 0.0;
    for (int ey = max(j - R, 0); ey < min(j + R, g.ny); ++ey) {
      const double dy = ey + 0.5 - j;
      for (int ex = max(i - R, 0); ex < min(i + R, g.nx); ++ex) {
        const double dx = ex + 0.5 - i;
        const double w = r - sqrt(dx * dx + dy * dy + dz * dz);
        if (w > 0.0) {
          acc -= w * dc[geo_elem(g, ex, ey, ez)];
          ws += w;
        }
      }
    }
  }
  ns[geo_node(g, i, j, k)] = acc / ws;
}

// Block partials of min and max of v (2 values per block).
__global__ __launch_bounds__(VB) void k_minmax(const double* __restrict__ v, long long n, double* __restrict__ part) {
  __shared__ double lo[VB], hi[VB];
  double a = INFINITY, b = -INFINITY;
  for (long long t = blockIdx.x * (long long)VB + threadIdx.x; t < n; t += (long long)gridDim.x * VB) {
    a = fmin(a, v[t]);
    b = fmax(b, v[t]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int o = VB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + o]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = lo[0];
    part[2 * blockIdx.x + 1] = hi[0];
  }
}

// Bracket of the bisection: lo = min ns - 1 (every element solid), hi = max ns
// (every element void).
__global__ void k_smooth_init(SmoothDev* st, const double* __restrict__ part, int np) {
  if (threadIdx.x != 0) return;
  double a = INFINITY, b = -INFINITY;
  for (int q = 0; q < np; ++q) {
    a = fmin(a, part[2 * q]);
    b = fmax(b, part[2 * q + 1]);
  }
  st->lo = a - 1.0;
  st->hi = b;
  st->width0 = st->hi - st->lo;
  st->steps = 0;
  st->done = 0;
}

// Eq 24-27 for every element at the level of the current step (mid of the
// bracket; final = 1: the lower end), optional rho output, and the block
// partial of the volume in lattice-point counts (a solid element counts all
// (nsub+1)^d points): whole numbers, so their FP64 sum is exact in any order.
template <int DIM>
__global__ __launch_bounds__(TBX* TBY) void k_smooth_rho(Geo g, const double* __restrict__ ns, const SmoothDev* st,
                                                         int final_pass, int nsub, double* __restrict__ rho,
                                                         double* __restrict__ part) {
  __shared__ double sh[TBX * TBY / 64];
  if (!final_pass && st->done) return;
  const double level = final_pass ? st->lo : 0.5 * (st->lo + st->hi);
  const int ex = blockIdx.x * TBX + threadIdx.x;
  const int ey = blockIdx.y * TBY + threadIdx.y;
  const int ez = blockIdx.z;
  constexpr int NC = DIM == 3 ? 8 : 4;
  double v = 0.0;
  if (ex < g.nx && ey < g.ny) {
    double c[NC];
    bool above = true, below = true;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      c[q] = ns[geo_node(g, ex + (q & 1), ey + ((q >> 1) & 1), DIM == 3 ? ez + ((q >> 2) & 1) : 0)];
      above = above && c[q] > level;
      below = below && c[q] < level;
    }
    const int np1 = nsub + 1;
    const int npts = DIM == 3 ? np1 * np1 * np1 : np1 * np1;
    if (above) {
      v = (double)npts;
    } else if (!below) {
      // Eq 25-26 at the (nsub + 1)^d lattice points of local coordinates
      // -1 + 2 a / nsub, Eq 27: the points above the level
      int cnt = 0;
      for (int pz = 0; pz < (DIM == 3 ? np1 : 1); ++pz) {
        const double zt = DIM == 3 ? -1.0 + 2.0 * pz / nsub : 0.0;
        for (int py = 0; py < np1; ++py) {
          const double yt = -1.0 + 2.0 * py / nsub;
          for (int px = 0; px < np1; ++px) {
            const double xt = -1.0 + 2.0 * px / nsub;
            double val = 0.0;
#pragma unroll
            for (int q = 0; q < NC; ++q) {
              double w = (1.0 + xt * ((q & 1) ? 1.0 : -1.0)) * 0.5 * (1.0 + yt * ((q & 2) ? 1.0 : -1.0)) * 0.5;
              if (DIM == 3) w *= (1.0 + zt * ((q & 4) ? 1.0 : -1.0)) * 0.5;
              val += w * c[q];
            }
            cnt += val > level;
          }
        }
      }
      v = (double)cnt;
    }
    if (rho) rho[geo_elem(g, ex, ey, ez)] = v / (double)npts;
  }
  const double bs = block_sum(v, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    part[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = bs;
}

// One bisection step from the volume partials at mid (lattice-point counts):
// lo = mid if the count is >= target * npts, else hi = mid; done once the
// bracket is below 1e-14 of its initial width or after max_steps. final = 1:
// store the volume at lo (count / npts) instead.
__global__ __launch_bounds__(VB) void k_smooth_step(SmoothDev* st, const double* __restrict__ part, int np,
                                                    double target, int npts, int max_steps, int final_pass) {
  __shared__ double sh[VB / 64];
  if (!final_pass && st->done) return;
  double v = 0.0;
  for (int q = threadIdx.x; q < np; q += VB) v += part[q];
  const double vol = block_sum(v, sh);
  if (threadIdx.x != 0) return;
  if (final_pass) {
    st->vol = vol / (double)npts;
    return;
  }
  const double mid = 0.5 * (st->lo + st->hi);
  if (vol >= target * (double)npts) st->lo = mid;
  else st->hi = mid;
  st->steps += 1;
  if (st->hi - st->lo <= 1e-14 * st->width0 || st->steps >= max_steps) st->done = 1;
}

dim3 egrid(const Geo& g) { return dim3((g.nx + TBX - 1) / TBX, (g.ny + TBY - 1) / TBY, g.nz); }

}  // namespace

int smooth_num_partials(const Geo& g) {
  const dim3 e = egrid(g);
  const long long n = (long long)e.x * e.y * e.z;
  const long long m = 2LL * nblocks(g.nn);
  return (int)(n > m ? n : m);
}

void launch_node_project(const Geo& g, const double* dc, double r, double* ns, hipStream_t st) {
  const int R = (int)ceil(r) + 1;
  const dim3 grid((g.nnx + TBX - 1) / TBX, (g.nny + TBY - 1) / TBY, g.nnz);
  if (g.dim == 2) k_node_project<2><<<grid, dim3(TBX, TBY, 1), 0, st>>>(g, dc, r, R, ns);
  else k_node_project<3><<<grid, dim3(TBX, TBY, 1), 0, st>>>(g, dc, r, R, ns);
}

void launch_smooth_bisect(const Geo& g, const double* ns, double target, int nsub, int max_steps, SmoothDev* sd,
                          double* rho, double* part, hipStream_t st) {
  const int nb = nblocks(g.nn);
  k_minmax<<<nb, VB, 0, st>>>(ns, g.nn, part);
  k_smooth_init<<<1, 64, 0, st>>>(sd, part, nb);
  const dim3 eg = egrid(g);
  const int np = (int)(eg.x * eg.y * eg.z);
  const int npts = g.dim == 3 ? (nsub + 1) * (nsub + 1) * (nsub + 1) : (nsub + 1) * (nsub + 1);
  for (int it = 0; it <= max_steps; ++it) {
    const int fin = it == max_steps;
    if (g.dim == 2)
      k_smooth_rho<2><<<eg, dim3(TBX, TBY, 1), 0, st>>>(g, ns, sd, fin, nsub, fin ? rho : nullptr, part);
    else
      k_smooth_rho<3><<<eg, dim3(TBX, TBY, 1), 0, st>>>(g, ns, sd, fin, nsub, fin ? rho : nullptr, part);
    k_smooth_step<<<1, VB, 0, st>>>(sd, part, np, target, npts, max_steps, fin);
  }
}
