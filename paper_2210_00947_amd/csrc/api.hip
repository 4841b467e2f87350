// Host orchestration of libmgar: handle, MG hierarchy, V-cycle, MGCG, MGAR
// reanalysis, sensitivities and the OC update, behind the C ABI of mgar.h.
//
// Every numerical step runs in the kernels of stencil.hip, vec.hip and
// topopt.hip on the handle's stream. The host only sequences launches and
// reads back a few scalars (stopping flags, the Eq 28 residual, compliance).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mgar.h"
#include "mgar_launch.h"

namespace {

struct LevelBuf {
  Geo g;
  double* k = nullptr;   // element conductivities of the K0 hierarchy on this grid
  double* b = nullptr;   // right-hand side (grids >= 1)
  double* xa = nullptr;  // iterate before the post-smoother
  double* xb = nullptr;  // iterate after the post-smoother (grids >= 1)
};

}  // namespace

// Pinned host image of the CG state and the status word behind it (the same
// layout as on the device), plus a few FP64 scalars read in the same
// synchronisation.
struct HostPin {
  CgState s;
  int status;
  int pad;
  double extra[4];
  OcDev oc;
};
static_assert(offsetof(HostPin, status) == sizeof(CgState), "status word follows the state");

struct mgar_handle {
  mgar_params p;
  hipStream_t s = nullptr;
  int L = 0;
  std::vector<LevelBuf> lv;
  long long N = 0, E = 0;
  double* kcur = nullptr;                 // K(xphys) of the current call, finest grid
  double* rtmp = nullptr;                 // residual scratch (finest size)
  double* Ainv = nullptr;                 // coarsest-grid inverse
  int* dstatus = nullptr;                 // device status word (coarsest pivots), right after *st
  HostPin* hpin = nullptr;                // pinned host buffer of the state readbacks
  int status_host = 0;                    // the status word, read with the CG state ...
  bool status_valid = false;              // ... after the main stream waited for the latest build
  double *qm = nullptr, *cx = nullptr, *cr = nullptr, *cz = nullptr, *cp = nullptr, *cw = nullptr;
  double* cp2 = nullptr;                  // second CG direction buffer (fused direction update)
  double* dg0 = nullptr;                  // diagonal of K0 on the finest grid (3D, FP64 hierarchy)
  bool dg0_valid = false;
  double *pa = nullptr, *pb = nullptr, *pc = nullptr;  // partial-sum buffers
  long long part_cap = 0;
  double* scal = nullptr;                 // device scalars
  CgState* st = nullptr;
  MgarDev* md = nullptr;
  OcDev* oc = nullptr;
  double oc_hint = 0.0;                   // multiplier of the last OC update (first candidates of the next)
  double *R = nullptr, *Wm = nullptr;     // basis block and K times basis, N x m
  double *invHs = nullptr, *wvol = nullptr, *gtmp = nullptr;
  int* tap_off = nullptr;
  double* tap_w = nullptr;
  int ntap = 0;
  int tap_cap = 0;                        // taps the device table holds
  int tap_hr = 0;                         // largest |offset| of a filter tap
  double filter_r = 0.0;                  // radius of the current filter
  SmoothDev* sdev = nullptr;              // boundary-smoothing bisection state (allocated on first use)
  double* spart = nullptr;                // its partial sums
  long long spart_cap = 0;
  int pcg_hint = 0;                       // iterations of the last FP64 PCG solve
  bool timing = true;                     // per-solve device time (stats->ms; one host sync)
  double rate32 = -1.0;                   // last observed contraction per FP32 PCG iteration
  bool has_k0 = false;
  int lt = 1;                             // first grid handled by the V-cycle tail kernel
  TailSpec tail;
  // mixed precision: FP32 multigrid and inner PCG over BF16 densities
  bool mixed = false;
  uint16_t* dens = nullptr;               // BF16 physical densities of the current call
  uint16_t* dens0 = nullptr;              // BF16 densities of K0 (finest grid of the FP32 hierarchy)
  std::vector<float*> kf, bf, xaf, xbf;   // FP32 hierarchy: cells (grids >= 1) and vectors
  float *rtmpf = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *w32 = nullptr,
        *d32 = nullptr;
  float* k32 = nullptr;                   // FP32 conductivities of the current call (inner operator)
  float* p32b = nullptr;                  // second inner direction buffer (fused direction update)
  float* dg32 = nullptr;                  // diagonal of the BF16 finest operator (3D)
  bool dg32_valid = false;
  int ltf = 1;
  TailSpec tailf;
  float kmin_f = 0.f, kdiff_f = 0.f;
  int refine_max = 40;
  // launch shape of every stencil: [class: 0 FP64, 1 FP32][grid level][mode]
  std::vector<std::array<StencilCfg, 7>> scfg[2];
  // Captured PCG iterations (class 0: FP64 pcg, 1: FP32 inner pcg32): graphs
  // of 1, 2, 4 and 8 iterations for the (tol, cg_max) they were captured
  // with, replayed on the handle's own stream `gs` (a graph cannot be
  // captured on the legacy default stream) ordered after and before `s`.
  bool use_graphs = false;               // replay captured iterations (eager launches measured faster)
  hipStream_t gs = nullptr;
  hipEvent_t gin = nullptr, gout = nullptr;
  hipGraph_t gg[2][4] = {};
  hipGraphExec_t gx[2][4] = {};
  double g_tol[2] = {-1.0, -1.0};
  int g_max[2] = {-1, -1};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // the coarsest inverse is built on a side stream, overlapping the solver's
  // set-up; the main stream waits for it before the first use of Ainv
  hipStream_t cs = nullptr;
  hipEvent_t cev0 = nullptr, cev1 = nullptr;
  bool coarse_pending = false;
  // kernel timing (instrumentation)
  unsigned prof_mask = 0;
  int tag_base = 0;                       // CG iteration of the next eager iteration (timing tags)
  std::vector<hipEvent_t> prof_ev;        // pool, pairs
  std::vector<double> prof_bytes;         // bytes of each recorded pair
  std::vector<int> prof_tag;              // CG iteration of each pair (-1: not in a CG loop)
  size_t prof_used = 0;
  long long prof_launches = 0;
  double prof_ms = 0.0, prof_total_bytes = 0.0;
};

namespace {

#define HIPCK(x)                                  \
  do {                                            \
    hipError_t err_ = (x);                        \
    if (err_ != hipSuccess) return MGAR_E_HIP;    \
  } while (0)

#define LAUNCHCK() HIPCK(hipGetLastError())

Geo make_geo(const mgar_params& p, int l) {
  Geo g;
  std::memset(&g, 0, sizeof(g));
  const int s = 1 << l;
  g.dim = p.dim;
  g.nx = p.nelx / s;
  g.ny = p.nely / s;
  g.nz = (p.dim == 3) ? p.nelz / s : 1;
  g.nnx = g.nx + 1;
  g.nny = g.ny + 1;
  g.nnz = (p.dim == 3) ? g.nz + 1 : 1;
  auto cdiv = [](int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); };
  auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
  // coarse node I is fixed iff the finest node I*2^l lies in the box
  g.f0x = cdiv(p.fix_lo[0], s); g.f1x = fdiv(p.fix_hi[0], s);
  g.f0y = cdiv(p.fix_lo[1], s); g.f1y = fdiv(p.fix_hi[1], s);
  if (p.dim == 3) { g.f0z = cdiv(p.fix_lo[2], s); g.f1z = fdiv(p.fix_hi[2], s); }
  else { g.f0z = 0; g.f1z = 0; }
  g.h = (double)s;
  g.nn = (long long)g.nnx * g.nny * g.nnz;
  g.ne = (long long)g.nx * g.ny * g.nz;
  return g;
}

long long count_fixed(const Geo& g) {
  auto span = [](int lo, int hi, int n) -> long long {
    const int a = lo < 0 ? 0 : lo, b = hi > n - 1 ? n - 1 : hi;
    return b >= a ? (long long)(b - a + 1) : 0;
  };
  return span(g.f0x, g.f1x, g.nnx) * span(g.f0y, g.f1y, g.nny) * span(g.f0z, g.f1z, g.nnz);
}

template <typename T>
int dalloc(T** p, long long n) {
  if (n <= 0) n = 1;
  HIPCK(hipMalloc((void**)p, sizeof(T) * (size_t)n));
  return MGAR_OK;
}

#define ACK(x)                      \
  do {                              \
    int rc_ = (x);                  \
    if (rc_ != MGAR_OK) return rc_; \
  } while (0)

int validate(const mgar_params* p) {
  if (!p) return MGAR_E_ARG;
  if (p->dim != 2 && p->dim != 3) return MGAR_E_ARG;
  if (p->nelx < 1 || p->nely < 1 || (p->dim == 3 && p->nelz < 1)) return MGAR_E_ARG;
  if (p->levels < 1 || p->levels > 16) return MGAR_E_ARG;
  if (p->n_basis < 1 || p->n_basis > MGAR_MAX_BASIS) return MGAR_E_ARG;
  if (!(p->omega > 0.0) || !(p->filter_r > 0.0) || p->cg_max < 0) return MGAR_E_ARG;
  if (!(p->k0 > 0.0) || !(p->kmin > 0.0) || !(p->penal >= 1.0)) return MGAR_E_ARG;
  if (p->precision != MGAR_PREC_FP64 && p->precision != MGAR_PREC_MIXED) return MGAR_E_PRECISION;
  if (p->precision == MGAR_PREC_MIXED && p->penal != 3.0) return MGAR_E_PRECISION;
  if (p->precision == MGAR_PREC_MIXED && !(p->inner_tol > 0.0 && p->inner_tol < 1.0)) return MGAR_E_ARG;
  if ((int)std::ceil(p->filter_r) > (p->dim == 3 ? MGAR_MAX_FILTER_R3 : MGAR_MAX_FILTER_R2)) return MGAR_E_ARG;
  const int s = 1 << (p->levels - 1);
  if (p->nelx % s || p->nely % s || (p->dim == 3 && p->nelz % s)) return MGAR_E_DIMS;
  return MGAR_OK;
}

// ------------------------------------------------------------------ MG

// Make the main stream wait for a coarsest-inverse build still running on the
// side stream (no-op otherwise).
int sync_coarse(mgar_handle* h) {
  if (!h->coarse_pending) return MGAR_OK;
  h->coarse_pending = false;
  HIPCK(hipStreamWaitEvent(h->s, h->cev1, 0));
  return MGAR_OK;
}

// The single-workgroup build of the coarsest inverse runs on a side stream
// (default priority) beside the solver's work on the main stream, after what
// the main stream has enqueued so far; sync_coarse makes the main stream wait
// for it before its first reader.
int coarse_side_begin(mgar_handle* h) {
  if (!h->cs) {
    HIPCK(hipStreamCreateWithFlags(&h->cs, hipStreamNonBlocking));
    HIPCK(hipEventCreateWithFlags(&h->cev0, hipEventDisableTiming));
    HIPCK(hipEventCreateWithFlags(&h->cev1, hipEventDisableTiming));
  }
  HIPCK(hipEventRecord(h->cev0, h->s));
  HIPCK(hipStreamWaitEvent(h->cs, h->cev0, 0));
  HIPCK(hipMemsetAsync(h->dstatus, 0, sizeof(int), h->cs));
  return MGAR_OK;
}

int coarse_side_end(mgar_handle* h) {
  HIPCK(hipEventRecord(h->cev1, h->cs));
  h->coarse_pending = true;
  h->status_valid = false;
  LAUNCHCK();
  return MGAR_OK;
}

// The CG state to the host through the pinned buffer (one synchronisation),
// with the coarsest-build status word behind it when the main stream has
// already waited for the latest build (check_coarse then needs no copy of its
// own), and optionally n (<= 4) FP64 scalars from dev_extra.
int read_cg_state(mgar_handle* h, CgState* hs, const double* dev_extra = nullptr, int n = 0,
                  double* extra = nullptr) {
  const bool with_status = !h->coarse_pending;
  if (n > 0)
    HIPCK(hipMemcpyAsync(h->hpin->extra, dev_extra, sizeof(double) * n, hipMemcpyDeviceToHost, h->s));
  HIPCK(hipMemcpyAsync(h->hpin, h->st, sizeof(CgState) + (with_status ? sizeof(int) : 0),
                       hipMemcpyDeviceToHost, h->s));
  HIPCK(hipStreamSynchronize(h->s));
  *hs = h->hpin->s;
  for (int i = 0; i < n; ++i) extra[i] = h->hpin->extra[i];
  if (with_status) {
    h->status_host = h->hpin->status;
    h->status_valid = true;
  }
  return MGAR_OK;
}

int build_hierarchy(mgar_handle* h) {
  ACK(sync_coarse(h));   // Ainv and dstatus are rewritten below
  if (h->dg0) launch_diag(h->lv[0].g, h->lv[0].k, h->dg0, h->s);
  h->dg0_valid = h->dg0 != nullptr;
  for (int l = 1; l < h->L; ++l) launch_coarsen(h->lv[l - 1].g, h->lv[l].g, h->lv[l - 1].k, h->lv[l].k, h->s);
  ACK(coarse_side_begin(h));
  launch_coarse_build(h->lv[h->L - 1].g, h->lv[h->L - 1].k, h->Ainv, h->dstatus, h->cs);
  ACK(coarse_side_end(h));
  return MGAR_OK;
}

// Algorithmic bytes of one stencil launch (each operand read once, result written once).
double stencil_bytes(const Geo& g, int mode) {
  const double N = (double)g.nn, E = (double)g.ne;
  switch (mode) {
    case SM_APPLY: case SM_APPLY_DOT: return 8.0 * (2 * N + E);
    case SM_RESID: case SM_JACOBI: case SM_JACOBI_DOT: return 8.0 * (3 * N + E);
    case SM_JACOBI0: return 8.0 * (2 * N + E);
    case SM_NEG_DK: return 8.0 * (2 * N + 2 * E);
    case SM_PAPPLY_DOT: return 8.0 * (4 * N + E);   // z, p_old, cells in; p, K p out
  }
  return 0.0;
}

// Block partials written by a dot-producing stencil mode on the finest grid.
int nparts_at(const mgar_handle* h, int cls, int mode) {
  return stencil_num_partials(h->lv[0].g, &h->scfg[cls][0][mode]);
}

// Stencil launch on grid `level`; finest-grid launches selected by the
// profiling mask are bracketed by HIP events on the same stream.
int stencil_at(mgar_handle* h, int level, int mode, const double* x, const double* k,
               const double* kref, const double* b, double* out, double omega, double* part,
               const int* done, int* nparts = nullptr, int tag = -1, unsigned* cnt = nullptr,
               double* rout = nullptr) {
  const Geo& g = h->lv[level].g;
  const bool timed = level == 0 && (h->prof_mask >> mode) & 1u;
  if (timed && h->prof_used + 2 > h->prof_ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      HIPCK(hipEventCreate(&e));
      h->prof_ev.push_back(e);
    }
  }
  int np;
  const StencilCfg* cfg = &h->scfg[0][level][mode];
  if (timed && stencil_records_events(g, cfg)) {
    // events recorded by the launch itself at kernel start and end
    np = launch_stencil(g, mode, x, k, kref, b, out, omega, part, done, h->s, cnt, rout,
                        h->prof_ev[h->prof_used], h->prof_ev[h->prof_used + 1], cfg);
  } else {
    if (timed) HIPCK(hipEventRecord(h->prof_ev[h->prof_used], h->s));
    np = launch_stencil(g, mode, x, k, kref, b, out, omega, part, done, h->s, cnt, rout, nullptr,
                        nullptr, cfg);
    if (timed) HIPCK(hipEventRecord(h->prof_ev[h->prof_used + 1], h->s));
  }
  if (nparts) *nparts = np;
  if (timed) {
    h->prof_bytes.push_back(stencil_bytes(g, mode));
    h->prof_tag.push_back(tag);
    h->prof_used += 2;
  }
  LAUNCHCK();
  return MGAR_OK;
}

// Fused direction update + apply + dot on the finest grid with the shape tuned
// for SM_APPLY_DOT: w = K p into cw, partials into pc. *nparts = -1 (nothing
// launched) when that shape cannot run it. Timed like stencil_at under the
// SM_APPLY_DOT profiling bit, with the fused kernel's bytes.
int papply_at(mgar_handle* h, const double* z, const PFuse& pf, const int* done, int* nparts, int tag) {
  const Geo& g = h->lv[0].g;
  const StencilCfg* cfg = &h->scfg[0][0][SM_APPLY_DOT];
  if (!papply_supported(g, cfg)) {
    *nparts = -1;
    return MGAR_OK;
  }
  const bool timed = (h->prof_mask >> SM_APPLY_DOT) & 1u;
  if (timed && h->prof_used + 2 > h->prof_ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      HIPCK(hipEventCreate(&e));
      h->prof_ev.push_back(e);
    }
  }
  *nparts = launch_papply_dot(g, z, h->kcur, h->cw, h->pc, done, h->s, pf, cfg,
                              timed ? h->prof_ev[h->prof_used] : nullptr,
                              timed ? h->prof_ev[h->prof_used + 1] : nullptr);
  if (timed) {
    h->prof_bytes.push_back(stencil_bytes(g, SM_PAPPLY_DOT));
    h->prof_tag.push_back(tag);
    h->prof_used += 2;
  }
  LAUNCHCK();
  return MGAR_OK;
}

// Accumulate the recorded event pairs (the stream must be idle). Pairs tagged
// with a CG iteration at or beyond `cutoff` belong to iterations that were
// enqueued after the stopping test fired; their kernels returned at once, so
// they are dropped.
int profile_harvest(mgar_handle* h, int cutoff = 1 << 30) {
  if (h->prof_used == 0) return MGAR_OK;
  HIPCK(hipEventSynchronize(h->prof_ev[h->prof_used - 1]));
  for (size_t i = 0; i + 1 < h->prof_used; i += 2) {
    if (h->prof_tag[i / 2] >= cutoff) continue;
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, h->prof_ev[i], h->prof_ev[i + 1]));
    h->prof_ms += ms;
    h->prof_total_bytes += h->prof_bytes[i / 2];
    h->prof_launches += 1;
  }
  h->prof_used = 0;
  h->prof_bytes.clear();
  h->prof_tag.clear();
  return MGAR_OK;
}

// One V-cycle (Table 1) on the K0 hierarchy: out = MG(K0, b0, x0). With
// dot_part set, the finest post-smoother also writes partials of b0 . out.
// Whether vcycle() from a zero guess starts with the fused first sweep +
// residual on the finest grid (and can take a fused stopping test).
bool j0resid_fusable(const mgar_handle* h) {
  const StencilCfg& c = h->scfg[0][0][SM_RESID];
  return h->L > 1 && h->lt > 0 && h->dg0_valid && !((h->prof_mask >> SM_RESID) & 1u) && c.kind == 2 &&
         stencil_cfg_valid(h->lv[0].g, c);
}

// check (optional): the previous CG iteration's stopping test, fused into the
// first finest-grid kernel; the caller has checked j0resid_fusable().
int vcycle(mgar_handle* h, const double* b0, const double* x0, double* out, double* dot_part,
           const int* done, int tag = -1, unsigned* dcnt = nullptr, double* dout = nullptr,
           const PFuse* check = nullptr) {
  const int L = h->L;
  const double w = h->p.omega;
  if (L == 1) {
    ACK(sync_coarse(h));   // the coarsest inverse may still be built on the side stream
    launch_coarse_solve(h->lv[0].g, h->Ainv, b0, out, done, h->s);
    if (dot_part) launch_dot(b0, out, h->N, dot_part, done, h->s, dcnt, dout);
    LAUNCHCK();
    return MGAR_OK;
  }
  const int lt = h->lt;   // grids lt..L-1 run inside one workgroup
  bool presmoothed = false;   // grid l's sweep from zero was fused into the restriction onto it
  for (int l = 0; l < lt; ++l) {
    LevelBuf& v = h->lv[l];
    const double* b = (l == 0) ? b0 : v.b;
    // finest grid from zero: first sweep and residual in one launch where the
    // residual's shape allows it
    const bool fused = l == 0 && !x0 && h->dg0_valid && !((h->prof_mask >> SM_RESID) & 1u) &&
                       launch_j0resid(v.g, b, v.k, h->dg0, v.xa, h->rtmp, w, done, h->s,
                                      &h->scfg[0][0][SM_RESID], check);
    if (l == 0 && x0) ACK(stencil_at(h, l, SM_JACOBI, x0, v.k, nullptr, b, v.xa, w, nullptr, done, nullptr, tag));
    else if (!presmoothed && !fused)
      ACK(stencil_at(h, l, SM_JACOBI0, nullptr, v.k, nullptr, b, v.xa, w, nullptr, done, nullptr, tag));
    if (!fused) ACK(stencil_at(h, l, SM_RESID, v.xa, v.k, nullptr, b, h->rtmp, w, nullptr, done, nullptr, tag));
    LevelBuf& c = h->lv[l + 1];
    presmoothed = l + 1 < lt && launch_restrict_j0_t<double, CellD>(v.g, c.g, h->rtmp, CellD{c.k}, c.b, c.xa,
                                                                        w, done, h->s);
    if (!presmoothed) launch_restrict(v.g, c.g, h->rtmp, c.b, done, h->s);
  }
  ACK(sync_coarse(h));   // first reader of the coarsest inverse
  launch_vtail(h->tail, h->lv[lt].b, h->lv[lt].xb, h->Ainv, w, done, h->s);
  const double* xfin = h->lv[lt].xb;
  for (int l = lt - 1; l >= 0; --l) {
    LevelBuf& v = h->lv[l];
    const double* b = (l == 0) ? b0 : v.b;
    double* o = (l == 0) ? out : v.xb;
    double* dp = (l == 0) ? dot_part : nullptr;
    // small grids (node-parallel shape): interpolation and sweep in one launch
    const bool fused = l > 0 && h->scfg[0][l][SM_JACOBI].kind == 0 &&
                       launch_prolong_jacobi_t<double, CellD>(v.g, h->lv[l + 1].g, xfin, v.xa, CellD{v.k}, b,
                                                              o, w, done, h->s);
    if (!fused) {
      launch_prolong(v.g, h->lv[l + 1].g, xfin, v.xa, done, h->s);
      ACK(stencil_at(h, l, dp ? SM_JACOBI_DOT : SM_JACOBI, v.xa, v.k, nullptr, b, o, w, dp, done,
                     nullptr, tag, dp ? dcnt : nullptr, dp ? dout : nullptr));
    }
    xfin = o;
  }
  LAUNCHCK();
  return MGAR_OK;
}

// ---------------------------------------------------------------- mixed precision
// FP32 stencil on grid `level` of the BF16/FP32 hierarchy: the finest grid reads
// BF16 densities (SIMP applied on load), coarser grids FP32 cell conductivities.
// kop (finest grid only): FP32 cell conductivities to use instead of densities.
int stencil32(mgar_handle* h, int level, int mode, const float* x, const float* b, float* out,
              double* part, const int* done, const uint16_t* dens = nullptr,
              const uint16_t* densref = nullptr, const float* kop = nullptr) {
  const Geo& g = h->lv[level].g;
  if (level == 0 && kop) {
    const CellF k{kop};
    launch_stencil_t<float, CellF>(g, mode, x, k, k, b, out, h->p.omega, part, done, h->s, nullptr,
                                   nullptr, nullptr, nullptr, &h->scfg[1][level][mode]);
  } else if (level == 0) {
    const CellB k{dens ? dens : h->dens0, h->kmin_f, h->kdiff_f};
    const CellB kr{densref ? densref : h->dens0, h->kmin_f, h->kdiff_f};
    launch_stencil_t<float, CellB>(g, mode, x, k, kr, b, out, h->p.omega, part, done, h->s, nullptr,
                                   nullptr, nullptr, nullptr, &h->scfg[1][level][mode]);
  } else {
    const CellF k{h->kf[level]};
    launch_stencil_t<float, CellF>(g, mode, x, k, k, b, out, h->p.omega, part, done, h->s, nullptr,
                                   nullptr, nullptr, nullptr, &h->scfg[1][level][mode]);
  }
  LAUNCHCK();
  return MGAR_OK;
}

// K0 := K(BF16 densities of `dens`): cell means of every coarser grid in FP32
// and the coarsest inverse in FP64.
int build_hierarchy32(mgar_handle* h) {
  ACK(sync_coarse(h));
  const int L = h->L;
  h->dg0_valid = false;   // lv[0].k no longer describes the preconditioner's K0
  launch_copy_u16(h->dens, h->dens0, h->E, h->s);
  const CellB k0{h->dens0, h->kmin_f, h->kdiff_f};
  if (h->dg32) launch_diag_t<float, CellB>(h->lv[0].g, k0, h->dg32, h->s);
  h->dg32_valid = h->dg32 != nullptr;
  if (L >= 2) launch_coarsen_t<CellB, float>(h->lv[0].g, h->lv[1].g, k0, h->kf[1], h->s);
  for (int l = 2; l < L; ++l)
    launch_coarsen_t<CellF, float>(h->lv[l - 1].g, h->lv[l].g, CellF{h->kf[l - 1]}, h->kf[l], h->s);
  ACK(coarse_side_begin(h));
  if (L == 1) launch_coarse_build_t<CellB>(h->lv[0].g, k0, h->Ainv, h->dstatus, h->cs);
  else launch_coarse_build_t<CellF>(h->lv[L - 1].g, CellF{h->kf[L - 1]}, h->Ainv, h->dstatus, h->cs);
  ACK(coarse_side_end(h));
  return MGAR_OK;
}

// One FP32 V-cycle on the BF16/FP32 K0 hierarchy (same sequence as vcycle()).
int vcycle32(mgar_handle* h, const float* b0, const float* x0, float* out, double* dot_part,
             const int* done) {
  const int L = h->L;
  if (L == 1) {
    ACK(sync_coarse(h));   // the coarsest inverse may still be built on the side stream
    launch_coarse_solve_t<float>(h->lv[0].g, h->Ainv, b0, out, done, h->s);
    if (dot_part) launch_dot_t<float, float>(b0, out, h->N, dot_part, done, h->s);
    LAUNCHCK();
    return MGAR_OK;
  }
  const int lt = h->ltf;
  bool presmoothed = false;
  for (int l = 0; l < lt; ++l) {
    const float* b = (l == 0) ? b0 : h->bf[l];
    const bool fused = l == 0 && !x0 && h->dg32_valid &&
                       launch_j0resid_t<float, CellB>(h->lv[0].g, b, CellB{h->dens0, h->kmin_f, h->kdiff_f},
                                                      h->dg32, h->xaf[0], h->rtmpf, h->p.omega, done, h->s,
                                                      &h->scfg[1][0][SM_RESID]);
    if (l == 0 && x0) ACK(stencil32(h, l, SM_JACOBI, x0, b, h->xaf[l], nullptr, done));
    else if (!presmoothed && !fused) ACK(stencil32(h, l, SM_JACOBI0, nullptr, b, h->xaf[l], nullptr, done));
    if (!fused) ACK(stencil32(h, l, SM_RESID, h->xaf[l], b, h->rtmpf, nullptr, done));
    presmoothed = l + 1 < lt && launch_restrict_j0_t<float, CellF>(h->lv[l].g, h->lv[l + 1].g, h->rtmpf,
                                                                   CellF{h->kf[l + 1]}, h->bf[l + 1],
                                                                   h->xaf[l + 1], h->p.omega, done, h->s);
    if (!presmoothed) launch_restrict_t<float>(h->lv[l].g, h->lv[l + 1].g, h->rtmpf, h->bf[l + 1], done, h->s);
  }
  ACK(sync_coarse(h));   // first reader of the coarsest inverse
  launch_vtail_t<float>(h->tailf, h->bf[lt], h->xbf[lt], h->Ainv, h->p.omega, done, h->s);
  const float* xfin = h->xbf[lt];
  for (int l = lt - 1; l >= 0; --l) {
    const float* b = (l == 0) ? b0 : h->bf[l];
    float* o = (l == 0) ? out : h->xbf[l];
    double* dp = (l == 0) ? dot_part : nullptr;
    const bool fused = l > 0 && h->scfg[1][l][SM_JACOBI].kind == 0 &&
                       launch_prolong_jacobi_t<float, CellF>(h->lv[l].g, h->lv[l + 1].g, xfin, h->xaf[l],
                                                             CellF{h->kf[l]}, b, o, h->p.omega, done, h->s);
    if (!fused) {
      launch_prolong_t<float>(h->lv[l].g, h->lv[l + 1].g, xfin, h->xaf[l], done, h->s);
      ACK(stencil32(h, l, dp ? SM_JACOBI_DOT : SM_JACOBI, h->xaf[l], b, o, dp, done));
    }
    xfin = o;
  }
  LAUNCHCK();
  return MGAR_OK;
}

// One PCG iteration of class 0 (FP64: K(kcur), V-cycle on the K0 hierarchy)
// or class 1 (FP32 inner solve of the mixed form). No host-side iteration
// index: the kernels read and advance st->it. tag: CG iteration for the
// profiler (eager launches only).
// One PCG iteration; with check_prev it first applies the stopping test of
// the previous iteration (fused into its first kernel where possible). The
// caller applies the test of the last enqueued iteration (launch_cg_check).
int enqueue_iter(mgar_handle* h, int cls, double tol, int cg_max, int nr, int tag, bool check_prev) {
  const long long N = h->N;
  const int* done = &h->st->done;
  const bool fchk = check_prev && cls == 0 && j0resid_fusable(h);
  if (check_prev && !fchk) launch_cg_check(h->st, h->pa, nr, tol, cg_max, h->s);
  if (cls == 0) {
    PFuse chk{};
    chk.st = h->st;
    chk.rzp = h->pa;
    chk.nrz = nr;
    chk.tol = tol;
    chk.cg_max = cg_max;
    ACK(vcycle(h, h->cr, nullptr, h->cz, h->pb, done, tag, nullptr, nullptr, fchk ? &chk : nullptr));
    const int nz = (h->L == 1) ? vec_num_blocks(N) : nparts_at(h, 0, SM_JACOBI_DOT);
    // direction update fused into the apply where the shape allows it (p in
    // cp / cp2 by iteration parity), else two launches on cp
    const PFuse pf{h->st, h->pb, nz, 0, {h->cp, h->cp2}};
    int nw = 0;
    ACK(papply_at(h, h->cz, pf, done, &nw, tag));
    if (nw < 0) {
      launch_p_update(h->cz, h->cp, N, h->st, h->s, h->pb, nz);
      ACK(stencil_at(h, 0, SM_APPLY_DOT, h->cp, h->kcur, nullptr, nullptr, h->cw, 0.0, h->pc, done, &nw, tag));
      launch_cg_update(h->cx, h->cr, h->cp, h->cw, N, h->st, h->pa, nullptr, tol, cg_max, h->s, h->pc, nw);
    } else {
      launch_cg_update(h->cx, h->cr, h->cp, h->cw, N, h->st, h->pa, nullptr, tol, cg_max, h->s, h->pc, nw,
                       h->cp2);
    }
  } else {
    ACK(vcycle32(h, h->r32, nullptr, h->z32, h->pb, done));
    const int nz = (h->L == 1) ? vec_num_blocks(N) : nparts_at(h, 1, SM_JACOBI_DOT);
    // the inner operator: FP32 conductivities of the current densities (BF16
    // densities only enter the V-cycle preconditioner); direction update fused
    // into it where the shape allows (p in p32 / p32b by iteration parity)
    const PFuse pf{h->st, h->pb, nz, 0, {h->p32, h->p32b}, nullptr, nullptr};
    const int nw = launch_papply_dot_t<float, CellF>(h->lv[0].g, h->z32, CellF{h->k32}, h->w32, h->pc, done,
                                                     h->s, pf, &h->scfg[1][0][SM_APPLY_DOT]);
    if (nw < 0) {
      launch_p_update_t<float>(h->z32, h->p32, N, h->st, h->s, h->pb, nz);
      ACK(stencil32(h, 0, SM_APPLY_DOT, h->p32, nullptr, h->w32, h->pc, done, nullptr, nullptr, h->k32));
      launch_cg_update_t<float>(h->d32, h->r32, h->p32, h->w32, N, h->st, h->pa, nullptr, tol, cg_max, h->s,
                                h->pc, nparts_at(h, 1, SM_APPLY_DOT));
    } else {
      LAUNCHCK();
      launch_cg_update_t<float>(h->d32, h->r32, h->p32, h->w32, N, h->st, h->pa, nullptr, tol, cg_max, h->s,
                                h->pc, nw, h->p32b);
    }
  }
  LAUNCHCK();
  return MGAR_OK;
}

void drop_graphs(mgar_handle* h) {
  for (int c = 0; c < 2; ++c) {
    for (int k = 0; k < 4; ++k) {
      if (h->gx[c][k]) (void)hipGraphExecDestroy(h->gx[c][k]);
      if (h->gg[c][k]) (void)hipGraphDestroy(h->gg[c][k]);
      h->gx[c][k] = nullptr;
      h->gg[c][k] = nullptr;
    }
    h->g_tol[c] = -1.0;
    h->g_max[c] = -1;
  }
}

// Capture graphs of 1, 2, 4 and 8 iterations of class cls on the handle's
// own stream (the launch helpers enqueue on h->s, so it is swapped meanwhile).
int capture_iters(mgar_handle* h, int cls, double tol, int cg_max, int nr) {
  ACK(sync_coarse(h));   // no cross-stream wait inside a capture
  for (int k = 0; k < 4; ++k) {
    if (h->gx[cls][k]) (void)hipGraphExecDestroy(h->gx[cls][k]);
    if (h->gg[cls][k]) (void)hipGraphDestroy(h->gg[cls][k]);
    h->gx[cls][k] = nullptr;
    h->gg[cls][k] = nullptr;
  }
  if (!h->gs) {
    HIPCK(hipStreamCreateWithFlags(&h->gs, hipStreamNonBlocking));
    HIPCK(hipEventCreateWithFlags(&h->gin, hipEventDisableTiming));
    HIPCK(hipEventCreateWithFlags(&h->gout, hipEventDisableTiming));
  }
  hipStream_t user = h->s;
  for (int k = 0; k < 4; ++k) {
    HIPCK(hipStreamBeginCapture(h->gs, hipStreamCaptureModeThreadLocal));
    h->s = h->gs;
    int rc = MGAR_OK;
    for (int i = 0; i < (1 << k) && rc == MGAR_OK; ++i) rc = enqueue_iter(h, cls, tol, cg_max, nr, -1, i > 0);
    if (rc == MGAR_OK) launch_cg_check(h->st, h->pa, nr, tol, cg_max, h->s);
    h->s = user;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->gs, &g);
    if (rc != MGAR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    HIPCK(e);
    h->gg[cls][k] = g;
    HIPCK(hipGraphInstantiate(&h->gx[cls][k], g, nullptr, nullptr, 0));
  }
  h->g_tol[cls] = tol;
  h->g_max[cls] = cg_max;
  return MGAR_OK;
}

// n PCG iterations of class cls: replayed graphs (binary decomposition of n)
// unless graphs are off or kernel timing is on (then eager launches).
int run_iters(mgar_handle* h, int cls, double tol, int cg_max, int n, int nr) {
  if (n <= 0) return MGAR_OK;
  // eager launches wait for a coarsest inverse still being built right before
  // its first reader (the V-cycle tail), so the finest-grid kernels of the
  // first iteration run beside the build
  if (!h->use_graphs || h->prof_mask) {
    for (int i = 0; i < n; ++i) ACK(enqueue_iter(h, cls, tol, cg_max, nr, h->tag_base + i, i > 0));
    launch_cg_check(h->st, h->pa, nr, tol, cg_max, h->s);
    h->tag_base += n;
    return MGAR_OK;
  }
  // replayed graphs run on another stream behind an event of h->s: the wait for
  // a coarsest inverse still being built must be on h->s before that event
  ACK(sync_coarse(h));
  if (!h->gx[cls][0] || h->g_tol[cls] != tol || h->g_max[cls] != cg_max)
    ACK(capture_iters(h, cls, tol, cg_max, nr));
  HIPCK(hipEventRecord(h->gin, h->s));
  HIPCK(hipStreamWaitEvent(h->gs, h->gin, 0));
  for (int k = 3; k >= 0; --k)
    while (n >= (1 << k)) {
      HIPCK(hipGraphLaunch(h->gx[cls][k], h->gs));
      n -= 1 << k;
    }
  HIPCK(hipEventRecord(h->gout, h->gs));
  HIPCK(hipStreamWaitEvent(h->s, h->gout, 0));
  return MGAR_OK;
}

// Enqueue one segment of the FP32 PCG run of the mixed form: n iterations on
// K32 d = r32 from d = 0 (no host synchronisation). fresh starts the Krylov
// recurrences; otherwise they continue from the previous segment, whose
// iterate the caller has folded into the FP64 solution and whose residual it
// has replaced by the FP64 one. The device stops the segment early once
// ||r32|| has dropped by inner_tol sqrt(qscale2) (or at the CG budget); FP64
// accumulation of every inner product.
int enqueue_seg32(mgar_handle* h, bool fresh, double qscale2, int n) {
  const long long N = h->N;
  const double tol_in = h->p.inner_tol;
  HIPCK(hipMemsetAsync(h->d32, 0, sizeof(float) * N, h->s));
  const int nr = launch_dot_t<float, float>(h->r32, h->r32, N, h->pa, nullptr, h->s);
  launch_cg_start(h->st, h->pa, nr, qscale2, fresh, tol_in, h->p.cg_max, h->s);
  if (fresh) launch_fill_t<float>(h->p32b, N, 0.f, 0.f, h->s);   // p_old of iteration 0 (weight 0)
  ACK(run_iters(h, 1, tol_in, h->p.cg_max, n, nr));
  // the update of d of the last iteration may still be pending (fused path)
  if (papply_supported(h->lv[0].g, &h->scfg[1][0][SM_APPLY_DOT]))
    launch_cg_flush_t<float>(h->d32, h->p32, N, h->st, h->s);
  LAUNCHCK();
  return MGAR_OK;
}

// Mixed form: one FP32 PCG run (FP32 operator of the current densities, FP32
// V-cycles over BF16 densities) in segments with FP64 residual replacement.
// A segment runs the number of iterations predicted to reduce the residual
// by inner_tol (the last one: to 0.7 tol ||q||; a segment that would leave
// less than a factor 10 to go becomes the last one); its FP32 correction is
// then added to the FP64 solution x, and r = q - K64 x is computed in FP64,
// with one host synchronisation per segment. The next segment continues the
// same Krylov recurrences from that r as long as it is within twice the
// recursive residual it replaces (else beta = rz_new / rz_old would be
// inflated and the new direction mostly the old one: the run starts afresh
// from r, as plain iterative refinement does). The stopping test
// ||r|| <= tol ||q|| is on the FP64 residual. x in h->cx on entry and exit;
// *nref: segments run.
int solve_mixed(mgar_handle* h, double tol, int* iters, int* conv, double* relres, int* nref) {
  const long long N = h->N;
  const Geo& g = h->lv[0].g;
  const int cg_max = h->p.cg_max;
  launch_cast_f32(h->kcur, h->k32, h->E, h->s);
  const int nq = launch_dot(h->qm, h->qm, N, h->pb, nullptr, h->s);
  launch_finalize(h->pb, nq, &h->scal[2], nullptr, h->s);
  auto fp64_residual = [&]() -> int {
    ACK(stencil_at(h, 0, SM_RESID, h->cx, h->kcur, nullptr, h->qm, h->cr, 0.0, nullptr, nullptr));
    const int nr = launch_dot(h->cr, h->cr, N, h->pa, nullptr, h->s);
    launch_finalize(h->pa, nr, &h->scal[3], nullptr, h->s);
    return MGAR_OK;
  };
  ACK(fp64_residual());
  double qr[2];
  HIPCK(hipMemcpyAsync(qr, &h->scal[2], 2 * sizeof(double), hipMemcpyDeviceToHost, h->s));
  HIPCK(hipStreamSynchronize(h->s));
  int total = 0, seg = 0, it_run = 0;
  double rr_rec = -1.0;
  *conv = 0;
  for (;; ++seg) {
    *relres = qr[0] > 0.0 ? std::sqrt(qr[1] / qr[0]) : 0.0;
    if (*relres <= tol) { *conv = 1; break; }
    if (total >= cg_max || seg >= h->refine_max) break;
    launch_mask_copy_t<double, float>(g, h->cr, h->r32, h->s);
    const double fin = 0.7 * tol / *relres;
    const double tau = fin * 10.0 >= h->p.inner_tol ? fin : h->p.inner_tol;
    const double qs = (tau / h->p.inner_tol) * (tau / h->p.inner_tol);
    const double rate = (h->rate32 > 0.0 && h->rate32 < 0.999) ? h->rate32 : 0.5;
    const int n = std::max(1, std::min({(int)std::ceil(std::log(tau) / std::log(rate)), 32, cg_max - total}));
    const bool fresh = seg == 0 || !(rr_rec > 0.0 && qr[1] <= 4.0 * rr_rec);
    if (fresh) it_run = 0;
    ACK(enqueue_seg32(h, fresh, qs, n));
    launch_add_f32(h->cx, h->d32, N, h->s);
    ACK(fp64_residual());
    CgState hs;
    ACK(read_cg_state(h, &hs, &h->scal[2], 2, qr));
    const int its = hs.it - it_run;
    total += its;
    it_run = hs.it;
    // contraction per iteration of the recursive residual over the segment
    // (its initial ||r32||^2 is st->qq / qs)
    const double r0 = hs.qq / qs;
    if (its > 0 && r0 > 0.0 && hs.rr > 0.0) {
      const double r = std::pow(hs.rr / r0, 0.5 / (double)its);
      if (r > 0.0 && r < 0.999) h->rate32 = r;
    }
    rr_rec = hs.rr;
    LAUNCHCK();
  }
  *iters = total;
  *nref = seg;
  return MGAR_OK;
}

// PCG with one V-cycle as preconditioner on K(kfine); x (h->cx) holds the
// initial guess on entry and the solution on exit; h->qm the masked load.
// nr0 > 0: h->cr already holds r = q - K x with nr0 block partials of ||r||^2
// in h->pa, and ||q||^2 is in md->qq (the reanalysis has formed both).
int pcg(mgar_handle* h, const double* kfine, double tol, int* iters, int* conv, double* relres, int nr0 = 0) {
  const long long N = h->N;
  const int cg_max = h->p.cg_max;
  int nr = nr0;
  if (nr0 > 0) {
    launch_cg_init(h->st, &h->md->qq, 1, h->pa, nr0, tol, cg_max, h->s);
  } else {
    ACK(stencil_at(h, 0, SM_RESID, h->cx, kfine, nullptr, h->qm, h->cr, 0.0, nullptr, nullptr));
    nr = launch_dot(h->cr, h->cr, N, h->pa, nullptr, h->s);
    const int nq = launch_dot(h->qm, h->qm, N, h->pb, nullptr, h->s);
    launch_cg_init(h->st, h->pb, nq, h->pa, nr, tol, cg_max, h->s);
  }
  // the fused direction update reads p_old = cp2 at iteration 0 (weight 0):
  // keep it finite whatever an earlier solve left there
  launch_fill_t<double>(h->cp2, N, 0.f, 0.f, h->s);
  LAUNCHCK();
  (void)kfine;   // the iterations apply K(h->kcur)
  h->tag_base = 0;
  int it = 0;
  // first chunk: a little below the previous solve's count (iteration counts
  // change slowly from one optimisation cycle to the next), else 3
  int chunk = h->pcg_hint > 6 ? h->pcg_hint - 3 : 3;
  double rr_prev = -1.0;
  int it_prev = 0;
  CgState hs;
  for (;;) {
    // Enqueue up to `chunk` iterations. The stopping test runs on the device
    // (before iteration 0 in cg_init, then at the end of every update); once
    // it fires, every later kernel returns immediately, so the iterates are
    // those of a loop that tests before every iteration.
    const int c = std::min(chunk, cg_max - it);
    ACK(run_iters(h, 0, tol, cg_max, c, nr));
    it += c;
    ACK(read_cg_state(h, &hs));
    if (hs.done) break;
    if (it >= cg_max) return MGAR_E_HIP;   // the device test must have fired by now
    // predict the remaining iterations from the observed contraction rate
    const double rr = hs.rr;
    int next = (rr_prev <= 0.0 && h->pcg_hint >= it) ? h->pcg_hint - it + 1 : 4;
    if (rr_prev > 0.0 && rr > 0.0 && it > it_prev) {
      const double rate = std::pow(rr / rr_prev, 0.5 / (double)(it - it_prev));
      const double goal = tol * std::sqrt(hs.qq) / std::sqrt(rr);
      if (rate > 0.0 && rate < 0.999 && goal < 1.0) next = (int)std::ceil(std::log(goal) / std::log(rate));
    }
    if (next < 1) next = 1;
    if (next > 16) next = 16;
    rr_prev = rr;
    it_prev = it;
    chunk = next;
  }
  // the x update of the last iteration may still be pending (fused path)
  if (papply_supported(h->lv[0].g, &h->scfg[0][0][SM_APPLY_DOT]))
    launch_cg_flush_t<double>(h->cx, h->cp, N, h->st, h->s);
  LAUNCHCK();
  ACK(profile_harvest(h, hs.iters));
  h->pcg_hint = hs.iters;
  *iters = hs.iters;
  *conv = hs.converged;
  *relres = (hs.qq > 0.0) ? std::sqrt(hs.rr / hs.qq) : 0.0;
  return MGAR_OK;
}

// Cone filter of radius r (Eq 7-8): the taps (offsets within the radius,
// weight r - distance), 1/Hs and the filtered-volume weights w = H^T (1/Hs),
// which are also dv. The tap table grows on demand (its device copy is
// reallocated only when a larger radius needs more taps than it holds).
int set_filter(mgar_handle* h, double r) {
  const int Rw = (int)std::ceil(r);
  std::vector<int> off;
  std::vector<double> w;
  int hr = 0;
  const int rz = (h->p.dim == 3) ? Rw : 0;
  for (int dz = -rz; dz <= rz; ++dz)
    for (int dy = -Rw; dy <= Rw; ++dy)
      for (int dx = -Rw; dx <= Rw; ++dx) {
        const double d = std::sqrt((double)(dx * dx + dy * dy + dz * dz));
        const double wt = r - d;
        if (wt > 0.0) {
          off.push_back(dx); off.push_back(dy); off.push_back(dz);
          w.push_back(wt);
          hr = std::max({hr, std::abs(dx), std::abs(dy), std::abs(dz)});
        }
      }
  const int n = (int)w.size();
  if (n > h->tap_cap) {
    HIPCK(hipStreamSynchronize(h->s));   // earlier filter launches may still read the old table
    if (h->tap_off) HIPCK(hipFree(h->tap_off));
    if (h->tap_w) HIPCK(hipFree(h->tap_w));
    h->tap_off = nullptr;
    h->tap_w = nullptr;
    h->tap_cap = 0;
    ACK(dalloc(&h->tap_off, 3LL * n));
    ACK(dalloc(&h->tap_w, (long long)n));
    h->tap_cap = n;
  }
  // stream-ordered upload: the launches that read the table follow on h->s
  HIPCK(hipMemcpyAsync(h->tap_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, h->s));
  HIPCK(hipMemcpyAsync(h->tap_w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, h->s));
  h->ntap = n;
  h->tap_hr = hr;
  h->filter_r = r;
  const Geo& g0 = h->lv[0].g;
  launch_filter_hs(g0, h->tap_off, h->tap_w, h->ntap, h->invHs, h->s);
  launch_filter_fwd(g0, h->tap_off, h->tap_w, h->ntap, h->tap_hr, h->invHs, nullptr, h->wvol, h->s);
  LAUNCHCK();
  // the host vectors are released on return: the copies must have left them
  HIPCK(hipStreamSynchronize(h->s));
  return MGAR_OK;
}

int check_coarse(mgar_handle* h) {
  if (h->status_valid && !h->coarse_pending) {   // read with the solver's last CG state
    h->status_valid = false;
    return h->status_host ? MGAR_E_NOT_SPD : MGAR_OK;
  }
  ACK(sync_coarse(h));
  int st = 0;
  HIPCK(hipMemcpyAsync(&st, h->dstatus, sizeof(int), hipMemcpyDeviceToHost, h->s));
  HIPCK(hipStreamSynchronize(h->s));
  return st ? MGAR_E_NOT_SPD : MGAR_OK;
}

void stats_init(mgar_stats* st) {
  if (!st) return;
  std::memset(st, 0, sizeof(*st));
  st->res_ca = std::nan("");
  st->res_final = std::nan("");
}

int finish_timing(mgar_handle* h, mgar_stats* st) {
  if (!h->timing) {
    if (st) st->ms = -1.f;
    return MGAR_OK;
  }
  HIPCK(hipEventRecord(h->e1, h->s));
  HIPCK(hipEventSynchronize(h->e1));
  if (st) {
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, h->e0, h->e1));
    st->ms = ms;
  }
  return MGAR_OK;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

void mgar_default_params(mgar_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dim = 2;
  p->levels = 1;
  p->fix_lo[0] = p->fix_lo[1] = p->fix_lo[2] = 0;
  p->fix_hi[0] = p->fix_hi[1] = p->fix_hi[2] = -1;
  p->k0 = 1.0;
  p->kmin = 1e-3;
  p->penal = 3.0;
  p->omega = 0.8;
  p->n_basis = 2;
  p->eps_accept = 1e-8;
  p->cg_max = 200;
  p->basis_x0_zero = 0;
  p->precision = MGAR_PREC_FP64;
  p->filter_r = 1.5;
  p->inner_tol = 1e-3;
}

const char* mgar_strerror(int code) {
  switch (code) {
    case MGAR_OK: return "ok";
    case MGAR_W_NOT_CONVERGED: return "warning: cg_max reached before the tolerance";
    case MGAR_E_ARG: return "bad argument or null pointer";
    case MGAR_E_DIMS: return "elements per axis not a multiple of 2^(levels-1), or coarsest grid above 1024 nodes";
    case MGAR_E_SINGULAR: return "coarsest grid has no Dirichlet node";
    case MGAR_E_HIP: return "HIP runtime error";
    case MGAR_E_NOT_SPD: return "non-positive pivot in the reduced or coarsest system";
    case MGAR_E_PRECISION: return "unsupported precision mode";
    case MGAR_E_STATE: return "reanalysis needs a factorised K0: run mgcg_solve first";
    default: return "unknown error";
  }
}

void mgar_destroy(mgar_handle* h) {
  if (!h) return;
  if (h->cs) (void)hipStreamSynchronize(h->cs);
  for (auto& v : h->lv) {
    if (v.k) (void)hipFree(v.k);
    if (v.b) (void)hipFree(v.b);
    if (v.xa) (void)hipFree(v.xa);
    if (v.xb) (void)hipFree(v.xb);
  }
  void* ptrs[] = {h->kcur, h->rtmp, h->Ainv, h->qm, h->cx, h->cr, h->cz, h->cp, h->cp2, h->dg0,
                  h->cw, h->pa, h->pb, h->pc, h->scal, h->st, h->md, h->oc, h->R, h->Wm,
                  h->invHs, h->wvol, h->gtmp, h->tap_off, h->tap_w, h->sdev, h->spart};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (h->hpin) (void)hipHostFree(h->hpin);
  for (auto* v : {&h->kf, &h->bf, &h->xaf, &h->xbf})
    for (float* q : *v)
      if (q) (void)hipFree(q);
  void* mptrs[] = {h->dens, h->dens0, h->rtmpf, h->r32, h->z32, h->p32, h->w32, h->d32, h->k32, h->p32b,
                   h->dg32};
  for (void* q : mptrs)
    if (q) (void)hipFree(q);
  for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
  drop_graphs(h);
  if (h->gin) (void)hipEventDestroy(h->gin);
  if (h->gout) (void)hipEventDestroy(h->gout);
  if (h->gs) (void)hipStreamDestroy(h->gs);
  if (h->e0) (void)hipEventDestroy(h->e0);
  if (h->e1) (void)hipEventDestroy(h->e1);
  if (h->cev0) (void)hipEventDestroy(h->cev0);
  if (h->cev1) (void)hipEventDestroy(h->cev1);
  if (h->cs) (void)hipStreamDestroy(h->cs);
  delete h;
}

static int setup_impl(const mgar_params* p, void* stream, mgar_handle** out) {
  ACK(validate(p));
  mgar_handle* h = new mgar_handle();
  *out = h;
  h->p = *p;
  if (p->dim == 2) { h->p.nelz = 0; h->p.fix_lo[2] = 0; h->p.fix_hi[2] = 0; }
  h->s = (hipStream_t)stream;
  h->L = p->levels;
  h->lv.resize(h->L);
  for (int l = 0; l < h->L; ++l) h->lv[l].g = make_geo(h->p, l);
  for (int c = 0; c < 2; ++c) {
    h->scfg[c].resize(h->L);
    for (int l = 0; l < h->L; ++l) h->scfg[c][l].fill(stencil_default_cfg(h->lv[l].g));
  }
  const Geo& g0 = h->lv[0].g;
  const Geo& gc = h->lv[h->L - 1].g;
  if (gc.nn > 1024) return MGAR_E_DIMS;
  if (count_fixed(gc) == 0) return MGAR_E_SINGULAR;
  h->N = g0.nn;
  h->E = g0.ne;
  for (int l = 0; l < h->L; ++l) {
    LevelBuf& v = h->lv[l];
    ACK(dalloc(&v.k, v.g.ne));
    ACK(dalloc(&v.xa, v.g.nn));
    if (l > 0) {
      ACK(dalloc(&v.b, v.g.nn));
      ACK(dalloc(&v.xb, v.g.nn));
    }
  }
  const long long N = h->N, E = h->E;
  ACK(dalloc(&h->kcur, E));
  ACK(dalloc(&h->rtmp, N));
  ACK(dalloc(&h->Ainv, gc.nn * gc.nn));
  ACK(dalloc(&h->qm, N));
  ACK(dalloc(&h->cx, N));
  ACK(dalloc(&h->cr, N));
  ACK(dalloc(&h->cz, N));
  ACK(dalloc(&h->cp, N));
  ACK(dalloc(&h->cp2, N));
  if (g0.dim == 3) ACK(dalloc(&h->dg0, N));
  ACK(dalloc(&h->cw, N));
  long long cap = stencil_num_partials(g0);
  {
    StencilCfg cand[STENCIL_MAX_CANDIDATES];
    const int nc = stencil_candidates(g0, cand, STENCIL_MAX_CANDIDATES);
    for (int i = 0; i < nc; ++i) cap = std::max<long long>(cap, stencil_num_partials(g0, &cand[i]));
  }
  cap = cap > 1024LL * 64 ? cap : 1024LL * 64;   // multi-value partials (Gram, OC)
  h->part_cap = cap;
  ACK(dalloc(&h->pa, cap));
  ACK(dalloc(&h->pb, cap));
  ACK(dalloc(&h->pc, cap));
  ACK(dalloc(&h->scal, 16));
  // the coarsest-build status word follows the CG state, so that one copy
  // to the host brings both
  ACK(dalloc(&h->st, 2));
  h->dstatus = reinterpret_cast<int*>(h->st + 1);
  HIPCK(hipHostMalloc((void**)&h->hpin, sizeof(HostPin), hipHostMallocDefault));
  ACK(dalloc(&h->md, 1));
  ACK(dalloc(&h->oc, 1));
  ACK(dalloc(&h->R, N * p->n_basis));
  ACK(dalloc(&h->Wm, N * p->n_basis));
  ACK(dalloc(&h->invHs, E));
  ACK(dalloc(&h->wvol, E));
  ACK(dalloc(&h->gtmp, E));
  HIPCK(hipEventCreate(&h->e0));
  HIPCK(hipEventCreate(&h->e1));
  if (h->L >= 2) {
    std::vector<Geo> gs(h->L);
    std::vector<const void*> ks(h->L);
    for (int l = 0; l < h->L; ++l) { gs[l] = h->lv[l].g; ks[l] = h->lv[l].k; }
    h->lt = h->L - 1;
    for (int lt = 1; lt < h->L; ++lt) {
      TailSpec T;
      if (tail_plan(gs.data(), ks.data(), lt, h->L, sizeof(double), &T)) { h->lt = lt; break; }
    }
    if (!tail_plan(gs.data(), ks.data(), h->lt, h->L, sizeof(double), &h->tail)) return MGAR_E_DIMS;
  }
  if (p->precision == MGAR_PREC_MIXED) {
    h->mixed = true;
    h->kmin_f = (float)p->kmin;
    h->kdiff_f = (float)(p->k0 - p->kmin);
    ACK(dalloc(&h->dens, E));
    ACK(dalloc(&h->dens0, E));
    ACK(dalloc(&h->k32, E));
    h->kf.assign(h->L, nullptr);
    h->bf.assign(h->L, nullptr);
    h->xaf.assign(h->L, nullptr);
    h->xbf.assign(h->L, nullptr);
    for (int l = 0; l < h->L; ++l) {
      const Geo& gl = h->lv[l].g;
      ACK(dalloc(&h->xaf[l], gl.nn));
      if (l > 0) {
        ACK(dalloc(&h->kf[l], gl.ne));
        ACK(dalloc(&h->bf[l], gl.nn));
        ACK(dalloc(&h->xbf[l], gl.nn));
      }
    }
    ACK(dalloc(&h->rtmpf, N));
    ACK(dalloc(&h->r32, N));
    ACK(dalloc(&h->z32, N));
    ACK(dalloc(&h->p32, N));
    ACK(dalloc(&h->p32b, N));
    if (g0.dim == 3) ACK(dalloc(&h->dg32, N));
    ACK(dalloc(&h->w32, N));
    ACK(dalloc(&h->d32, N));
    if (h->L >= 2) {
      std::vector<Geo> gs(h->L);
      std::vector<const void*> ks(h->L);
      for (int l = 0; l < h->L; ++l) { gs[l] = h->lv[l].g; ks[l] = h->kf[l]; }
      h->ltf = h->L - 1;
      for (int lt = 1; lt < h->L; ++lt) {
        TailSpec T;
        if (tail_plan(gs.data(), ks.data(), lt, h->L, sizeof(float), &T)) { h->ltf = lt; break; }
      }
      if (!tail_plan(gs.data(), ks.data(), h->ltf, h->L, sizeof(float), &h->tailf)) return MGAR_E_DIMS;
    }
  }
  ACK(set_filter(h, p->filter_r));
  HIPCK(hipStreamSynchronize(h->s));
  return MGAR_OK;
}

int mgar_setup(const mgar_params* p, void* stream, mgar_handle** out) {
  if (!out) return MGAR_E_ARG;
  *out = nullptr;
  mgar_handle* h = nullptr;
  const int rc = setup_impl(p, stream, &h);
  if (rc != MGAR_OK) {
    mgar_destroy(h);
    return rc;
  }
  *out = h;
  return MGAR_OK;
}

int mgar_set_stream(mgar_handle* h, void* stream) {
  if (!h) return MGAR_E_ARG;
  h->s = (hipStream_t)stream;
  return MGAR_OK;
}

int mgar_sizes(const mgar_handle* h, int level, long long* nnodes, long long* nelem) {
  if (!h || level < 0 || level >= h->L) return MGAR_E_ARG;
  if (nnodes) *nnodes = h->lv[level].g.nn;
  if (nelem) *nelem = h->lv[level].g.ne;
  return MGAR_OK;
}

int mgar_load_vector(mgar_handle* h, const double* Qe, double* q) {
  if (!h || !Qe || !q) return MGAR_E_ARG;
  launch_load(h->lv[0].g, Qe, q, h->s);
  LAUNCHCK();
  return MGAR_OK;
}

int mgar_density_filter(mgar_handle* h, const double* x, double* xphys) {
  if (!h || !x || !xphys) return MGAR_E_ARG;
  launch_filter_fwd(h->lv[0].g, h->tap_off, h->tap_w, h->ntap, h->tap_hr, x, h->invHs, xphys, h->s);
  LAUNCHCK();
  return MGAR_OK;
}

int mgar_smooth_boundary(mgar_handle* h, const double* dc, double volfrac, double r, int nsub, double* rho,
                         double* ns, double* level, double* volume) {
  if (!h || !dc || !rho || !(volfrac > 0.0 && volfrac <= 1.0) || !(r > 0.0) || nsub < 1 || nsub > 64)
    return MGAR_E_ARG;
  if ((int)std::ceil(r) > (h->p.dim == 3 ? MGAR_MAX_FILTER_R3 : MGAR_MAX_FILTER_R2)) return MGAR_E_ARG;
  const Geo& g = h->lv[0].g;
  if (!h->sdev) ACK(dalloc(&h->sdev, 1));
  const long long need = smooth_num_partials(g);
  if (need > h->spart_cap) {
    if (h->spart) HIPCK(hipFree(h->spart));
    h->spart = nullptr;
    h->spart_cap = 0;
    ACK(dalloc(&h->spart, need));
    h->spart_cap = need;
  }
  double* nsv = ns ? ns : h->rtmp;
  launch_node_project(g, dc, r, nsv, h->s);
  launch_smooth_bisect(g, nsv, volfrac * (double)h->E, nsub, 100, h->sdev, rho, h->spart, h->s);
  LAUNCHCK();
  SmoothDev hs;
  HIPCK(hipMemcpyAsync(&hs, h->sdev, sizeof(SmoothDev), hipMemcpyDeviceToHost, h->s));
  HIPCK(hipStreamSynchronize(h->s));
  if (level) *level = hs.lo;
  if (volume) *volume = hs.vol;
  return MGAR_OK;
}

int mgar_set_filter_radius(mgar_handle* h, double r) {
  if (!h || !(r > 0.0)) return MGAR_E_ARG;
  if ((int)std::ceil(r) > (h->p.dim == 3 ? MGAR_MAX_FILTER_R3 : MGAR_MAX_FILTER_R2)) return MGAR_E_ARG;
  if (r == h->filter_r) return MGAR_OK;
  return set_filter(h, r);
}

int mgcg_solve(mgar_handle* h, const double* xphys, const double* q, const double* T0,
               double tol, double* T, mgar_stats* stats) {
  if (!h || !xphys || !q || !T) return MGAR_E_ARG;
  stats_init(stats);
  HIPCK(hipEventRecord(h->e0, h->s));
  const Geo& g = h->lv[0].g;
  launch_simp(xphys, h->kcur, h->E, h->p.k0, h->p.kmin, h->p.penal, h->s);
  int nref = 0;
  launch_copy(h->kcur, h->lv[0].k, h->E, h->s);
  if (h->mixed) {
    launch_cast_bf16(xphys, h->dens, h->E, h->s);
    ACK(build_hierarchy32(h));
  } else {
    ACK(build_hierarchy(h));
  }
  launch_mask_copy(g, q, h->qm, h->s);
  if (T0) launch_mask_copy(g, T0, h->cx, h->s);
  else HIPCK(hipMemsetAsync(h->cx, 0, sizeof(double) * h->N, h->s));
  int iters = 0, conv = 0;
  double rel = 0.0;
  if (h->mixed) ACK(solve_mixed(h, tol, &iters, &conv, &rel, &nref));
  else ACK(pcg(h, h->kcur, tol, &iters, &conv, &rel));
  launch_copy(h->cx, T, h->N, h->s);
  LAUNCHCK();
  ACK(check_coarse(h));
  h->has_k0 = true;
  ACK(finish_timing(h, stats));
  if (stats) {
    stats->path = MGAR_PATH_MGCG;
    stats->cg_iters = iters;
    stats->vcycles = iters;
    stats->refinements = nref;
    stats->res_final = rel;
  }
  return conv ? MGAR_OK : MGAR_W_NOT_CONVERGED;
}

int mgar_solve(mgar_handle* h, const double* xphys, const double* q, const double* T0,
               double tol, double* T, mgar_stats* stats) {
  if (!h || !xphys || !q || !T) return MGAR_E_ARG;
  if (!h->has_k0) return MGAR_E_STATE;
  stats_init(stats);
  HIPCK(hipEventRecord(h->e0, h->s));
  const Geo& g = h->lv[0].g;
  const long long N = h->N;
  const int m = h->p.n_basis;
  launch_simp(xphys, h->kcur, h->E, h->p.k0, h->p.kmin, h->p.penal, h->s);
  if (h->mixed) launch_cast_bf16(xphys, h->dens, h->E, h->s);
  launch_mask_copy(g, q, h->qm, h->s);
  // r_1 = t_prev
  if (T0) launch_mask_copy(g, T0, h->R, h->s);
  else HIPCK(hipMemsetAsync(h->R, 0, sizeof(double) * N, h->s));
  // r_i = MG(K0, -dK r_{i-1}, x0, P)   (Eq 17)
  for (int i = 1; i < m; ++i) {
    const double* prev = h->R + (long long)(i - 1) * N;
    if (h->mixed) {
      // -dK r in FP64 from the FP64 conductivities (a difference of two nearby
      // operators: BF16 densities would lose most of its digits), then one FP32
      // V-cycle on the BF16 K0 hierarchy; the column is kept in FP64
      ACK(stencil_at(h, 0, SM_NEG_DK, prev, h->kcur, h->lv[0].k, nullptr, h->cz, 0.0, nullptr, nullptr));
      launch_mask_copy_t<double, float>(g, h->cz, h->z32, h->s);
      if (!h->p.basis_x0_zero) launch_mask_copy_t<double, float>(g, prev, h->r32, h->s);
      ACK(vcycle32(h, h->z32, h->p.basis_x0_zero ? nullptr : h->r32, h->w32, nullptr, nullptr));
      launch_mask_copy_t<float, double>(g, h->w32, h->R + (long long)i * N, h->s);
    } else {
      ACK(stencil_at(h, 0, SM_NEG_DK, prev, h->kcur, h->lv[0].k, nullptr, h->cz, 0.0, nullptr, nullptr));
      ACK(vcycle(h, h->cz, h->p.basis_x0_zero ? nullptr : prev, h->R + (long long)i * N, nullptr, nullptr));
    }
  }
  // Eq 18 (as Gram-Schmidt, FP64 in both forms), Eq 19-21; ||q||^2 comes
  // with the Gram products
  launch_gs_fused(h->R, m, N, N, h->md, h->pa, h->pb, h->s);
  for (int j = 0; j < m; ++j)
    ACK(stencil_at(h, 0, SM_APPLY, h->R + (long long)j * N, h->kcur, nullptr, nullptr,
                   h->Wm + (long long)j * N, 0.0, nullptr, nullptr));
  const int np = launch_gram(h->R, h->Wm, h->qm, m, N, N, h->pb, h->s);
  // reduced solve, t~ = Q y in cx; FP64: also r = q - W y in cr, the residual
  // of t~ the fallback PCG starts from (its ||r||^2 partials stay in pa)
  const int nres = launch_combine(h->R, h->Wm, h->qm, m, N, N, h->md, h->cx, h->pa, h->s,
                                  h->mixed ? nullptr : h->cr, h->pb, np);
  launch_finalize(h->pa, nres, &h->md->res2, nullptr, h->s);
  LAUNCHCK();
  MgarDev hm;
  HIPCK(hipMemcpyAsync(&hm, h->md, sizeof(MgarDev), hipMemcpyDeviceToHost, h->s));
  HIPCK(hipStreamSynchronize(h->s));
  const double res = (hm.qq > 0.0) ? std::sqrt(hm.res2 / hm.qq) : 0.0;
  if (stats) {
    stats->res_ca = res;
    stats->vcycles = m - 1;
  }
  if (hm.spd_fail) return MGAR_E_NOT_SPD;
  int rc = MGAR_OK;
  if (res <= h->p.eps_accept) {
    launch_copy(h->cx, T, N, h->s);
    LAUNCHCK();
    if (stats) {
      stats->path = MGAR_PATH_ACCEPT;
      stats->res_final = res;
    }
  } else {
    // reconstruction: K becomes the new K0, MGCG from the reduced solution
    int iters = 0, conv = 0, nref = 0;
    double rel = 0.0;
    launch_copy(h->kcur, h->lv[0].k, h->E, h->s);
    if (h->mixed) {
      ACK(build_hierarchy32(h));
      ACK(solve_mixed(h, tol, &iters, &conv, &rel, &nref));
    } else {
      ACK(build_hierarchy(h));
      ACK(pcg(h, h->kcur, tol, &iters, &conv, &rel, nres));
    }
    if (stats) stats->refinements = nref;
    launch_copy(h->cx, T, N, h->s);
    LAUNCHCK();
    ACK(check_coarse(h));
    if (stats) {
      stats->path = MGAR_PATH_FALLBACK;
      stats->cg_iters = iters;
      stats->vcycles += iters;
      stats->res_final = rel;
    }
    rc = conv ? MGAR_OK : MGAR_W_NOT_CONVERGED;
  }
  ACK(finish_timing(h, stats));
  return rc;
}

// Sensitivities and their filter; with `compliance`, q^T T is also reduced
// into h->scal[1] (no host synchronisation here).
static void enqueue_sens(mgar_handle* h, const double* xphys, const double* T, const double* q, double* dc,
                  double* dv, bool compliance) {
  const Geo& g = h->lv[0].g;
  launch_sens_elem(g, xphys, T, h->invHs, h->p.k0, h->p.kmin, h->p.penal, h->gtmp, h->s);
  launch_filter_fwd(g, h->tap_off, h->tap_w, h->ntap, h->tap_hr, h->gtmp, nullptr, dc, h->s);
  launch_copy(h->wvol, dv, h->E, h->s);
  if (compliance) {
    launch_mask_copy(g, q, h->qm, h->s);
    const int np = launch_dot(h->qm, T, h->N, h->pa, nullptr, h->s);
    launch_finalize(h->pa, np, &h->scal[1], nullptr, h->s);
  }
}

int sens_filter(mgar_handle* h, const double* xphys, const double* T, const double* q, double* dc,
                double* dv, double* compliance) {
  if (!h || !xphys || !T || !q || !dc || !dv) return MGAR_E_ARG;
  enqueue_sens(h, xphys, T, q, dc, dv, compliance != nullptr);
  LAUNCHCK();
  if (compliance) {
    HIPCK(hipMemcpyAsync(compliance, &h->scal[1], sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCK(hipStreamSynchronize(h->s));
  }
  return MGAR_OK;
}

// The OC update; with dev_scalar, that device value comes back to
// *host_scalar in the first synchronisation (through the pinned buffer).
static int oc_run(mgar_handle* h, const double* x, const double* dc, const double* dv, double volfrac,
                  double move, double* x_new, double* lambda, const double* dev_scalar, double* host_scalar) {
  const double target = volfrac * (double)h->E;
  const bool hinted = h->oc_hint > 0.0;
  launch_oc_init(h->oc, target, h->oc_hint, h->s);
  OcDev ho;
  int passes = 0;
  for (;;) {
    // typically 4-7 passes (one fewer from the last multiplier); passes after
    // convergence return at once, so the first batch is sized to need no
    // second synchronisation
    const int chunk = passes == 0 ? (hinted ? 6 : 7) : 4;
    for (int c = 0; c < chunk; ++c) {
      const int np = launch_oc_pass(x, dc, dv, h->E, move, h->oc, h->pa, h->s);
      launch_oc_walk(h->oc, h->pa, np, target, 1e-10, h->s);
    }
    // the update from the multiplier reached so far, enqueued before the
    // synchronisation (it only reads the bisection state); when more passes
    // follow, the next one overwrites x_new. Not when x_new is x itself:
    // later passes still read x.
    if (x_new != x) launch_oc_final(x, dc, dv, h->E, move, h->oc, x_new, h->s);
    LAUNCHCK();
    if (passes == 0 && dev_scalar)
      HIPCK(hipMemcpyAsync(&h->hpin->extra[0], dev_scalar, sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCK(hipMemcpyAsync(&h->hpin->oc, h->oc, sizeof(OcDev), hipMemcpyDeviceToHost, h->s));
    HIPCK(hipStreamSynchronize(h->s));
    if (passes == 0 && dev_scalar) *host_scalar = h->hpin->extra[0];
    ho = h->hpin->oc;
    passes += chunk;
    if (ho.done || passes > 64) break;
  }
  if (x_new == x) launch_oc_final(x, dc, dv, h->E, move, h->oc, x_new, h->s);
  LAUNCHCK();
  const double lam = 0.5 * (ho.l1 + ho.l2);
  h->oc_hint = (ho.done && lam > 0.0 && lam < 1e9) ? lam : 0.0;
  if (lambda) *lambda = lam;
  return MGAR_OK;
}

int oc_update(mgar_handle* h, const double* x, const double* dc, const double* dv, double volfrac,
              double move, double* x_new, double* lambda) {
  if (!h || !x || !dc || !dv || !x_new) return MGAR_E_ARG;
  return oc_run(h, x, dc, dv, volfrac, move, x_new, lambda, nullptr, nullptr);
}

int mgar_sens_oc(mgar_handle* h, const double* xphys, const double* T, const double* q, const double* x,
                 double volfrac, double move, double* dc, double* dv, double* x_new, double* compliance,
                 double* lambda) {
  if (!h || !xphys || !T || !q || !x || !dc || !dv || !x_new) return MGAR_E_ARG;
  enqueue_sens(h, xphys, T, q, dc, dv, compliance != nullptr);
  LAUNCHCK();
  return oc_run(h, x, dc, dv, volfrac, move, x_new, lambda, compliance ? &h->scal[1] : nullptr, compliance);
}

int mgar_set_timing(mgar_handle* h, int on) {
  if (!h) return MGAR_E_ARG;
  h->timing = on != 0;
  return MGAR_OK;
}

int mgar_reset(mgar_handle* h) {
  if (!h) return MGAR_E_ARG;
  h->has_k0 = false;
  h->oc_hint = 0.0;
  return MGAR_OK;
}

int mgar_op_apply(mgar_handle* h, int level, const double* k, const double* x, double* y) {
  if (!h || !k || !x || !y || level < 0 || level >= h->L) return MGAR_E_ARG;
  const Geo& g = h->lv[level].g;
  launch_mask_copy(g, x, h->rtmp, h->s);
  launch_stencil(g, SM_APPLY, h->rtmp, k, nullptr, nullptr, y, 0.0, nullptr, nullptr, h->s, nullptr,
                 nullptr, nullptr, nullptr, &h->scfg[0][level][SM_APPLY]);
  LAUNCHCK();
  return MGAR_OK;
}

int mgar_op_jacobi(mgar_handle* h, int level, const double* k, const double* b, const double* x,
                   double* out) {
  if (!h || !k || !b || !x || !out || level < 0 || level >= h->L) return MGAR_E_ARG;
  const Geo& g = h->lv[level].g;
  launch_mask_copy(g, x, h->rtmp, h->s);
  launch_mask_copy(g, b, h->cz, h->s);
  launch_stencil(g, SM_JACOBI, h->rtmp, k, nullptr, h->cz, out, h->p.omega, nullptr, nullptr, h->s,
                 nullptr, nullptr, nullptr, nullptr, &h->scfg[0][level][SM_JACOBI]);
  LAUNCHCK();
  return MGAR_OK;
}

int mgar_op_restrict(mgar_handle* h, int level, const double* rf, double* rc) {
  if (!h || !rf || !rc || level < 0 || level + 1 >= h->L) return MGAR_E_ARG;
  launch_mask_copy(h->lv[level].g, rf, h->rtmp, h->s);
  launch_restrict(h->lv[level].g, h->lv[level + 1].g, h->rtmp, rc, nullptr, h->s);
  LAUNCHCK();
  return MGAR_OK;
}

int mgar_op_prolong(mgar_handle* h, int level, const double* xc, double* xf) {
  if (!h || !xc || !xf || level < 0 || level + 1 >= h->L) return MGAR_E_ARG;
  launch_mask_copy(h->lv[level + 1].g, xc, h->rtmp, h->s);
  launch_mask_copy(h->lv[level].g, xf, xf, h->s);
  launch_prolong(h->lv[level].g, h->lv[level + 1].g, h->rtmp, xf, nullptr, h->s);
  LAUNCHCK();
  return MGAR_OK;
}

int mgar_op_coarsen(mgar_handle* h, int level, const double* kf, double* kc) {
  if (!h || !kf || !kc || level < 0 || level + 1 >= h->L) return MGAR_E_ARG;
  launch_coarsen(h->lv[level].g, h->lv[level + 1].g, kf, kc, h->s);
  LAUNCHCK();
  return MGAR_OK;
}

int mgar_build_hierarchy(mgar_handle* h, const double* xphys) {
  if (!h || !xphys) return MGAR_E_ARG;
  launch_simp(xphys, h->lv[0].k, h->E, h->p.k0, h->p.kmin, h->p.penal, h->s);
  if (h->mixed) {
    launch_cast_bf16(xphys, h->dens, h->E, h->s);
    ACK(build_hierarchy32(h));
  } else {
    ACK(build_hierarchy(h));
  }
  ACK(check_coarse(h));
  h->has_k0 = true;
  return MGAR_OK;
}

int mgar_vcycle(mgar_handle* h, const double* b, const double* x0, double* x) {
  if (!h || !b || !x) return MGAR_E_ARG;
  if (!h->has_k0) return MGAR_E_STATE;
  const Geo& g = h->lv[0].g;
  if (h->mixed) {
    launch_mask_copy_t<double, float>(g, b, h->z32, h->s);
    if (x0) launch_mask_copy_t<double, float>(g, x0, h->r32, h->s);
    ACK(vcycle32(h, h->z32, x0 ? h->r32 : nullptr, h->w32, nullptr, nullptr));
    launch_mask_copy_t<float, double>(g, h->w32, x, h->s);
    LAUNCHCK();
    return MGAR_OK;
  }
  launch_mask_copy(g, b, h->cz, h->s);
  if (x0) launch_mask_copy(g, x0, h->cr, h->s);
  ACK(vcycle(h, h->cz, x0 ? h->cr : nullptr, x, nullptr, nullptr));
  return MGAR_OK;
}

int mgar_op_dk(mgar_handle* h, const double* xphys, const double* r, double* b) {
  if (!h || !xphys || !r || !b) return MGAR_E_ARG;
  if (!h->has_k0) return MGAR_E_STATE;
  const Geo& g = h->lv[0].g;
  launch_simp(xphys, h->kcur, h->E, h->p.k0, h->p.kmin, h->p.penal, h->s);
  launch_mask_copy(g, r, h->rtmp, h->s);
  launch_stencil(g, SM_NEG_DK, h->rtmp, h->kcur, h->lv[0].k, nullptr, b, 0.0, nullptr, nullptr, h->s,
                 nullptr, nullptr, nullptr, nullptr, &h->scfg[0][0][SM_NEG_DK]);
  LAUNCHCK();
  return MGAR_OK;
}

int mgar_op_bf16(mgar_handle* h, const double* x, void* out) {
  if (!h || !x || !out) return MGAR_E_ARG;
  launch_cast_bf16(x, static_cast<uint16_t*>(out), h->E, h->s);
  LAUNCHCK();
  return MGAR_OK;
}

// ---------------------------------------------------------------- launch-shape tuning

int mgar_tune_get(const mgar_handle* h, int cls, int level, int mode, int* shape) {
  if (!h || !shape || cls < 0 || cls > 1 || level < 0 || level >= h->L || mode < 0 || mode > 6)
    return MGAR_E_ARG;
  const StencilCfg& c = h->scfg[cls][level][mode];
  shape[0] = c.kind;
  shape[1] = c.kz;
  shape[2] = c.zd;
  shape[3] = c.ntx;
  return MGAR_OK;
}

int mgar_tune_set(mgar_handle* h, int cls, int level, int mode, const int* shape) {
  if (!h || !shape || cls < 0 || cls > 1 || level < 0 || level >= h->L || mode < 0 || mode > 6)
    return MGAR_E_ARG;
  const StencilCfg c{shape[0], shape[1], shape[2], shape[3]};
  const Geo& g = h->lv[level].g;
  if (!stencil_cfg_valid(g, c)) return MGAR_E_ARG;
  if (stencil_num_partials(g, &c) > h->part_cap) return MGAR_E_ARG;
  h->scfg[cls][level][mode] = c;
  drop_graphs(h);   // captured iterations hold the old shapes
  return MGAR_OK;
}

int mgar_set_graphs(mgar_handle* h, int on) {
  if (!h) return MGAR_E_ARG;
  h->use_graphs = on != 0;
  return MGAR_OK;
}

namespace {

// Times every candidate shape of one (class, level, mode) on scratch data and
// keeps the fastest. Returns the best average launch time in microseconds.
// Each timed launch records its own pair of events at kernel start and end,
// so the comparison is of kernel durations, not of launch overheads.
int tune_one(mgar_handle* h, int cls, int level, int mode, int reps, double* xd, double* bd,
             double* od, double* kd, uint16_t* kb, const std::vector<hipEvent_t>& ev,
             double* best_us) {
  const Geo& g = h->lv[level].g;
  StencilCfg cand[STENCIL_MAX_CANDIDATES];
  const int nc = stencil_candidates(g, cand, STENCIL_MAX_CANDIDATES);
  double best = -1.0;
  int bi = 0;
  for (int i = 0; i < nc; ++i) {
    if (stencil_num_partials(g, &cand[i]) > h->part_cap) continue;
    // events (when given) are recorded at the start and end of the kernel itself
    auto launch = [&](hipEvent_t e0, hipEvent_t e1) {
      if (cls == 0) {
        launch_stencil(g, mode, xd, kd, kd + g.ne, bd, od, h->p.omega, h->pa, nullptr, h->s, nullptr,
                       nullptr, e0, e1, &cand[i]);
      } else if (level == 0) {
        const CellB k{kb, h->kmin_f, h->kdiff_f}, kr{kb + g.ne, h->kmin_f, h->kdiff_f};
        launch_stencil_t<float, CellB>(g, mode, (const float*)xd, k, kr, (const float*)bd, (float*)od,
                                       h->p.omega, h->pa, nullptr, h->s, nullptr, nullptr, e0, e1,
                                       &cand[i]);
      } else {
        const CellF k{(const float*)kd}, kr{(const float*)kd + g.ne};
        launch_stencil_t<float, CellF>(g, mode, (const float*)xd, k, kr, (const float*)bd, (float*)od,
                                       h->p.omega, h->pa, nullptr, h->s, nullptr, nullptr, e0, e1,
                                       &cand[i]);
      }
    };
    launch(nullptr, nullptr);
    launch(nullptr, nullptr);
    for (int r = 0; r < reps; ++r) launch(ev[2 * r], ev[2 * r + 1]);
    HIPCK(hipEventSynchronize(ev[2 * reps - 1]));
    LAUNCHCK();
    double us = 0.0;
    for (int r = 0; r < reps; ++r) {
      float ms = 0.f;
      HIPCK(hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]));
      us += 1e3 * (double)ms;
    }
    us /= reps;
    if (best < 0.0 || us < best) { best = us; bi = i; }
  }
  if (best >= 0.0) h->scfg[cls][level][mode] = cand[bi];
  *best_us = best;
  return MGAR_OK;
}

}  // namespace

int mgar_autotune(mgar_handle* h, int reps, double* best_us) {
  if (!h || reps < 1) return MGAR_E_ARG;
  drop_graphs(h);
  const int L = h->L;
  if (best_us)
    for (int i = 0; i < 2 * L * 7; ++i) best_us[i] = 0.0;
  const long long N = h->N, E = h->E;
  double *xd = nullptr, *bd = nullptr, *od = nullptr, *kd = nullptr;
  uint16_t* kb = nullptr;
  std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
  int rc = MGAR_OK;
  do {
    if (hipMalloc((void**)&xd, sizeof(double) * N) != hipSuccess ||
        hipMalloc((void**)&bd, sizeof(double) * N) != hipSuccess ||
        hipMalloc((void**)&od, sizeof(double) * N) != hipSuccess ||
        hipMalloc((void**)&kd, sizeof(double) * 2 * E) != hipSuccess ||
        hipMalloc((void**)&kb, sizeof(uint16_t) * 2 * E) != hipSuccess) {
      rc = MGAR_E_HIP;
      break;
    }
    for (hipEvent_t& e : ev)
      if (hipEventCreate(&e) != hipSuccess) rc = MGAR_E_HIP;
    if (rc != MGAR_OK) break;
    const int ncls = h->mixed ? 2 : 1;
    for (int cls = 0; cls < ncls && rc == MGAR_OK; ++cls) {
      // scratch contents: smooth positive values of the class's element type
      if (cls == 0) {
        launch_fill_t<double>(xd, N, 0.5f, 0.001f, h->s);
        launch_fill_t<double>(bd, N, 0.1f, 0.001f, h->s);
        launch_fill_t<double>(kd, 2 * E, 0.3f, 0.005f, h->s);
      } else {
        launch_fill_t<float>((float*)xd, N, 0.5f, 0.001f, h->s);
        launch_fill_t<float>((float*)bd, N, 0.1f, 0.001f, h->s);
        launch_fill_t<float>((float*)kd, 2 * E, 0.3f, 0.005f, h->s);
        launch_fill_bf16(kb, 2 * E, h->s);
      }
      const int lt = (cls == 0) ? h->lt : h->ltf;
      for (int l = 0; l < L && rc == MGAR_OK; ++l) {
        if (l > 0 && l >= lt) break;   // grids below handled by the tail kernel
        for (int m = 0; m < 7 && rc == MGAR_OK; ++m) {
          // coarser grids only run the smoother sweeps and the residual
          if (l > 0 && m != SM_JACOBI0 && m != SM_RESID && m != SM_JACOBI) continue;
          double us = 0.0;
          rc = tune_one(h, cls, l, m, reps, xd, bd, od, kd, kb, ev, &us);
          if (best_us) best_us[(cls * L + l) * 7 + m] = us;
        }
      }
    }
  } while (0);
  (void)hipStreamSynchronize(h->s);
  if (xd) (void)hipFree(xd);
  if (bd) (void)hipFree(bd);
  if (od) (void)hipFree(od);
  if (kd) (void)hipFree(kd);
  if (kb) (void)hipFree(kb);
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

int mgar_profile(mgar_handle* h, unsigned mode_mask) {
  if (!h) return MGAR_E_ARG;
  h->prof_mask = mode_mask;
  return MGAR_OK;
}

int mgar_profile_read(mgar_handle* h, long long* launches, double* total_ms, double* total_bytes) {
  if (!h) return MGAR_E_ARG;
  HIPCK(hipStreamSynchronize(h->s));
  ACK(profile_harvest(h));
  if (launches) *launches = h->prof_launches;
  if (total_ms) *total_ms = h->prof_ms;
  if (total_bytes) *total_bytes = h->prof_total_bytes;
  h->prof_launches = 0;
  h->prof_ms = 0.0;
  h->prof_total_bytes = 0.0;
  return MGAR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- residual check

int mgar_residual(mgar_handle* h, const double* xphys, const double* q, const double* T, double* relres) {
  if (!h || !xphys || !q || !T || !relres) return MGAR_E_ARG;
  const Geo& g = h->lv[0].g;
  const long long N = h->N;
  launch_simp(xphys, h->kcur, h->E, h->p.k0, h->p.kmin, h->p.penal, h->s);
  launch_mask_copy(g, q, h->qm, h->s);
  launch_mask_copy(g, T, h->cz, h->s);
  launch_stencil(g, SM_RESID, h->cz, h->kcur, nullptr, h->qm, h->cr, 0.0, nullptr, nullptr, h->s, nullptr,
                 nullptr, nullptr, nullptr, &h->scfg[0][0][SM_RESID]);
  const int nr = launch_dot(h->cr, h->cr, N, h->pa, nullptr, h->s);
  launch_finalize(h->pa, nr, &h->scal[4], nullptr, h->s);
  const int nq = launch_dot(h->qm, h->qm, N, h->pb, nullptr, h->s);
  launch_finalize(h->pb, nq, &h->scal[5], nullptr, h->s);
  LAUNCHCK();
  double v[2];
  HIPCK(hipMemcpyAsync(v, &h->scal[4], 2 * sizeof(double), hipMemcpyDeviceToHost, h->s));
  HIPCK(hipStreamSynchronize(h->s));
  *relres = v[1] > 0.0 ? std::sqrt(v[0] / v[1]) : 0.0;
  return MGAR_OK;
}

// ---------------------------------------------------------------- shared with batch.hip
Geo mgar_internal_geo(const mgar_params& p, int level) { return make_geo(p, level); }
long long mgar_internal_count_fixed(const Geo& g) { return count_fixed(g); }
int mgar_internal_validate(const mgar_params* p) { return validate(p); }
