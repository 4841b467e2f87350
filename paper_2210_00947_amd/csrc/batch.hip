// Batched solves: many independent designs (uneven grids, 2D and 3D) advanced
// together. Every stage of a V-cycle, of a PCG iteration and of the
// reanalysis step is ONE launch per dimension group over a work list of
// (design, grid) items, so a batch of small designs costs about as many
// launches as one design. Convergence is per design: the PCG state of each
// design (BCgState, iteration counter included) lives on the device and every
// kernel skips the blocks of designs that are done, so the launches of a PCG
// iteration are captured once in a hipGraph and replayed until all designs
// have stopped.
//
// Arrays passed through the ABI are concatenations over designs in the order
// of the params array (layout from mgar_batch_layout). The arithmetic per
// design is that of the single-design FP64 path (same stencil, transfer,
// smoother, tail and coarsest-inverse code); only dot products are summed in
// a different block order.
//
// Mixed precision (every design MGAR_PREC_MIXED): the preconditioner is an
// FP32 V-cycle over BF16-stored densities (FP32 cell means below the finest
// grid, FP64 coarsest inverse), the basis vectors of the reanalysis come from
// FP32 V-cycles on FP64 right-hand sides, and the PCG is plain iterative
// refinement: r = q - K x in FP64, an FP32 PCG run on K32 d = r until its
// residual has dropped by inner_tol, x += d, repeated per design until
// ||r|| <= tol ||q|| in FP64 (or the design's CG budget or the refinement
// limit is spent). The single-design mixed path instead continues one Krylov
// run across its residual replacements; the batched form restarts each
// inner run so that designs stay independent with a scalar inner tolerance.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "mgar.h"
#include "mgar_launch.h"

namespace {

#define BHIP(x)                                   \
  do {                                            \
    hipError_t err_ = (x);                        \
    if (err_ != hipSuccess) return MGAR_E_HIP;    \
  } while (0)
#define BACK(x)                                   \
  do {                                            \
    int rc_ = (x);                                \
    if (rc_ != MGAR_OK) return rc_;               \
  } while (0)
#define BLAUNCH() BHIP(hipGetLastError())

constexpr int ST_STRIDE = (int)(sizeof(BCgState) / sizeof(int));
constexpr int MD_STRIDE = (int)(sizeof(MgarDev) / sizeof(double));
static_assert(sizeof(BCgState) % sizeof(int) == 0, "BCgState stride");
static_assert(sizeof(MgarDev) % sizeof(double) == 0, "MgarDev stride");
constexpr int ITERS_PER_GRAPH = 4;
constexpr int REFINE_MAX = 40;   // FP64 residual replacements per mixed solve
constexpr int BATCH_MIN_BS = 64;  // smallest block of the node-parallel launches

template <typename T>
int dalloc(T** p, long long n) {
  *p = nullptr;
  if (n <= 0) n = 1;
  BHIP(hipMalloc((void**)p, sizeof(T) * (size_t)n));
  return MGAR_OK;
}

// A list of work items in device memory (host copy kept for block counts).
struct ItemList {
  std::vector<BItem> h;
  BItem* d = nullptr;
  int nblk = 0;
  int bs = 256;            // threads (nodes) per block of its launches
  int n() const { return (int)h.size(); }
};

struct Design {
  mgar_params p;
  int L = 0, lt = 1;
  std::vector<Geo> g;
  long long noff = 0, eoff = 0;          // offsets in the concatenated finest arrays
  std::vector<long long> aoff, aeoff;    // offsets in the group arenas, levels >= 1
  long long Aoff = 0;                    // offset of the coarsest inverse
};

struct Group {
  int dim = 0;
  std::vector<int> designs;
  int maxL = 0, maxlt = 0;
  // arenas of grids >= 1 (index l; entry 0 unused): FP64, or FP32 in a
  // mixed batch
  std::vector<double*> b, xa, xb, rt, k;
  std::vector<float*> bf, xaf, xbf, rtf, kf;
  std::vector<ItemList> down, restr, prol, coarsen;   // per level
  ItemList fine;          // finest grid of every design: vector and dot items
  ItemList cells;         // finest cells of every design
  BTail* tails = nullptr;
  int ntails = 0, tail_lds = 0;
  BCoarse* cb_reg = nullptr;
  BCoarse* cb_gen = nullptr;
  int n_reg = 0, n_gen = 0;
};

int upload(ItemList& L) {
  int first = 0;
  for (BItem& it : L.h) {
    it.first = first;
    first += it.nblk;
  }
  L.nblk = first;
  if (L.h.empty()) return MGAR_OK;
  BACK(dalloc(&L.d, (long long)L.h.size()));
  BHIP(hipMemcpy(L.d, L.h.data(), sizeof(BItem) * L.h.size(), hipMemcpyHostToDevice));
  return MGAR_OK;
}

BItem make_item(const Geo& g, const Geo& gc, long long off, long long coff, long long eoff,
                long long ceoff, int design, int nblk) {
  BItem it;
  std::memset(&it, 0, sizeof(it));
  it.g = g;
  it.gc = gc;
  it.off = off;
  it.coff = coff;
  it.eoff = eoff;
  it.ceoff = ceoff;
  it.design = design;
  it.nblk = nblk;
  return it;
}

int blocks_of(long long n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace

struct mgar_batch {
  int nd = 0;
  hipStream_t s = nullptr;
  std::vector<Design> d;
  std::vector<Group> grp;
  long long N = 0, E = 0, Atot = 0;
  int m = 2;
  double omega = 0.8, eps = 1e-8;
  int cg_max = 200;
  int basis_x0_zero = 0;
  bool has_k0 = false;
  bool use_graph = true;
  int bs = 256;            // threads per block of the node-parallel launches (tuned)
  // finest-grid concatenations
  double *kcur = nullptr, *k0 = nullptr;
  double *qm = nullptr, *cx = nullptr, *cr = nullptr, *cz = nullptr, *cp = nullptr, *cw = nullptr;
  double *xa0 = nullptr, *rt0 = nullptr;
  double *R = nullptr, *Wm = nullptr;
  double* Ainv = nullptr;
  double *pa = nullptr, *pb = nullptr, *pc = nullptr;
  BCgState* st = nullptr;
  MgarDev* md = nullptr;
  int *keep = nullptr, *path = nullptr, *status = nullptr;
  double *res = nullptr, *nrm = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // iteration graphs: [0] FP64 PCG, [1] FP32 inner PCG of the mixed form
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  // mixed precision
  bool mixed = false;
  double inner_tol = 1e-3;
  float kmin_f = 0.f, kdiff_f = 0.f;
  uint16_t *dens = nullptr, *dens0 = nullptr;   // BF16 densities: current, K0
  float* k32 = nullptr;                          // FP32 conductivities (inner operator)
  float *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *w32 = nullptr, *d32 = nullptr;
  float *xa32 = nullptr, *rt32 = nullptr;
  int* odone = nullptr;                          // per design: refinement finished
  double *nq = nullptr, *nr = nullptr;           // per design ||q||^2, ||r||^2
  std::vector<int> h_odone, h_iters, h_nref, h_conv;
  std::vector<double> h_rel;
  double tol_captured[2] = {-1.0, -1.0};
  // Work runs on `s`. A graph cannot be captured on the legacy default
  // stream, so when the caller passes NULL the batch owns a stream of its own
  // (default priority) and orders it after the caller's stream at every entry.
  hipStream_t user_s = nullptr;
  bool own_stream = false;
  hipEvent_t ein = nullptr;
};

namespace {

const int* st_done(const mgar_batch* b) { return &b->st[0].done; }

// ---------------------------------------------------------------- stages

// One V-cycle of Table 1 for every design of group G on its K0 hierarchy:
// out = MG(b0, x0) (x0 may be null = zero guess); with part, the final sweep
// also writes the partials of b0 . out per finest block. skip: designs to leave
// untouched.
int bvcycle(mgar_batch* B, Group& G, const double* b0, const double* x0, double* out, double* part,
            const int* skip) {
  const int ss = ST_STRIDE;
  for (int l = 0; l < G.maxlt; ++l) {
    ItemList& D = G.down[l];
    if (D.h.empty()) continue;
    const double* bl = (l == 0) ? b0 : G.b[l];
    double* xal = (l == 0) ? B->xa0 : G.xa[l];
    double* rtl = (l == 0) ? B->rt0 : G.rt[l];
    const double* kl = (l == 0) ? B->k0 : G.k[l];
    if (l == 0 && x0)
      launch_bstencil(G.dim, SM_JACOBI, D.d, D.n(), D.nblk, D.bs, x0, kl, nullptr, bl, xal, B->omega, nullptr,
                      skip, ss, B->s);
    else
      launch_bstencil(G.dim, SM_JACOBI0, D.d, D.n(), D.nblk, D.bs, bl, kl, nullptr, bl, xal, B->omega, nullptr,
                      skip, ss, B->s);
    launch_bstencil(G.dim, SM_RESID, D.d, D.n(), D.nblk, D.bs, xal, kl, nullptr, bl, rtl, B->omega, nullptr,
                    skip, ss, B->s);
    ItemList& Rs = G.restr[l];
    launch_brestrict(G.dim, Rs.d, Rs.n(), Rs.nblk, Rs.bs, rtl, G.b[l + 1], skip, ss, B->s);
  }
  launch_bvtail(G.dim, G.tails, G.ntails, G.tail_lds, B->omega, skip, ss, B->s);
  for (int l = G.maxlt - 1; l >= 0; --l) {
    ItemList& D = G.down[l];
    if (D.h.empty()) continue;
    const double* bl = (l == 0) ? b0 : G.b[l];
    double* xal = (l == 0) ? B->xa0 : G.xa[l];
    const double* kl = (l == 0) ? B->k0 : G.k[l];
    ItemList& P = G.prol[l];
    launch_bprolong(G.dim, P.d, P.n(), P.nblk, P.bs, G.xb[l + 1], xal, skip, ss, B->s);
    double* o = (l == 0) ? out : G.xb[l];
    const int mode = (l == 0 && part) ? SM_JACOBI_DOT : SM_JACOBI;
    launch_bstencil(G.dim, mode, D.d, D.n(), D.nblk, D.bs, xal, kl, nullptr, bl, o, B->omega, part, skip, ss,
                    B->s);
  }
  BLAUNCH();
  return MGAR_OK;
}

// K0 := K(kcur) for every design of G whose keep flag is 0 (all with keep null):
// finest cells, cell means of every coarser grid, coarsest inverses.
int bbuild(mgar_batch* B, Group& G, const int* keep) {
  launch_bcopy_cells(G.cells.d, G.cells.n(), G.cells.nblk, G.cells.bs, B->kcur, B->k0, keep, 1, B->s);
  for (int l = 0; l + 1 < G.maxL; ++l) {
    ItemList& C = G.coarsen[l];
    launch_bcoarsen(G.dim, C.d, C.n(), C.nblk, C.bs, (l == 0) ? B->k0 : G.k[l], G.k[l + 1], keep, 1, B->s);
  }
  launch_bcoarse_build(G.dim, G.cb_reg, G.n_reg, true, B->status, keep, 1, B->s);
  launch_bcoarse_build(G.dim, G.cb_gen, G.n_gen, false, B->status, keep, 1, B->s);
  BLAUNCH();
  return MGAR_OK;
}

// One PCG iteration for every design of G that is not done (device-side
// iteration counters, so the sequence can be captured and replayed).
int biter(mgar_batch* B, Group& G, double tol) {
  ItemList& F = G.fine;
  const int* skip = st_done(B);
  double* rz = &B->st[0].rz[0];
  BACK(bvcycle(B, G, B->cr, nullptr, B->cz, B->pb, skip));
  launch_bfinalize(F.d, F.n(), B->pb, 1, rz, (int)(sizeof(BCgState) / sizeof(double)), &B->st[0].it, skip,
                   ST_STRIDE, B->s);
  launch_bp_update(F.d, F.n(), F.nblk, F.bs, B->cz, B->cp, B->st, B->s);
  launch_bstencil(G.dim, SM_APPLY_DOT, F.d, F.n(), F.nblk, F.bs, B->cp, B->kcur, nullptr, nullptr, B->cw, 0.0,
                  B->pc, skip, ST_STRIDE, B->s);
  launch_bfinalize(F.d, F.n(), B->pc, 1, &B->st[0].pw, (int)(sizeof(BCgState) / sizeof(double)), nullptr,
                   skip, ST_STRIDE, B->s);
  launch_bcg_update(F.d, F.n(), F.nblk, F.bs, B->cx, B->cr, B->cp, B->cw, B->st, B->pa, B->s);
  launch_bcg_check(F.d, F.n(), B->st, B->pa, tol, B->cg_max, B->s);
  BLAUNCH();
  return MGAR_OK;
}

// ---------------------------------------------------------------- FP32 stages

CellB cells_b(const mgar_batch* B, const uint16_t* d) { return CellB{d, B->kmin_f, B->kdiff_f}; }

// FP32 stencil of grid l of group G: the finest grid reads the BF16 K0
// densities, coarser grids FP32 cell means.
void bst32(mgar_batch* B, Group& G, int l, int mode, const ItemList& D, const float* x, const float* b,
           float* out, double* part, const int* skip) {
  if (l == 0)
    launch_bstencil_t<float, CellB>(G.dim, mode, D.d, D.n(), D.nblk, D.bs, x, cells_b(B, B->dens0),
                                    cells_b(B, nullptr), b, out, B->omega, part, skip, ST_STRIDE, B->s);
  else
    launch_bstencil_t<float, CellF>(G.dim, mode, D.d, D.n(), D.nblk, D.bs, x, CellF{G.kf[l]}, CellF{nullptr}, b,
                                    out, B->omega, part, skip, ST_STRIDE, B->s);
}

// The V-cycle of bvcycle in FP32 on the BF16/FP32 K0 hierarchy (FP64
// coarsest inverse); partials of b0 . out in FP64.
int bvcycle32(mgar_batch* B, Group& G, const float* b0, const float* x0, float* out, double* part,
              const int* skip) {
  const int ss = ST_STRIDE;
  for (int l = 0; l < G.maxlt; ++l) {
    ItemList& D = G.down[l];
    if (D.h.empty()) continue;
    const float* bl = (l == 0) ? b0 : G.bf[l];
    float* xal = (l == 0) ? B->xa32 : G.xaf[l];
    float* rtl = (l == 0) ? B->rt32 : G.rtf[l];
    if (l == 0 && x0) bst32(B, G, l, SM_JACOBI, D, x0, bl, xal, nullptr, skip);
    else bst32(B, G, l, SM_JACOBI0, D, bl, bl, xal, nullptr, skip);
    bst32(B, G, l, SM_RESID, D, xal, bl, rtl, nullptr, skip);
    ItemList& Rs = G.restr[l];
    launch_brestrict_t<float>(G.dim, Rs.d, Rs.n(), Rs.nblk, Rs.bs, rtl, G.bf[l + 1], skip, ss, B->s);
  }
  launch_bvtail_t<float>(G.dim, G.tails, G.ntails, G.tail_lds, B->omega, skip, ss, B->s);
  for (int l = G.maxlt - 1; l >= 0; --l) {
    ItemList& D = G.down[l];
    if (D.h.empty()) continue;
    const float* bl = (l == 0) ? b0 : G.bf[l];
    float* xal = (l == 0) ? B->xa32 : G.xaf[l];
    ItemList& P = G.prol[l];
    launch_bprolong_t<float>(G.dim, P.d, P.n(), P.nblk, P.bs, G.xbf[l + 1], xal, skip, ss, B->s);
    float* o = (l == 0) ? out : G.xbf[l];
    bst32(B, G, l, (l == 0 && part) ? SM_JACOBI_DOT : SM_JACOBI, D, xal, bl, o, part, skip);
  }
  BLAUNCH();
  return MGAR_OK;
}

// K0 := K(dens) for every design of G whose keep flag is 0: BF16 densities
// and FP64 cells of the finest grid (the latter for the -dK products of the
// reanalysis), FP32 cell means below, FP64 coarsest inverses.
int bbuild32(mgar_batch* B, Group& G, const int* keep) {
  launch_bcopy_cells_t<uint16_t>(G.cells.d, G.cells.n(), G.cells.nblk, G.cells.bs, B->dens, B->dens0, keep, 1, B->s);
  launch_bcopy_cells(G.cells.d, G.cells.n(), G.cells.nblk, G.cells.bs, B->kcur, B->k0, keep, 1, B->s);
  for (int l = 0; l + 1 < G.maxL; ++l) {
    ItemList& C = G.coarsen[l];
    if (l == 0)
      launch_bcoarsen_t<CellB, float>(G.dim, C.d, C.n(), C.nblk, C.bs, cells_b(B, B->dens0), G.kf[1], keep, 1, B->s);
    else
      launch_bcoarsen_t<CellF, float>(G.dim, C.d, C.n(), C.nblk, C.bs, CellF{G.kf[l]}, G.kf[l + 1], keep, 1, B->s);
  }
  launch_bcoarse_build_t<CellF>(G.dim, G.cb_reg, G.n_reg, true, B->status, keep, 1, B->s);
  launch_bcoarse_build_t<CellF>(G.dim, G.cb_gen, G.n_gen, false, B->status, keep, 1, B->s);
  BLAUNCH();
  return MGAR_OK;
}

// One FP32 PCG iteration on K32 d = r32 for every design that is not done
// (FP64 inner products and scalars).
int biter32(mgar_batch* B, Group& G, double tol) {
  ItemList& F = G.fine;
  const int* skip = st_done(B);
  double* rz = &B->st[0].rz[0];
  BACK(bvcycle32(B, G, B->r32, nullptr, B->z32, B->pb, skip));
  launch_bfinalize(F.d, F.n(), B->pb, 1, rz, (int)(sizeof(BCgState) / sizeof(double)), &B->st[0].it, skip,
                   ST_STRIDE, B->s);
  launch_bp_update_t<float>(F.d, F.n(), F.nblk, F.bs, B->z32, B->p32, B->st, B->s);
  launch_bstencil_t<float, CellF>(G.dim, SM_APPLY_DOT, F.d, F.n(), F.nblk, F.bs, B->p32, CellF{B->k32},
                                  CellF{nullptr}, nullptr, B->w32, 0.0, B->pc, skip, ST_STRIDE, B->s);
  launch_bfinalize(F.d, F.n(), B->pc, 1, &B->st[0].pw, (int)(sizeof(BCgState) / sizeof(double)), nullptr,
                   skip, ST_STRIDE, B->s);
  launch_bcg_update_t<float>(F.d, F.n(), F.nblk, F.bs, B->d32, B->r32, B->p32, B->w32, B->st, B->pa, B->s);
  launch_bcg_check(F.d, F.n(), B->st, B->pa, tol, B->cg_max, B->s);
  BLAUNCH();
  return MGAR_OK;
}

// cls 0: FP64 PCG iterations; cls 1: FP32 inner iterations of the mixed form
int enqueue_iters(mgar_batch* B, int cls, double tol, int n) {
  for (int i = 0; i < n; ++i)
    for (Group& G : B->grp) BACK(cls == 0 ? biter(B, G, tol) : biter32(B, G, tol));
  return MGAR_OK;
}

// Iterations of class cls until every design's PCG state is done (the state
// was initialised by the caller). The iteration is captured as a graph once
// per class and tolerance and replayed in chunks of ITERS_PER_GRAPH.
int run_until_done(mgar_batch* B, int cls, double tol) {
  if (B->use_graph && (!B->gexec[cls] || B->tol_captured[cls] != tol)) {
    if (B->gexec[cls]) { (void)hipGraphExecDestroy(B->gexec[cls]); B->gexec[cls] = nullptr; }
    if (B->graph[cls]) { (void)hipGraphDestroy(B->graph[cls]); B->graph[cls] = nullptr; }
    BHIP(hipStreamBeginCapture(B->s, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_iters(B, cls, tol, ITERS_PER_GRAPH);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(B->s, &gr);
    if (rc != MGAR_OK) return rc;
    BHIP(e);
    B->graph[cls] = gr;
    BHIP(hipGraphInstantiate(&B->gexec[cls], gr, nullptr, nullptr, 0));
    B->tol_captured[cls] = tol;
  }
  std::vector<BCgState> hs(B->nd);
  int done_iters = 0;
  for (;;) {
    BHIP(hipMemcpyAsync(hs.data(), B->st, sizeof(BCgState) * B->nd, hipMemcpyDeviceToHost, B->s));
    BHIP(hipStreamSynchronize(B->s));
    bool all = true;
    for (const BCgState& x : hs) all = all && x.done;
    if (all) break;
    if (done_iters > B->cg_max + ITERS_PER_GRAPH) return MGAR_E_HIP;   // the device test must have fired
    if (B->use_graph) BHIP(hipGraphLaunch(B->gexec[cls], B->s));
    else BACK(enqueue_iters(B, cls, tol, ITERS_PER_GRAPH));
    done_iters += ITERS_PER_GRAPH;
  }
  return MGAR_OK;
}

// PCG from cx for every design (those with keep_done set stay as they are):
// r = q - K x, stopping test, then iterations until every design stopped.
int bpcg(mgar_batch* B, double tol, const int* keep_done) {
  for (Group& G : B->grp) {
    ItemList& F = G.fine;
    launch_bstencil(G.dim, SM_RESID, F.d, F.n(), F.nblk, F.bs, B->cx, B->kcur, nullptr, B->qm, B->cr, 0.0, nullptr,
                    nullptr, 0, B->s);
    launch_bdot(F.d, F.n(), F.nblk, F.bs, B->cr, B->cr, B->pa, nullptr, 0, B->s);
    launch_bdot(F.d, F.n(), F.nblk, F.bs, B->qm, B->qm, B->pb, nullptr, 0, B->s);
    launch_bcg_init(F.d, F.n(), B->st, B->pb, B->pa, tol, B->cg_max, keep_done, B->s);
  }
  BLAUNCH();
  return run_until_done(B, 0, tol);
}

// Mixed form, per design from x = cx (designs with keep_done set are left as
// they are): r = q - K(kcur) x in FP64; stop when ||r|| <= tol ||q||, when the
// design has spent cg_max inner iterations or after REFINE_MAX replacements;
// else an FP32 PCG run from d = 0 on K32 d = r (K32: the FP32 rounding of the
// current conductivities; preconditioner: the FP32 V-cycle on the BF16 K0
// hierarchy) until ||r32|| <= inner_tol ||r32(0)|| or cg_max iterations, and
// x += d in FP64. One host synchronisation per replacement (the per-design
// decisions) besides those of the inner runs.
int bsolve_mixed(mgar_batch* B, double tol, const int* keep_done) {
  const int nd = B->nd;
  const long long N = B->N;
  launch_cast_f32(B->kcur, B->k32, B->E, B->s);
  for (Group& G : B->grp) {
    ItemList& F = G.fine;
    launch_bdot(F.d, F.n(), F.nblk, F.bs, B->qm, B->qm, B->pb, nullptr, 0, B->s);
    launch_bfinalize(F.d, F.n(), B->pb, 1, B->nq, 1, nullptr, nullptr, 0, B->s);
  }
  B->h_odone.assign(nd, 0);
  B->h_iters.assign(nd, 0);
  B->h_nref.assign(nd, 0);
  B->h_conv.assign(nd, 0);
  B->h_rel.assign(nd, NAN);
  if (keep_done) {
    BHIP(hipMemcpyAsync(B->h_odone.data(), keep_done, sizeof(int) * nd, hipMemcpyDeviceToHost, B->s));
    BHIP(hipMemcpyAsync(B->odone, keep_done, sizeof(int) * nd, hipMemcpyDeviceToDevice, B->s));
  } else {
    BHIP(hipMemsetAsync(B->odone, 0, sizeof(int) * nd, B->s));
  }
  std::vector<double> hq(nd), hr(nd);
  std::vector<BCgState> hs(nd);
  for (;;) {
    for (Group& G : B->grp) {
      ItemList& F = G.fine;
      launch_bstencil(G.dim, SM_RESID, F.d, F.n(), F.nblk, F.bs, B->cx, B->kcur, nullptr, B->qm, B->cr, 0.0, nullptr,
                      B->odone, 1, B->s);
      launch_bdot(F.d, F.n(), F.nblk, F.bs, B->cr, B->cr, B->pa, B->odone, 1, B->s);
      launch_bfinalize(F.d, F.n(), B->pa, 1, B->nr, 1, nullptr, B->odone, 1, B->s);
    }
    BLAUNCH();
    BHIP(hipMemcpyAsync(hq.data(), B->nq, sizeof(double) * nd, hipMemcpyDeviceToHost, B->s));
    BHIP(hipMemcpyAsync(hr.data(), B->nr, sizeof(double) * nd, hipMemcpyDeviceToHost, B->s));
    BHIP(hipStreamSynchronize(B->s));
    bool all = true;
    for (int d = 0; d < nd; ++d) {
      if (B->h_odone[d]) continue;
      const double rel = hq[d] > 0.0 ? std::sqrt(hr[d] / hq[d]) : 0.0;
      B->h_rel[d] = rel;
      if (rel <= tol) { B->h_conv[d] = 1; B->h_odone[d] = 1; }
      else if (B->h_iters[d] >= B->cg_max || B->h_nref[d] >= REFINE_MAX) B->h_odone[d] = 1;
      all = all && B->h_odone[d];
    }
    if (all) break;
    // B->h_odone is not written again before the next synchronisation
    BHIP(hipMemcpyAsync(B->odone, B->h_odone.data(), sizeof(int) * nd, hipMemcpyHostToDevice, B->s));
    BHIP(hipMemsetAsync(B->d32, 0, sizeof(float) * N, B->s));
    for (Group& G : B->grp) {
      ItemList& F = G.fine;
      launch_bmask_copy_t<double, float>(F.d, F.n(), F.nblk, F.bs, B->cr, B->r32, B->s);
      launch_bdot_t<float>(F.d, F.n(), F.nblk, F.bs, B->r32, B->r32, B->pa, nullptr, 0, B->s);
      launch_bcg_init(F.d, F.n(), B->st, B->pa, B->pa, B->inner_tol, B->cg_max, B->odone, B->s);
    }
    BLAUNCH();
    BACK(run_until_done(B, 1, B->inner_tol));
    BHIP(hipMemcpyAsync(hs.data(), B->st, sizeof(BCgState) * nd, hipMemcpyDeviceToHost, B->s));
    launch_add_f32(B->cx, B->d32, N, B->s);
    BLAUNCH();
    BHIP(hipStreamSynchronize(B->s));
    for (int d = 0; d < nd; ++d)
      if (!B->h_odone[d]) {
        B->h_iters[d] += hs[d].it;
        B->h_nref[d] += 1;
      }
  }
  return MGAR_OK;
}

int finish(mgar_batch* B, double* T, mgar_stats* stats, int default_path) {
  launch_copy(B->cx, T, B->N, B->s);
  BLAUNCH();
  BHIP(hipEventRecord(B->e1, B->s));
  std::vector<BCgState> hs(B->nd);
  std::vector<int> hp(B->nd, default_path), hstat(B->nd, 0);
  std::vector<double> hr(B->nd, NAN);
  BHIP(hipMemcpyAsync(hs.data(), B->st, sizeof(BCgState) * B->nd, hipMemcpyDeviceToHost, B->s));
  BHIP(hipMemcpyAsync(hstat.data(), B->status, sizeof(int) * B->nd, hipMemcpyDeviceToHost, B->s));
  if (default_path < 0) {
    BHIP(hipMemcpyAsync(hp.data(), B->path, sizeof(int) * B->nd, hipMemcpyDeviceToHost, B->s));
    BHIP(hipMemcpyAsync(hr.data(), B->res, sizeof(double) * B->nd, hipMemcpyDeviceToHost, B->s));
  }
  BHIP(hipStreamSynchronize(B->s));
  float ms = 0.f;
  BHIP(hipEventElapsedTime(&ms, B->e0, B->e1));
  int rc = MGAR_OK;
  for (int i = 0; i < B->nd; ++i) {
    if (hstat[i]) return MGAR_E_NOT_SPD;
    const bool accepted = (hp[i] == MGAR_PATH_ACCEPT);
    const bool conv = B->mixed ? B->h_conv[i] != 0 : hs[i].conv != 0;
    if (!accepted && !conv) rc = MGAR_W_NOT_CONVERGED;
    if (stats) {
      mgar_stats& o = stats[i];
      std::memset(&o, 0, sizeof(o));
      o.path = hp[i];
      o.cg_iters = accepted ? 0 : (B->mixed ? B->h_iters[i] : hs[i].it);
      o.vcycles = (default_path < 0 ? B->m - 1 : 0) + o.cg_iters;
      o.refinements = (accepted || !B->mixed) ? 0 : B->h_nref[i];
      o.res_ca = hr[i];
      o.res_final = accepted ? hr[i]
                    : B->mixed ? B->h_rel[i]
                               : (hs[i].qq > 0.0 ? std::sqrt(hs[i].rr / hs[i].qq) : 0.0);
      o.ms = ms;
    }
  }
  return rc;
}

}  // namespace

extern "C" {

void mgar_batch_destroy(mgar_batch* b) {
  if (!b) return;
  for (int c = 0; c < 2; ++c) {
    if (b->gexec[c]) (void)hipGraphExecDestroy(b->gexec[c]);
    if (b->graph[c]) (void)hipGraphDestroy(b->graph[c]);
  }
  auto f = [](void* p) { if (p) (void)hipFree(p); };
  for (Group& G : b->grp) {
    for (size_t l = 0; l < G.b.size(); ++l) { f(G.b[l]); f(G.xa[l]); f(G.xb[l]); f(G.rt[l]); f(G.k[l]); }
    for (size_t l = 0; l < G.bf.size(); ++l) { f(G.bf[l]); f(G.xaf[l]); f(G.xbf[l]); f(G.rtf[l]); f(G.kf[l]); }
    for (auto* v : {&G.down, &G.restr, &G.prol, &G.coarsen})
      for (ItemList& L : *v) f(L.d);
    f(G.fine.d); f(G.cells.d); f(G.tails); f(G.cb_reg); f(G.cb_gen);
  }
  for (void* p : {(void*)b->kcur, (void*)b->k0, (void*)b->qm, (void*)b->cx, (void*)b->cr, (void*)b->cz,
                  (void*)b->cp, (void*)b->cw, (void*)b->xa0, (void*)b->rt0, (void*)b->R, (void*)b->Wm,
                  (void*)b->Ainv, (void*)b->pa, (void*)b->pb, (void*)b->pc, (void*)b->st, (void*)b->md,
                  (void*)b->keep, (void*)b->path, (void*)b->status, (void*)b->res, (void*)b->nrm,
                  (void*)b->dens, (void*)b->dens0, (void*)b->k32, (void*)b->r32, (void*)b->z32, (void*)b->p32,
                  (void*)b->w32, (void*)b->d32, (void*)b->xa32, (void*)b->rt32, (void*)b->odone, (void*)b->nq,
                  (void*)b->nr})
    f(p);
  if (b->e0) (void)hipEventDestroy(b->e0);
  if (b->e1) (void)hipEventDestroy(b->e1);
  if (b->ein) (void)hipEventDestroy(b->ein);
  if (b->own_stream && b->s) (void)hipStreamDestroy(b->s);
  delete b;
}

// (Re)build the work lists of every group for blocks of bs threads (one
// node, element or coarse node per thread); captured iterations refer to the
// old lists and are dropped.
static int build_lists(mgar_batch* B, int bs) {
  auto f = [](void* p) { if (p) (void)hipFree(p); };
  for (int c = 0; c < 2; ++c) {
    if (B->gexec[c]) { (void)hipGraphExecDestroy(B->gexec[c]); B->gexec[c] = nullptr; }
    if (B->graph[c]) { (void)hipGraphDestroy(B->graph[c]); B->graph[c] = nullptr; }
    B->tol_captured[c] = -1.0;
  }
  for (Group& G : B->grp) {
    for (auto* v : {&G.down, &G.restr, &G.prol, &G.coarsen})
      for (ItemList& L : *v) f(L.d);
    f(G.fine.d);
    f(G.cells.d);
    G.fine = ItemList();
    G.cells = ItemList();
    G.down.assign(G.maxL, ItemList());
    G.restr.assign(G.maxL, ItemList());
    G.prol.assign(G.maxL, ItemList());
    G.coarsen.assign(G.maxL, ItemList());
    for (int i : G.designs) {
      Design& D = B->d[i];
      const Geo& g0 = D.g[0];
      G.fine.h.push_back(make_item(g0, g0, D.noff, 0, D.eoff, 0, i, batch_item_blocks(g0, bs)));
      G.cells.h.push_back(make_item(g0, g0, D.noff, 0, D.eoff, 0, i, blocks_of(g0.ne, bs)));
      for (int l = 0; l < D.L; ++l) {
        const long long off = (l == 0) ? D.noff : D.aoff[l];
        const long long eo = (l == 0) ? D.eoff : D.aeoff[l];
        if (l < D.lt) {
          const Geo &gf = D.g[l], &gc = D.g[l + 1];
          G.down[l].h.push_back(make_item(gf, gf, off, 0, eo, 0, i, batch_item_blocks(gf, bs)));
          G.restr[l].h.push_back(make_item(gf, gc, off, D.aoff[l + 1], eo, D.aeoff[l + 1], i,
                                           batch_item_blocks(gc, bs)));
          G.prol[l].h.push_back(make_item(gf, gc, off, D.aoff[l + 1], eo, D.aeoff[l + 1], i,
                                          batch_item_blocks(gc, bs)));
        }
        if (l + 1 < D.L) {
          const Geo &gf = D.g[l], &gc = D.g[l + 1];
          G.coarsen[l].h.push_back(make_item(gf, gc, off, D.aoff[l + 1], eo, D.aeoff[l + 1], i,
                                             blocks_of(gc.ne, bs)));
        }
      }
    }
    G.fine.bs = G.cells.bs = bs;
    BACK(upload(G.fine));
    BACK(upload(G.cells));
    for (int l = 0; l < G.maxL; ++l) {
      for (ItemList* L : {&G.down[l], &G.restr[l], &G.prol[l], &G.coarsen[l]}) {
        L->bs = bs;
        BACK(upload(*L));
      }
    }
  }
  B->bs = bs;
  return MGAR_OK;
}

static int batch_setup_impl(const mgar_params* p, int nd, void* stream, mgar_batch* B) {
  B->nd = nd;
  B->user_s = (hipStream_t)stream;
  if (B->user_s) {
    B->s = B->user_s;
  } else {
    BHIP(hipStreamCreateWithFlags(&B->s, hipStreamNonBlocking));
    B->own_stream = true;
  }
  B->m = p[0].n_basis;
  B->omega = p[0].omega;
  B->eps = p[0].eps_accept;
  B->cg_max = p[0].cg_max;
  B->basis_x0_zero = p[0].basis_x0_zero;
  B->mixed = p[0].precision == MGAR_PREC_MIXED;
  B->inner_tol = p[0].inner_tol;
  B->kmin_f = (float)p[0].kmin;
  B->kdiff_f = (float)(p[0].k0 - p[0].kmin);
  const size_t esz = B->mixed ? sizeof(float) : sizeof(double);   // multigrid value type
  B->d.resize(nd);
  for (int i = 0; i < nd; ++i) {
    BACK(mgar_internal_validate(&p[i]));
    if (p[i].precision != MGAR_PREC_FP64 && p[i].precision != MGAR_PREC_MIXED) return MGAR_E_PRECISION;
    if (p[i].precision == MGAR_PREC_MIXED && p[i].penal != 3.0) return MGAR_E_PRECISION;
    if (p[i].levels < 2) return MGAR_E_DIMS;
    if (p[i].n_basis != B->m || p[i].omega != B->omega || p[i].eps_accept != B->eps ||
        p[i].cg_max != B->cg_max || p[i].basis_x0_zero != B->basis_x0_zero ||
        p[i].precision != p[0].precision || p[i].k0 != p[0].k0 || p[i].kmin != p[0].kmin ||
        p[i].penal != p[0].penal)
      return MGAR_E_ARG;
    if (B->mixed && (p[i].inner_tol != B->inner_tol || !(B->inner_tol > 0.0 && B->inner_tol < 1.0)))
      return MGAR_E_ARG;
    Design& D = B->d[i];
    D.p = p[i];
    if (D.p.dim == 2) { D.p.nelz = 0; D.p.fix_lo[2] = 0; D.p.fix_hi[2] = 0; }
    D.L = D.p.levels;
    for (int l = 0; l < D.L; ++l) D.g.push_back(mgar_internal_geo(D.p, l));
    const Geo& gc = D.g[D.L - 1];
    if (gc.nn > 1024) return MGAR_E_DIMS;
    if (mgar_internal_count_fixed(gc) == 0) return MGAR_E_SINGULAR;
    if (D.g[0].nn * 8 >= (1LL << 31)) return MGAR_E_DIMS;
    D.noff = B->N;
    D.eoff = B->E;
    B->N += D.g[0].nn;
    B->E += D.g[0].ne;
    D.Aoff = B->Atot;
    B->Atot += gc.nn * gc.nn;
  }
  // groups by dimension
  for (int dim = 2; dim <= 3; ++dim) {
    Group G;
    G.dim = dim;
    for (int i = 0; i < nd; ++i)
      if (B->d[i].p.dim == dim) G.designs.push_back(i);
    if (G.designs.empty()) continue;
    for (int i : G.designs) G.maxL = std::max(G.maxL, B->d[i].L);
    G.b.assign(G.maxL, nullptr);
    G.xa.assign(G.maxL, nullptr);
    G.xb.assign(G.maxL, nullptr);
    G.rt.assign(G.maxL, nullptr);
    G.k.assign(G.maxL, nullptr);
    G.bf.assign(G.maxL, nullptr);
    G.xaf.assign(G.maxL, nullptr);
    G.xbf.assign(G.maxL, nullptr);
    G.rtf.assign(G.maxL, nullptr);
    G.kf.assign(G.maxL, nullptr);
    // arenas of grids >= 1
    for (int l = 1; l < G.maxL; ++l) {
      long long nn = 0, ne = 0;
      for (int i : G.designs) {
        Design& D = B->d[i];
        D.aoff.resize(D.L, 0);
        D.aeoff.resize(D.L, 0);
        if (l < D.L) {
          D.aoff[l] = nn;
          D.aeoff[l] = ne;
          nn += D.g[l].nn;
          ne += D.g[l].ne;
        }
      }
      if (B->mixed) {
        BACK(dalloc(&G.bf[l], nn));
        BACK(dalloc(&G.xaf[l], nn));
        BACK(dalloc(&G.xbf[l], nn));
        BACK(dalloc(&G.rtf[l], nn));
        BACK(dalloc(&G.kf[l], ne));
      } else {
        BACK(dalloc(&G.b[l], nn));
        BACK(dalloc(&G.xa[l], nn));
        BACK(dalloc(&G.xb[l], nn));
        BACK(dalloc(&G.rt[l], nn));
        BACK(dalloc(&G.k[l], ne));
      }
    }
    B->grp.push_back(G);
  }
  // tail level of every design (same rule as a single handle)
  for (Group& G : B->grp) {
    std::vector<BTail> tails;
    std::vector<BCoarse> creg, cgen;
    for (int i : G.designs) {
      Design& D = B->d[i];
      std::vector<const void*> ks(D.L, nullptr);
      ks[0] = nullptr;
      for (int l = 1; l < D.L; ++l)
        ks[l] = B->mixed ? (const void*)(G.kf[l] + D.aeoff[l]) : (const void*)(G.k[l] + D.aeoff[l]);
      TailSpec T;
      D.lt = -1;
      for (int lt = 1; lt < D.L; ++lt)
        if (tail_plan(D.g.data(), ks.data(), lt, D.L, esz, &T)) { D.lt = lt; break; }
      if (D.lt < 0) return MGAR_E_DIMS;
      BTail bt;
      std::memset(&bt, 0, sizeof(bt));
      (void)tail_plan(D.g.data(), ks.data(), D.lt, D.L, esz, &bt.ts);
      if (B->mixed) {
        bt.bin = G.bf[D.lt] + D.aoff[D.lt];
        bt.xout = G.xbf[D.lt] + D.aoff[D.lt];
      } else {
        bt.bin = G.b[D.lt] + D.aoff[D.lt];
        bt.xout = G.xb[D.lt] + D.aoff[D.lt];
      }
      bt.design = i;
      tails.push_back(bt);
      G.tail_lds = std::max(G.tail_lds, bt.ts.lds_elems);
      G.maxlt = std::max(G.maxlt, D.lt);
      BCoarse c;
      std::memset(&c, 0, sizeof(c));
      c.g = D.g[D.L - 1];
      c.k = B->mixed ? (const void*)(G.kf[D.L - 1] + D.aeoff[D.L - 1])
                     : (const void*)(G.k[D.L - 1] + D.aeoff[D.L - 1]);
      c.design = i;
      (c.g.nn <= 128 ? creg : cgen).push_back(c);
    }
    // Ainv pointers once allocated below
    G.ntails = (int)tails.size();
    BACK(dalloc(&G.tails, G.ntails));
    // patch A pointers after Ainv exists
    if (!B->Ainv) BACK(dalloc(&B->Ainv, B->Atot));
    for (BTail& t : tails) t.A = B->Ainv + B->d[t.design].Aoff;
    for (BCoarse& c : creg) c.A = B->Ainv + B->d[c.design].Aoff;
    for (BCoarse& c : cgen) c.A = B->Ainv + B->d[c.design].Aoff;
    BHIP(hipMemcpy(G.tails, tails.data(), sizeof(BTail) * tails.size(), hipMemcpyHostToDevice));
    G.n_reg = (int)creg.size();
    G.n_gen = (int)cgen.size();
    BACK(dalloc(&G.cb_reg, G.n_reg));
    BACK(dalloc(&G.cb_gen, G.n_gen));
    if (G.n_reg) BHIP(hipMemcpy(G.cb_reg, creg.data(), sizeof(BCoarse) * creg.size(), hipMemcpyHostToDevice));
    if (G.n_gen) BHIP(hipMemcpy(G.cb_gen, cgen.data(), sizeof(BCoarse) * cgen.size(), hipMemcpyHostToDevice));
    if ((size_t)G.tail_lds * esz > 64 * 1024) return MGAR_E_DIMS;
  }
  BACK(build_lists(B, 256));
  // finest-grid workspace
  const long long N = B->N, E = B->E;
  BACK(dalloc(&B->kcur, E));
  BACK(dalloc(&B->k0, E));
  for (double** v : {&B->qm, &B->cx, &B->cr, &B->cz, &B->cp, &B->cw}) BACK(dalloc(v, N));
  if (!B->mixed)
    for (double** v : {&B->xa0, &B->rt0}) BACK(dalloc(v, N));
  BACK(dalloc(&B->R, N * B->m));
  BACK(dalloc(&B->Wm, N * B->m));
  // block partials: sized for the smallest block size a list may be built with
  long long nb = 0;
  for (Group& G : B->grp) {
    long long n = 0;
    for (int i : G.designs) n += batch_item_blocks(B->d[i].g[0], BATCH_MIN_BS);
    nb = std::max(nb, n);
  }
  const long long nv = (long long)B->m * (B->m + 1) / 2 + B->m;
  BACK(dalloc(&B->pa, nb * std::max<long long>(nv, 8)));
  BACK(dalloc(&B->pb, nb * std::max<long long>(nv, 8)));
  BACK(dalloc(&B->pc, nb * std::max<long long>(nv, 8)));
  BACK(dalloc(&B->st, nd));
  BACK(dalloc(&B->md, nd));
  BACK(dalloc(&B->keep, nd));
  BACK(dalloc(&B->path, nd));
  BACK(dalloc(&B->status, nd));
  BACK(dalloc(&B->res, nd));
  BACK(dalloc(&B->nrm, nd));
  if (B->mixed) {
    BACK(dalloc(&B->dens, E));
    BACK(dalloc(&B->dens0, E));
    BACK(dalloc(&B->k32, E));
    for (float** v : {&B->r32, &B->z32, &B->p32, &B->w32, &B->d32, &B->xa32, &B->rt32}) BACK(dalloc(v, N));
    BACK(dalloc(&B->odone, nd));
    BACK(dalloc(&B->nq, nd));
    BACK(dalloc(&B->nr, nd));
  }
  BHIP(hipMemset(B->st, 0, sizeof(BCgState) * nd));
  BHIP(hipMemset(B->md, 0, sizeof(MgarDev) * nd));
  BHIP(hipMemset(B->status, 0, sizeof(int) * nd));
  BHIP(hipMemset(B->keep, 0, sizeof(int) * nd));
  BHIP(hipEventCreate(&B->e0));
  BHIP(hipEventCreate(&B->e1));
  BHIP(hipEventCreateWithFlags(&B->ein, hipEventDisableTiming));
  return MGAR_OK;
}

// Order the batch's own stream after the caller's (NULL) stream.
static int enter(mgar_batch* b) {
  if (!b->own_stream) return MGAR_OK;
  BHIP(hipEventRecord(b->ein, b->user_s));
  BHIP(hipStreamWaitEvent(b->s, b->ein, 0));
  return MGAR_OK;
}

int mgar_batch_setup(const mgar_params* p, int ndesigns, void* stream, mgar_batch** out) {
  if (!p || !out || ndesigns < 1) return MGAR_E_ARG;
  *out = nullptr;
  mgar_batch* B = new mgar_batch();
  const int rc = batch_setup_impl(p, ndesigns, stream, B);
  if (rc != MGAR_OK) {
    mgar_batch_destroy(B);
    return rc;
  }
  *out = B;
  return MGAR_OK;
}

int mgar_batch_layout(const mgar_batch* b, long long* node_off, long long* elem_off) {
  if (!b || !node_off || !elem_off) return MGAR_E_ARG;
  for (int i = 0; i < b->nd; ++i) {
    node_off[i] = b->d[i].noff;
    elem_off[i] = b->d[i].eoff;
  }
  node_off[b->nd] = b->N;
  elem_off[b->nd] = b->E;
  return MGAR_OK;
}

int mgar_batch_set_graph(mgar_batch* b, int use_graph) {
  if (!b) return MGAR_E_ARG;
  b->use_graph = use_graph != 0;
  return MGAR_OK;
}

int mgar_batch_set_block(mgar_batch* b, int bs) {
  if (!b || (bs != 64 && bs != 128 && bs != 256)) return MGAR_E_ARG;
  if (bs == b->bs) return MGAR_OK;
  BHIP(hipStreamSynchronize(b->s));   // queued work reads the lists being replaced
  return build_lists(b, bs);
}

int mgar_batch_get_block(const mgar_batch* b, int* bs) {
  if (!b || !bs) return MGAR_E_ARG;
  *bs = b->bs;
  return MGAR_OK;
}

int mgar_batch_autotune(mgar_batch* b, const double* xphys, const double* q, double tol, int reps, int* bs_out,
                        float* us_out) {
  if (!b || !xphys || !q || reps < 1) return MGAR_E_ARG;
  static const int cand[3] = {256, 128, 64};
  double* T = nullptr;
  BHIP(hipMalloc((void**)&T, sizeof(double) * (size_t)b->N));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = MGAR_OK;
  int best = 256;
  float best_ms = -1.0f;
  auto run = [&]() -> int {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MGAR_E_HIP;
    for (int c = 0; c < 3; ++c) {
      BACK(mgar_batch_set_block(b, cand[c]));
      const int w = mgcg_batch_solve(b, xphys, q, nullptr, tol, T, nullptr);   // warm-up and graph capture
      if (w < 0) return w;
      BHIP(hipEventRecord(e0, b->s));
      for (int r = 0; r < reps; ++r) {
        const int rr = mgcg_batch_solve(b, xphys, q, nullptr, tol, T, nullptr);
        if (rr < 0) return rr;
      }
      BHIP(hipEventRecord(e1, b->s));
      BHIP(hipEventSynchronize(e1));
      float ms = 0.f;
      BHIP(hipEventElapsedTime(&ms, e0, e1));
      ms /= (float)reps;
      if (us_out) us_out[c] = 1e3f * ms;
      if (best_ms < 0.f || ms < best_ms) { best_ms = ms; best = cand[c]; }
    }
    return mgar_batch_set_block(b, best);
  };
  rc = run();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(T);
  if (rc == MGAR_OK && bs_out) *bs_out = best;
  return rc;
}

int mgar_batch_load_vector(mgar_batch* b, const double* Qe, double* q) {
  if (!b || !Qe || !q) return MGAR_E_ARG;
  BACK(enter(b));
  for (const Design& D : b->d) launch_load(D.g[0], Qe + D.eoff, q + D.noff, b->s);
  BLAUNCH();
  BHIP(hipStreamSynchronize(b->s));
  return MGAR_OK;
}

int mgcg_batch_solve(mgar_batch* b, const double* xphys, const double* q, const double* T0, double tol,
                     double* T, mgar_stats* stats) {
  if (!b || !xphys || !q || !T) return MGAR_E_ARG;
  BACK(enter(b));
  BHIP(hipEventRecord(b->e0, b->s));
  const mgar_params& p0 = b->d[0].p;
  launch_simp(xphys, b->kcur, b->E, p0.k0, p0.kmin, p0.penal, b->s);
  if (b->mixed) launch_cast_bf16(xphys, b->dens, b->E, b->s);
  BHIP(hipMemsetAsync(b->status, 0, sizeof(int) * b->nd, b->s));
  for (Group& G : b->grp) {
    BACK(b->mixed ? bbuild32(b, G, nullptr) : bbuild(b, G, nullptr));
    launch_bmask_copy(G.fine.d, G.fine.n(), G.fine.nblk, G.fine.bs, q, b->qm, b->s);
    if (T0) launch_bmask_copy(G.fine.d, G.fine.n(), G.fine.nblk, G.fine.bs, T0, b->cx, b->s);
  }
  if (!T0) BHIP(hipMemsetAsync(b->cx, 0, sizeof(double) * b->N, b->s));
  BLAUNCH();
  BACK(b->mixed ? bsolve_mixed(b, tol, nullptr) : bpcg(b, tol, nullptr));
  b->has_k0 = true;
  return finish(b, T, stats, MGAR_PATH_MGCG);
}

int mgar_batch_solve(mgar_batch* b, const double* xphys, const double* q, const double* T0, double tol,
                     double* T, mgar_stats* stats) {
  if (!b || !xphys || !q || !T) return MGAR_E_ARG;
  if (!b->has_k0) return MGAR_E_STATE;
  BACK(enter(b));
  BHIP(hipEventRecord(b->e0, b->s));
  const mgar_params& p0 = b->d[0].p;
  const long long N = b->N;
  const int m = b->m;
  const int mds = MD_STRIDE;
  double* mdd = reinterpret_cast<double*>(b->md);
  launch_simp(xphys, b->kcur, b->E, p0.k0, p0.kmin, p0.penal, b->s);
  if (b->mixed) launch_cast_bf16(xphys, b->dens, b->E, b->s);
  BHIP(hipMemsetAsync(b->status, 0, sizeof(int) * b->nd, b->s));
  for (Group& G : b->grp) {
    ItemList& F = G.fine;
    launch_bmask_copy(F.d, F.n(), F.nblk, F.bs, q, b->qm, b->s);
    // r_1 = t_prev, r_i = MG(K0, -dK r_{i-1}, x0) (Eq 17)
    if (T0) launch_bmask_copy(F.d, F.n(), F.nblk, F.bs, T0, b->R, b->s);
    else BHIP(hipMemsetAsync(b->R, 0, sizeof(double) * N, b->s));
    for (int i = 1; i < m; ++i) {
      const double* prev = b->R + (long long)(i - 1) * N;
      launch_bstencil(G.dim, SM_NEG_DK, F.d, F.n(), F.nblk, F.bs, prev, b->kcur, b->k0, nullptr, b->cz, 0.0,
                      nullptr, nullptr, 0, b->s);
      if (b->mixed) {
        // -dK r in FP64 (a difference of nearby operators), one FP32 V-cycle
        // on the BF16 K0 hierarchy, the column kept in FP64
        launch_bmask_copy_t<double, float>(F.d, F.n(), F.nblk, F.bs, b->cz, b->z32, b->s);
        if (!b->basis_x0_zero) launch_bmask_copy_t<double, float>(F.d, F.n(), F.nblk, F.bs, prev, b->p32, b->s);
        BACK(bvcycle32(b, G, b->z32, b->basis_x0_zero ? nullptr : b->p32, b->w32, nullptr, nullptr));
        launch_bmask_copy_t<float, double>(F.d, F.n(), F.nblk, F.bs, b->w32, b->R + (long long)i * N, b->s);
      } else {
        BACK(bvcycle(b, G, b->cz, b->basis_x0_zero ? nullptr : prev, b->R + (long long)i * N, nullptr,
                     nullptr));
      }
    }
    // Gram-Schmidt applied twice per column (same rule as the single path)
    for (int j = 0; j < m; ++j) {
      double* v = b->R + (long long)j * N;
      launch_bdot(F.d, F.n(), F.nblk, F.bs, v, v, b->pa, nullptr, 0, b->s);
      launch_bfinalize(F.d, F.n(), b->pa, 1, mdd + offsetof(MgarDev, n0) / sizeof(double) + j, mds, nullptr,
                       nullptr, 0, b->s);
      if (j > 0) {
        for (int pass = 0; pass < 2; ++pass) {
          launch_bmultidot(F.d, F.n(), F.nblk, F.bs, b->R, N, j, v, b->pa, b->s);
          launch_bfinalize(F.d, F.n(), b->pa, j, mdd + offsetof(MgarDev, c) / sizeof(double), mds, nullptr,
                           nullptr, 0, b->s);
          launch_bgs_update(F.d, F.n(), F.nblk, F.bs, v, b->R, N, j, b->md, b->s);
        }
      }
      launch_bdot(F.d, F.n(), F.nblk, F.bs, v, v, b->pa, nullptr, 0, b->s);
      launch_bfinalize(F.d, F.n(), b->pa, 1, b->nrm, 1, nullptr, nullptr, 0, b->s);
      launch_bgs_normalize(F.d, F.n(), F.nblk, F.bs, v, b->md, j, b->nrm, 1, b->s);
    }
    // Eq 19-21 and Eq 28
    for (int j = 0; j < m; ++j)
      launch_bstencil(G.dim, SM_APPLY, F.d, F.n(), F.nblk, F.bs, b->R + (long long)j * N, b->kcur, nullptr, nullptr,
                      b->Wm + (long long)j * N, 0.0, nullptr, nullptr, 0, b->s);
    launch_bgram(F.d, F.n(), F.nblk, F.bs, b->R, b->Wm, b->qm, N, m, b->pa, b->s);
    launch_bgram_finalize(F.d, F.n(), b->pa, m, b->md, b->s);
    launch_bcombine(F.d, F.n(), F.nblk, F.bs, b->R, b->Wm, b->qm, N, m, b->md, b->cx, b->pa, b->s);
    launch_bfinalize(F.d, F.n(), b->pa, 1, mdd + offsetof(MgarDev, res2) / sizeof(double), mds, nullptr,
                     nullptr, 0, b->s);
    launch_bdot(F.d, F.n(), F.nblk, F.bs, b->qm, b->qm, b->pb, nullptr, 0, b->s);
    launch_bfinalize(F.d, F.n(), b->pb, 1, mdd + offsetof(MgarDev, qq) / sizeof(double), mds, nullptr,
                     nullptr, 0, b->s);
    launch_bdecide(F.d, F.n(), b->md, b->st, b->eps, b->keep, b->path, b->res, b->s);
    // rejected designs: K becomes the new K0, MGCG from the reduced solution
    BACK(b->mixed ? bbuild32(b, G, b->keep) : bbuild(b, G, b->keep));
  }
  BLAUNCH();
  BACK(b->mixed ? bsolve_mixed(b, tol, b->keep) : bpcg(b, tol, b->keep));
  return finish(b, T, stats, -1);
}

}  // extern "C"
