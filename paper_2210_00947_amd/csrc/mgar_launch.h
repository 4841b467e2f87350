// Host-side launch wrappers of the libmgar kernels (one definition per .hip file).
#pragma once
#include "mgar_common.h"
#include "mgar.h"

// Matrix-free stencil modes (y = K_l x with the rediscretised Q1 operator).
enum StencilMode {
  SM_APPLY = 0,      // out = K x
  SM_APPLY_DOT = 1,  // out = K x;            partial += x . out
  SM_RESID = 2,      // out = b - K x
  SM_JACOBI = 3,     // out = x + w D^-1 (b - K x)
  SM_JACOBI_DOT = 4, // as SM_JACOBI;         partial += b . out
  SM_JACOBI0 = 5,    // out = w D^-1 b        (sweep from a zero guess; x unused)
  SM_NEG_DK = 6,     // out = -(K(k) - K(kref)) x
  // CG direction update fused into the apply (two-row z-marching shapes only,
  // FP64): p = z + beta p_old with beta = rz_it / rz_(it-1) (0 at it = 0), rz_it
  // summed from its block partials; p is stored, out = K p, partial += p . out.
  // Launched by launch_papply_dot; tuned with the shape of SM_APPLY_DOT.
  SM_PAPPLY_DOT = 7,
  // First V-cycle sweep fused into the residual (two-row z-marching shapes
  // only, FP64): x = w b / diag(K) is formed where staged (diag precomputed),
  // stored to xout, and out = b - K x. Launched by launch_j0resid; tuned with
  // the shape of SM_RESID.
  SM_J0RESID = 8,
};

// Extra operands of the fused modes.
// SM_PAPPLY_DOT: the direction is double-buffered by iteration parity (p_old in
// pbuf[(it + 1) & 1], p written to pbuf[it & 1]): neighbouring blocks read
// p_old in their halo while this block writes p.
// SM_J0RESID: diag = diagonal of K per node, xout receives the sweep.
// Vectors are of the kernel's value type (double or float).
// SM_J0RESID with chk set also applies the stopping test of the previous CG
// iteration first (as launch_cg_check: rzp/nrz then hold the ||r||^2 partials
// of the x/r update); every block takes the same decision and returns if it
// fires, block 0 advances st.
struct PFuse {
  CgState* st;          // it, rz history; st->rz[it & 1] is stored by block 0
  const double* rzp;    // block partials of r . z of this iteration
  int nrz;
  int chk;
  void* pbuf[2];
  const void* diag;
  void* xout;
  double tol;
  int cg_max;
  int pad;
};

// stencil.hip ----------------------------------------------------------------
// Launch shape of a stencil on one grid. kind 0: node-parallel kernel (one
// thread per node, 64x4 blocks). kind 1: z-marching kernel (3D only): the node
// grid is cut into ntx x nty column tiles of width ceil(nnx/ntx) <= 64 and
// height filling 256 threads, and into z-chunks of kz node planes; each block
// marches one chunk with a load queue zd planes deep (1 to 4). kind 2: as
// kind 1 with two node rows per thread (tile width <= 128, an even tile
// height, zd 1 or 2). The arithmetic
// of every node is the same for every shape; only the order in which block
// partials of a dot are summed depends on it.
struct StencilCfg {
  int kind, kz, zd, ntx;
};
StencilCfg stencil_default_cfg(const Geo& g);
bool stencil_cfg_valid(const Geo& g, const StencilCfg& c);
// Candidate shapes for the tuner (the default first); returns how many were
// written (at most `cap`; STENCIL_MAX_CANDIDATES holds them all).
constexpr int STENCIL_MAX_CANDIDATES = 128;
int stencil_candidates(const Geo& g, StencilCfg* out, int cap);
// Value type T (double or float) and cell loader CL (CellD, CellF, CellB) are
// template parameters; FP64 entry points keep plain-pointer overloads. cfg
// null = stencil_default_cfg(g).
template <typename T, typename CL>
int launch_stencil_t(const Geo& g, int mode, const T* x, CL k, CL kref, const T* b, T* out,
                     double omega, double* part, const int* done, hipStream_t s,
                     unsigned* cnt = nullptr, double* rout = nullptr, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr, const StencilCfg* cfg = nullptr);
// Returns the number of block partials written to `part` (0 for modes without a
// dot). With cnt != null the dot is also reduced in the same launch (last block
// sums the partials in order) and stored to *rout. ev0/ev1 (may be null):
// events recorded at the start and end of the kernel itself.
int launch_stencil(const Geo& g, int mode, const double* x, const double* k, const double* kref,
                   const double* b, double* out, double omega, double* part, const int* done,
                   hipStream_t s, unsigned* cnt = nullptr, double* rout = nullptr,
                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                   const StencilCfg* cfg = nullptr);
bool stencil_records_events(const Geo& g, const StencilCfg* cfg = nullptr);
// SM_PAPPLY_DOT on grid g with launch shape cfg: returns the number of block
// partials of p . out written to part, or -1 (nothing launched) when cfg is not
// a two-row z-marching shape (then p is updated and applied by separate launches).
// Whether launch_papply_dot_t runs the fused kernel for this grid and shape.
bool papply_supported(const Geo& g, const StencilCfg* cfg);
// Instantiated for (double, CellD) and (float, CellF).
template <typename T, typename CL>
int launch_papply_dot_t(const Geo& g, const T* z, CL k, T* out, double* part, const int* done,
                        hipStream_t s, const PFuse& pf, const StencilCfg* cfg, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
inline int launch_papply_dot(const Geo& g, const double* z, const double* k, double* out, double* part,
                             const int* done, hipStream_t s, const PFuse& pf, const StencilCfg* cfg,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  return launch_papply_dot_t<double, CellD>(g, z, CellD{k}, out, part, done, s, pf, cfg, ev0, ev1);
}
// SM_J0RESID on grid g (3D) with launch shape cfg (its queue depth is always 1):
// xout = w b / diag, out = b - K xout. Returns false (nothing launched) when cfg
// is not a two-row z-marching shape. Instantiated for (double, CellD) and
// (float, CellB).
// check (optional, FP64 only): the fused stopping test (PFuse::chk); done is
// then not read.
template <typename T, typename CL>
bool launch_j0resid_t(const Geo& g, const T* b, CL k, const T* diag, T* xout, T* out, double omega,
                      const int* done, hipStream_t s, const StencilCfg* cfg, const PFuse* check = nullptr);
inline bool launch_j0resid(const Geo& g, const double* b, const double* k, const double* diag, double* xout,
                           double* out, double omega, const int* done, hipStream_t s, const StencilCfg* cfg,
                           const PFuse* check = nullptr) {
  return launch_j0resid_t<double, CellD>(g, b, CellD{k}, diag, xout, out, omega, done, s, cfg, check);
}
// diag[n] = diagonal of K at node n (h/3 times the sum of its cells, summed in the
// order of the node formula, in the value type), 3D. Instantiated for
// (double, CellD) and (float, CellB).
template <typename T, typename CL>
void launch_diag_t(const Geo& g, CL k, T* diag, hipStream_t s);
inline void launch_diag(const Geo& g, const double* k, double* diag, hipStream_t s) {
  launch_diag_t<double, CellD>(g, CellD{k}, diag, s);
}
int stencil_num_partials(const Geo& g, const StencilCfg* cfg = nullptr);
template <typename T>
void launch_restrict_t(const Geo& gf, const Geo& gc, const T* rf, T* rc, const int* done, hipStream_t s);
// Restriction rf -> bc, then the coarse grid's sweep from zero bc -> xc with
// cells kc (one launch). Returns false, launching nothing, when a grid is too
// large for 32-bit buffer offsets (use the two separate launches then).
template <typename T, typename CL>
bool launch_restrict_j0_t(const Geo& gf, const Geo& gc, const T* rf, CL kc, T* bc, T* xc, double omega,
                          const int* done, hipStream_t s);
template <typename T>
void launch_prolong_t(const Geo& gf, const Geo& gc, const T* xc, T* xf, const int* done, hipStream_t s);
// Interpolation xpre + P xc then one Jacobi sweep on grid gf (cells k, right
// side b) into out, in one node-parallel launch; xpre is not written. Equal to
// launch_prolong_t followed by the stencil's Jacobi mode. Returns false
// (nothing launched) for grids too large for 32-bit buffer offsets.
// Instantiated for (double, CellD) and (float, CellF).
template <typename T, typename CL>
bool launch_prolong_jacobi_t(const Geo& gf, const Geo& gc, const T* xc, const T* xpre, CL k, const T* b,
                             T* out, double omega, const int* done, hipStream_t s);
template <typename CL, typename TO>
void launch_coarsen_t(const Geo& gf, const Geo& gc, CL kf, TO* kc, hipStream_t s);
template <typename CL>
void launch_coarse_build_t(const Geo& g, CL k, double* A, int* status, hipStream_t s);
template <typename T>
void launch_coarse_solve_t(const Geo& g, const double* A, const T* b, T* x, const int* done,
                           hipStream_t s);
template <typename TI, typename TO>
void launch_mask_copy_t(const Geo& g, const TI* in, TO* out, hipStream_t s);

inline void launch_restrict(const Geo& gf, const Geo& gc, const double* rf, double* rc,
                            const int* done, hipStream_t s) {
  launch_restrict_t<double>(gf, gc, rf, rc, done, s);
}
inline void launch_prolong(const Geo& gf, const Geo& gc, const double* xc, double* xf,
                           const int* done, hipStream_t s) {
  launch_prolong_t<double>(gf, gc, xc, xf, done, s);
}
inline void launch_coarsen(const Geo& gf, const Geo& gc, const double* kf, double* kc, hipStream_t s) {
  launch_coarsen_t<CellD, double>(gf, gc, CellD{kf}, kc, s);
}
inline void launch_coarse_build(const Geo& g, const double* k, double* A, int* status, hipStream_t s) {
  launch_coarse_build_t<CellD>(g, CellD{k}, A, status, s);
}
inline void launch_coarse_solve(const Geo& g, const double* A, const double* b, double* x,
                                const int* done, hipStream_t s) {
  launch_coarse_solve_t<double>(g, A, b, x, done, s);
}
inline void launch_mask_copy(const Geo& g, const double* in, double* out, hipStream_t s) {
  launch_mask_copy_t<double, double>(g, in, out, s);
}

// Bottom of the V-cycle in one workgroup: grids lt..L-1 of a hierarchy with
// their vectors in LDS. b_in: right-hand side on grid lt; x_out: the V-cycle
// result on grid lt.
#define MGAR_MAX_TAIL 8
struct TailSpec {
  int nl;                          // grids in the tail (>= 1); the last is the coarsest
  int lds_elems;                   // LDS footprint in values
  int elem;                        // bytes per value
  Geo g[MGAR_MAX_TAIL];
  const void* k[MGAR_MAX_TAIL];    // cell conductivities (global memory, value type)
  int off_b[MGAR_MAX_TAIL], off_xa[MGAR_MAX_TAIL], off_xb[MGAR_MAX_TAIL], off_k[MGAR_MAX_TAIL];
};
// Fills the LDS layout; returns false if grids lt.. do not fit.
bool tail_plan(const Geo* g, const void* const* k, int lt, int L, size_t elem, TailSpec* T);
template <typename T>
void launch_vtail_t(const TailSpec& TS, const T* b_in, T* x_out, const double* Ainv, double omega,
                    const int* done, hipStream_t s);
inline void launch_vtail(const TailSpec& TS, const double* b_in, double* x_out, const double* Ainv,
                         double omega, const int* done, hipStream_t s) {
  launch_vtail_t<double>(TS, b_in, x_out, Ainv, omega, done, s);
}

// vec.hip --------------------------------------------------------------------
int vec_num_blocks(long long n);
// partial[b] = sum over block b of a.b ; returns number of partials
int launch_dot(const double* a, const double* b, long long n, double* part, const int* done,
               hipStream_t s, unsigned* cnt = nullptr, double* rout = nullptr);
template <typename TA, typename TB>
int launch_dot_t(const TA* a, const TB* b, long long n, double* part, const int* done, hipStream_t s,
                 unsigned* cnt = nullptr, double* rout = nullptr);
// The CG kernels take the iteration index from st->it (advanced by
// launch_cg_check), never from the host. rzp / pwp (optional): block partials
// of r.z / p.w, summed inside the update (in place of a separate finalize
// launch) and stored to st->rz[st->it & 1] / st->pw.
template <typename T>
void launch_p_update_t(const T* z, T* p, long long n, CgState* st, hipStream_t s,
                       const double* rzp = nullptr, int np = 0);
template <typename T>
int launch_cg_update_t(T* x, T* r, const T* p, const T* w, long long n, CgState* st, double* part,
                       unsigned* cnt, double tol, int cg_max, hipStream_t s, const double* pwp = nullptr,
                       int npw = 0, const T* p_odd = nullptr);
// Pending x update of a loop run with p_odd (see k_cg_update): x += a_k p_k
// when the last completed iteration k is even and not flushed before; a no-op
// otherwise.
template <typename T>
void launch_cg_flush_t(T* x, const T* p_even, long long n, CgState* st, hipStream_t s);
// FP64 -> BF16 (RNE, through FP32); x64 += d32; device copy of BF16 arrays
void launch_cast_bf16(const double* a, uint16_t* b, long long n, hipStream_t s);
void launch_add_f32(double* x, const float* d, long long n, hipStream_t s);
void launch_cast_f32(const double* a, float* b, long long n, hipStream_t s);
void launch_copy_u16(const uint16_t* a, uint16_t* b, long long n, hipStream_t s);
// out = sum(part[0..n)) in a fixed order (single block)
void launch_finalize(const double* part, int n, double* out, const int* done, hipStream_t s);
// st->rz[st->it & 1] = sum of the partials (r.z of the current iteration)
void launch_finalize_rz(const double* part, int n, CgState* st, hipStream_t s);
// End of an iteration: st->it += 1 and the stopping test from the partials of ||r||^2.
void launch_cg_check(CgState* st, const double* part, int np, double tol, int cg_max, hipStream_t s);
// ||q||^2 and ||r_0||^2 from partials, and the stopping test before iteration 0.
void launch_cg_init(CgState* st, const double* part_qq, int nq, const double* part_rr, int nr,
                    double tol, int cg_max, hipStream_t s);
// Start (fresh) or continue a run on a new residual: stopping reference
// qq = qscale2 ||r||^2 from the partials of ||r||^2; continuing keeps the
// iteration count, the r.z / p.w history and the direction buffers.
void launch_cg_start(CgState* st, const double* part_rr, int nr, double qscale2, bool fresh, double tol,
                     int cg_max, hipStream_t s);
void launch_p_update(const double* z, double* p, long long n, CgState* st, hipStream_t s,
                     const double* rzp = nullptr, int np = 0);
// x += alpha p, r -= alpha w and partials of ||r||^2 (with p_odd, the
// direction buffers of SM_PAPPLY_DOT, p_odd on odd iterations, and x updated
// every second iteration: see launch_cg_flush_t); with cnt != null the sum
// is also reduced in the launch, st->it advanced and the stopping test applied
// by the last block (costs a device-scope fence per block).
int launch_cg_update(double* x, double* r, const double* p, const double* w, long long n,
                     CgState* st, double* part, unsigned* cnt, double tol, int cg_max, hipStream_t s,
                     const double* pwp = nullptr, int npw = 0, const double* p_odd = nullptr);
void launch_copy(const double* a, double* b, long long n, hipStream_t s);
template <typename T>
void launch_fill_t(T* a, long long n, float v0, float dv, hipStream_t s);
void launch_fill_bf16(uint16_t* a, long long n, hipStream_t s);
void launch_scale_into(const double* a, double* b, double alpha, long long n, hipStream_t s);
// Gram-Schmidt / reduced system helpers
// Block partials of K_R, q_R and ||q||^2 (m(m+1)/2 + m + 1 per block) into
// part; returns the block count.
int launch_gram(const double* Q, const double* W, const double* q, int m, long long ld,
                long long n, double* part, hipStream_t s);
// From the Gram partials (gpart, gnp blocks): K_R, q_R, ||q||^2 and the
// reduced Cholesky solve y (stored in md); t = Q y, partials of ||W y - q||^2
// into part (not gpart); with rq, also rq = q - W y.
int launch_combine(const double* Q, const double* W, const double* q, int m, long long ld,
                   long long n, MgarDev* md, double* t, double* part, hipStream_t s, double* rq,
                   const double* gpart, int gnp);
// Two-pass Gram-Schmidt of the m columns of R in place (three passes over
// the data per column; see k_gs_dots), leaving orthonormal columns, md->active
// and md->n0; dropped columns are zeroed. part, part2: two distinct buffers of
// vec_num_blocks(n) * (m + 1) doubles.
void launch_gs_fused(double* R, int m, long long ld, long long n, MgarDev* md, double* part, double* part2,
                     hipStream_t s);

// api.hip helpers shared with batch.hip (grid of a level, Dirichlet count,
// parameter validation of one design).
Geo mgar_internal_geo(const mgar_params& p, int level);
long long mgar_internal_count_fixed(const Geo& g);
int mgar_internal_validate(const mgar_params* p);

// Batched launches (several designs per launch) ----------------------------
// One work item per design and grid; items are sorted by `first`, the first
// block of the item in the launch, and a block finds its item by bisection.
// Offsets index the caller's concatenated arrays (node offsets for vectors,
// element offsets for cells; "c" = the coarse grid of a transfer).
struct BItem {
  Geo g, gc;
  long long off, coff, eoff, ceoff;
  int design, first, nblk, pad;
};
// Single-workgroup jobs: one block per design.
struct BTail {
  TailSpec ts;
  const void* bin;       // value type of the launch (double or float)
  void* xout;
  const double* A;
  int design, pad;
};
struct BCoarse {
  Geo g;
  const void* k;         // coarsest cells, value type of the cell loader
  double* A;
  int design, pad;
};
// skip (may be null): a block of design d returns at once when
// skip[d * sstride] != 0 (e.g. &BCgState::done of converged designs).
// stencil.hip
int batch_item_blocks(const Geo& g, int bs);   // blocks of one item of a node-parallel launch
// Value-type forms: T = double with CellD, T = float with CellF or CellB (the
// loader is moved to each design's cells). Coarsening from CellD to double
// or from CellB / CellF to float; tails of T; coarsest builds from CellD or
// CellF cells (the inverse is FP64 either way).
template <typename T, typename CL>
void launch_bstencil_t(int dim, int mode, const BItem* items, int nit, int nblk, int bs, const T* x, CL k, CL kref,
                       const T* b, T* out, double omega, double* part, const int* skip, int sstride,
                       hipStream_t s);
template <typename T>
void launch_brestrict_t(int dim, const BItem* items, int nit, int nblk, int bs, const T* rf, T* rc, const int* skip,
                        int sstride, hipStream_t s);
template <typename T>
void launch_bprolong_t(int dim, const BItem* items, int nit, int nblk, int bs, const T* xc, T* xf, const int* skip,
                       int sstride, hipStream_t s);
template <typename CL, typename TO>
void launch_bcoarsen_t(int dim, const BItem* items, int nit, int nblk, int bs, CL kf, TO* kc, const int* skip,
                       int sstride, hipStream_t s);
template <typename T>
void launch_bvtail_t(int dim, const BTail* jobs, int njobs, int lds_elems, double omega, const int* skip,
                     int sstride, hipStream_t s);
template <typename CL>
void launch_bcoarse_build_t(int dim, const BCoarse* jobs, int njobs, bool reg, int* status, const int* skip,
                            int sstride, hipStream_t s);
void launch_bstencil(int dim, int mode, const BItem* items, int nit, int nblk, int bs, const double* x,
                     const double* k, const double* kref, const double* b, double* out, double omega,
                     double* part, const int* skip, int sstride, hipStream_t s);
void launch_brestrict(int dim, const BItem* items, int nit, int nblk, int bs, const double* rf, double* rc,
                      const int* skip, int sstride, hipStream_t s);
void launch_bprolong(int dim, const BItem* items, int nit, int nblk, int bs, const double* xc, double* xf,
                     const int* skip, int sstride, hipStream_t s);
void launch_bcoarsen(int dim, const BItem* items, int nit, int nblk, int bs, const double* kf, double* kc,
                     const int* skip, int sstride, hipStream_t s);
void launch_bmask_copy(const BItem* items, int nit, int nblk, int bs, const double* in, double* out,
                       hipStream_t s);
// (double, float) and (float, double) conversions; fixed nodes become 0
template <typename TI, typename TO>
void launch_bmask_copy_t(const BItem* items, int nit, int nblk, int bs, const TI* in, TO* out, hipStream_t s);
void launch_bvtail(int dim, const BTail* jobs, int njobs, int lds_elems, double omega,
                   const int* skip, int sstride, hipStream_t s);
void launch_bcoarse_build(int dim, const BCoarse* jobs, int njobs, bool reg, int* status,
                          const int* skip, int sstride, hipStream_t s);
// vec.hip (items of the finest grid; vectors concatenated per design)
void launch_bdot(const BItem* items, int nit, int nblk, int bs, const double* a, const double* b,
                 double* part, const int* skip, int sstride, hipStream_t s);
// out[d * ostride + v] = sum of design d's partials of value v (nv values per
// block); with itsel, the target is shifted by (itsel[d * sstride] & 1).
void launch_bfinalize(const BItem* items, int nit, const double* part, int nv, double* out,
                      int ostride, const int* itsel, const int* skip, int sstride, hipStream_t s);
void launch_bcg_init(const BItem* items, int nit, BCgState* st, const double* part_qq,
                     const double* part_rr, double tol, int cg_max, const int* keep_done,
                     hipStream_t s);
void launch_bp_update(const BItem* items, int nit, int nblk, int bs, const double* z, double* p,
                      const BCgState* st, hipStream_t s);
void launch_bcg_update(const BItem* items, int nit, int nblk, int bs, double* x, double* r, const double* p,
                       const double* w, const BCgState* st, double* part, hipStream_t s);
void launch_bcg_check(const BItem* items, int nit, BCgState* st, const double* part, double tol,
                      int cg_max, hipStream_t s);
void launch_bmultidot(const BItem* items, int nit, int nblk, int bs, const double* Q, long long ld, int nc,
                      const double* v, double* part, hipStream_t s);
void launch_bgs_update(const BItem* items, int nit, int nblk, int bs, double* v, const double* Q, long long ld,
                       int nc, const MgarDev* md, hipStream_t s);
void launch_bgs_normalize(const BItem* items, int nit, int nblk, int bs, double* v, MgarDev* md, int col,
                          const double* nrm2, int nstride, hipStream_t s);
void launch_bgram(const BItem* items, int nit, int nblk, int bs, const double* Q, const double* W,
                  const double* q, long long ld, int m, double* part, hipStream_t s);
void launch_bgram_finalize(const BItem* items, int nit, const double* part, int m, MgarDev* md,
                           hipStream_t s);
void launch_bcombine(const BItem* items, int nit, int nblk, int bs, const double* Q, const double* W,
                     const double* q, long long ld, int m, MgarDev* md, double* t, double* part,
                     hipStream_t s);
// per design: Res = sqrt(res2 / qq); accept (path 1) when Res <= eps: the
// design's PCG state is marked done and keep[d] = 1 (K0 kept); otherwise
// path 2 and keep[d] = 0 (K0 renewed, MGCG runs). res_out[d] = Res.
void launch_bdecide(const BItem* items, int nit, MgarDev* md, BCgState* st, double eps, int* keep,
                    int* path, double* res_out, hipStream_t s);
void launch_bcopy_cells(const BItem* items, int nit, int nblk, int bs, const double* a, double* b,
                        const int* skip, int sstride, hipStream_t s);
// FP32 forms of the PCG vector kernels (inner products accumulated in FP64)
// and a copy of BF16 cells.
template <typename T>
void launch_bdot_t(const BItem* items, int nit, int nblk, int bs, const T* a, const T* b, double* part,
                   const int* skip, int sstride, hipStream_t s);
template <typename T>
void launch_bp_update_t(const BItem* items, int nit, int nblk, int bs, const T* z, T* p, const BCgState* st,
                        hipStream_t s);
template <typename T>
void launch_bcg_update_t(const BItem* items, int nit, int nblk, int bs, T* x, T* r, const T* p, const T* w,
                         const BCgState* st, double* part, hipStream_t s);
template <typename T>
void launch_bcopy_cells_t(const BItem* items, int nit, int nblk, int bs, const T* a, T* b, const int* skip,
                          int sstride, hipStream_t s);

// smooth.hip -----------------------------------------------------------------
// Boundary smoothing (Eq 24-27): nodal projection of -dc with cone weights of
// radius r, and the device bisection of the level that keeps the
// target volume (max_steps halvings of [min ns - 1, max ns], stopping at a
// bracket of 1e-14 of its initial width), followed by rho at the lower end
// and its volume in sd->vol. part: smooth_num_partials(g) doubles.
int smooth_num_partials(const Geo& g);
void launch_node_project(const Geo& g, const double* dc, double r, double* ns, hipStream_t st);
void launch_smooth_bisect(const Geo& g, const double* ns, double target, int nsub, int max_steps, SmoothDev* sd,
                          double* rho, double* part, hipStream_t st);

// topopt.hip -----------------------------------------------------------------
void launch_simp(const double* xphys, double* k, long long n, double k0, double kmin, double penal,
                 hipStream_t s);
void launch_load(const Geo& g, const double* Qe, double* q, hipStream_t s);
// y = (H x) * scale (scale may be null) with ntap taps off[3t..3t+2], w[t];
// hr = the largest |offset| of any tap (inputs are staged in LDS for hr <= 3).
void launch_filter_fwd(const Geo& g, const int* off, const double* w, int ntap, int hr, const double* x,
                       const double* invHs, double* y, hipStream_t s);
void launch_filter_hs(const Geo& g, const int* off, const double* w, int ntap, double* invHs,
                      hipStream_t s);
void launch_sens_elem(const Geo& g, const double* xphys, const double* T, const double* invHs,
                      double k0, double kmin, double penal, double* gout, hipStream_t s);
void launch_oc_init(OcDev* oc, double target, double hint, hipStream_t s);
int launch_oc_pass(const double* x, const double* dc, const double* dv, long long n, double move,
                   const OcDev* oc, double* part, hipStream_t s);
void launch_oc_walk(OcDev* oc, const double* part, int np, double target, double tol,
                    hipStream_t s);
void launch_oc_final(const double* x, const double* dc, const double* dv, long long n, double move,
                     const OcDev* oc, double* xnew, hipStream_t s);
