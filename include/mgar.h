/*
 * mgar.h -- C ABI of libmgar.so, a gfx950 (MI355X) implementation of the solve
 * path of Multigrid Assisted Reanalysis (MGAR) for SIMP heat-conduction
 * topology optimisation.
 *
 * Problem (Eq 2-5): steady isotropic conduction on a structured grid of unit
 * square (2D, bilinear) or cubic (3D, trilinear) cells, discretised to
 * K(rho~) t = q, with the SIMP conductivity of Eq 4 per element, Dirichlet
 * T = 0 on a box of nodes and a fixed internal heat source.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Numbering: node (i, j, k) -> i + (nelx+1) * (j + (nely+1) * k); element
 *   (ex, ey, ez) -> ex + nelx * (ey + nely * ez); in 2D k = ez = 0.
 *   An N-vector has (nelx+1)(nely+1)(nelz+1) entries (nelz+1 := 1 in 2D), an
 *   E-vector nelx*nely*nelz entries (nelz := 1 in 2D).
 * Memory: every array argument is a DEVICE pointer to contiguous FP64 data,
 *   owned by the caller, unless the comment says "host". The library never
 *   frees or keeps caller memory beyond a call. Outputs must not alias inputs
 *   unless stated.
 * Streams: all work is enqueued on the stream given to mgar_setup (or
 *   mgar_set_stream) in stream order. Entry points that return host scalars
 *   (stats, compliance, lambda) synchronise that stream before returning.
 * Dirichlet nodes: every N-vector the library writes is exactly 0 there;
 *   N-vector inputs are read as 0 there.
 * Errors: nothing throws across the ABI. 0 = success; > 0 = warning with the
 *   outputs written; < 0 = error, outputs unspecified but no memory owned by
 *   the caller is touched beyond the outputs. mgar_strerror() gives text.
 * Threading: a handle may be used by one host thread at a time.
 */
#ifndef MGAR_H
#define MGAR_H

#ifdef __cplusplus
extern "C" {
#endif

#define MGAR_OK 0
#define MGAR_W_NOT_CONVERGED 1   /* cg_max reached; outputs hold the last iterate */
#define MGAR_E_ARG (-1)          /* bad argument or null pointer */
#define MGAR_E_DIMS (-2)         /* elements per axis not a multiple of 2^(levels-1), or coarsest grid too large */
#define MGAR_E_SINGULAR (-3)     /* the coarsest grid holds no Dirichlet node */
#define MGAR_E_HIP (-4)          /* HIP runtime error */
#define MGAR_E_NOT_SPD (-5)      /* non-positive pivot in the reduced or coarsest system */
#define MGAR_E_PRECISION (-6)    /* unsupported precision mode */
#define MGAR_E_STATE (-7)        /* reanalysis called before any MGCG solve set K0 */

#define MGAR_PATH_MGCG 0         /* pure MGCG solve */
#define MGAR_PATH_ACCEPT 1       /* reduced (reanalysis) solution accepted, Eq 28 */
#define MGAR_PATH_FALLBACK 2     /* reduced solution rejected; MGCG from it, K0 renewed */

#define MGAR_PREC_FP64 0         /* every operation in FP64 */
#define MGAR_PREC_MIXED 1        /* FP32 multigrid PCG over BF16 densities with FP64 residual replacement */

#define MGAR_MAX_BASIS 8
#define MGAR_MAX_FILTER_R2 64    /* largest ceil(filter radius) in 2D (element lengths) */
#define MGAR_MAX_FILTER_R3 12    /* largest ceil(filter radius) in 3D */

typedef struct mgar_handle mgar_handle;

/* Problem and solver parameters (Sec. 2.1-3.2). */
typedef struct {
  int dim;                /* 2 or 3 */
  int nelx, nely, nelz;   /* elements per axis; nelz ignored in 2D */
  int levels;             /* number of MG grids including the finest (the paper's nl, Sec. 3.2) */
  int fix_lo[3];          /* inclusive node-index box of Dirichlet (T = 0) nodes, finest grid */
  int fix_hi[3];          /*   (third entries ignored in 2D) */
  double k0, kmin, penal; /* SIMP, Eq 4: 1, 1e-3, 3 */
  double omega;           /* damped-Jacobi weight (Sec. 2.2 (ii)); 0.8 */
  int n_basis;            /* m, reanalysis basis size (Eq 14), 1..MGAR_MAX_BASIS; 2 */
  double eps_accept;      /* eps1 of Eq 28 */
  int cg_max;             /* maximum CG iterations per MGCG solve */
  int basis_x0_zero;      /* 0: V-cycle initial guess r_{i-1} as printed in Eq 17; 1: zero */
  int precision;          /* MGAR_PREC_FP64 or MGAR_PREC_MIXED */
  double filter_r;        /* cone density-filter radius, Eq 7-8 (element lengths) */
  double inner_tol;       /* MGAR_PREC_MIXED: the FP32 PCG run folds its correction into the
                           * FP64 solution and replaces its residual by the FP64 one each
                           * time that residual has dropped by this factor (0 < inner_tol < 1;
                           * 1e-3); the Krylov recurrences carry on across replacements */
} mgar_params;

/* Per-solve report. */
typedef struct {
  int path;               /* MGAR_PATH_* */
  int cg_iters;           /* CG iterations (each applies one V-cycle) */
  int vcycles;            /* V-cycles, including those that built the basis */
  int refinements;        /* FP32 segments between FP64 residual replacements (mixed mode) */
  double res_ca;          /* Eq 28 residual of the reduced solution (NaN for pure MGCG) */
  double res_final;       /* ||q - K t|| / ||q|| of the returned t: recursive residual of the last CG iterate */
  float ms;               /* device time of the call, milliseconds (-1: timing off, mgar_set_timing) */
} mgar_stats;

/* Fill *p with the defaults above for a grid; fix box empty. */
void mgar_default_params(mgar_params* p);

/* Create a handle: validates the grid (levels, divisibility, a Dirichlet node
 * on the coarsest grid, coarsest grid at most 1024 nodes), allocates all
 * device workspace, precomputes the filter normalisation. `stream` is a
 * hipStream_t (NULL = default stream). Returns MGAR_OK and *out, or an error. */
int mgar_setup(const mgar_params* p, void* stream, mgar_handle** out);
void mgar_destroy(mgar_handle* h);
int mgar_set_stream(mgar_handle* h, void* stream);
/* Per-solve device timing (mgar_stats.ms) on (default) or off. Timing waits
 * for the solve's last kernel on the host; off, the solves return without that
 * synchronisation and ms is -1. */
int mgar_set_timing(mgar_handle* h, int on);
const char* mgar_strerror(int code);
/* Sizes: nodes, elements, and the nodes of grid `level`. */
int mgar_sizes(const mgar_handle* h, int level, long long* nnodes, long long* nelem);

/* Nodal heat load from a per-element source Qe (E-vector, source per unit
 * volume): q_i = sum over elements e at node i of Qe_e * |e| / 2^d, 0 on
 * Dirichlet nodes (consistent Q1 load of Eq 3). */
int mgar_load_vector(mgar_handle* h, const double* Qe, double* q);

/* Density filter, Eq 6-8: xphys_e = sum_j w_ej x_j / sum_j w_ej with the cone
 * weight w_ej = max(0, r - |c_e - c_j|), truncated at the domain boundary. */
int mgar_density_filter(mgar_handle* h, const double* x, double* xphys);

/* Change the density-filter radius (Eq 7-8) used by every later call of
 * mgar_density_filter, sens_filter, oc_update and mgar_sens_oc: the filter
 * taps, their normalisation Hs and the filtered-volume weights are rebuilt on
 * the device. This is the per-cycle step of continuous density filtering
 * (Eq 22-23: r^(k) = max(r_min, eta r^(k-1))), whose schedule the caller
 * runs. r > 0 with ceil(r) <= MGAR_MAX_FILTER_R2 (2D) or MGAR_MAX_FILTER_R3
 * (3D), else MGAR_E_ARG. Synchronises the handle's stream; reallocates the
 * tap table only when r needs more taps than any earlier radius. */
int mgar_set_filter_radius(mgar_handle* h, double r);

/* Boundary-smoothing post-process (Sec. 2.3, Eq 24-27), run once on the final
 * design. dc (E-vector): the filtered compliance sensitivities of that design
 * (Eq 9-11, as sens_filter writes them). Their negatives, large where
 * material pays most, are projected onto the nodes, ns_i = sum_e w_ie (-dc_e)
 * / sum_e w_ie with the cone weight w_ie = max(0, r - |x_i - c_e|) to the
 * element centroids (ns: N-vector output, may be NULL). Eq 24: rho_e = 1 when every node of e has
 * ns > level, 0 when every one has ns < level, otherwise (Eq 25-27) the
 * fraction of the (nsub+1)^d lattice points of e (corners included) at which
 * the Q1 interpolation of its nodal values exceeds the level. The level is
 * bisected on [min ns - 1, max ns] (100 halvings, or until the bracket is
 * 1e-14 of its initial width), keeping sum_e rho_e >= volfrac * E at the
 * lower end, which is returned in *level (host) with its volume sum_e rho_e
 * in *volume (host); rho (E-vector output) is taken there. 0 < volfrac <= 1,
 * 1 <= nsub <= 64, radius limits as mgar_set_filter_radius; synchronises. */
int mgar_smooth_boundary(mgar_handle* h, const double* dc, double volfrac, double r, int nsub, double* rho,
                         double* ns, double* level, double* volume);

/* MGCG: PCG preconditioned by one V-cycle on K(xphys), started from T0 (may be
 * NULL = 0), until ||r||/||q|| <= tol or cg_max iterations. Makes K(xphys) the
 * factorised matrix K0 used by mgar_solve. T: N-vector output. stats may be
 * NULL. Returns MGAR_OK or MGAR_W_NOT_CONVERGED. */
int mgcg_solve(mgar_handle* h, const double* xphys, const double* q, const double* T0,
               double tol, double* T, mgar_stats* stats);

/* MGAR reanalysis (Eq 12-21, Eq 28, Sec. 3.1): basis r_1 = T0, r_i = one
 * V-cycle on K0 for K0 r_i = -(K - K0) r_{i-1}; Gram-Schmidt; reduced solve;
 * accept when Res <= eps_accept, else MGCG from the reduced solution to tol,
 * renewing K0. Requires a previous mgcg_solve (MGAR_E_STATE otherwise). */
int mgar_solve(mgar_handle* h, const double* xphys, const double* q, const double* T0,
               double tol, double* T, mgar_stats* stats);

/* Compliance and sensitivities (Eq 5, 9-11): *compliance (host) = q^T T;
 * dc = filter adjoint of -p (k0-kmin) xphys^(p-1) T_e^T KE T_e; dv = filter
 * adjoint of 1. dc, dv: E-vector outputs. */
int sens_filter(mgar_handle* h, const double* xphys, const double* T, const double* q,
                double* dc, double* dv, double* compliance);

/* Optimality-criteria update: x_new = clamp(x sqrt(max(0,-dc)/(dv lambda)),
 * max(0, x-move), min(1, x+move)) with lambda bisected on [0, 1e9] until
 * (l2-l1)/(l1+l2) <= 1e-10 so that the filtered volume sum_e dv_e x_new_e
 * meets volfrac * E. *lambda (host) receives the final midpoint; may be NULL.
 * The bisection is evaluated at batches of candidate multipliers (the first
 * batch around the handle's previous result, if any); the midpoints and the
 * result are those of the plain bisection whatever the candidates. */
int oc_update(mgar_handle* h, const double* x, const double* dc, const double* dv,
              double volfrac, double move, double* x_new, double* lambda);

/* sens_filter followed by oc_update (the same kernels, results and outputs),
 * for the optimisation loop: the compliance comes back in the OC update's
 * first host synchronisation instead of one of its own. compliance and lambda
 * (host) may be NULL. */
int mgar_sens_oc(mgar_handle* h, const double* xphys, const double* T, const double* q, const double* x,
                 double volfrac, double move, double* dc, double* dv, double* x_new, double* compliance,
                 double* lambda);

/* Drop K0: the next mgar_solve returns MGAR_E_STATE until an mgcg_solve.
 * Also forgets the previous OC multiplier. */
int mgar_reset(mgar_handle* h);

/* ---- Operator-level entry points (same conventions). `level` 0 is the
 * finest grid; grid l has elements of edge 2^l. Element conductivities `k`
 * are E_l-vectors of grid `level`. -------------------------------------- */

/* y = K_l(k) x (Eq 3 on grid l, rediscretised). */
int mgar_op_apply(mgar_handle* h, int level, const double* k, const double* x, double* y);
/* One damped-Jacobi sweep on grid l: out = x + omega D^-1 (b - K_l x). */
int mgar_op_jacobi(mgar_handle* h, int level, const double* k, const double* b,
                   const double* x, double* out);
/* Restriction of Table 1 step 2: rc = P_l^T rf (grid l -> grid l+1). */
int mgar_op_restrict(mgar_handle* h, int level, const double* rf, double* rc);
/* Interpolation of Table 1 step 4: xf += P_l xc (grid l+1 -> grid l). */
int mgar_op_prolong(mgar_handle* h, int level, const double* xc, double* xf);
/* Coarse conductivity: kc = mean of the 2^d children of each grid-(l+1) element. */
int mgar_op_coarsen(mgar_handle* h, int level, const double* kf, double* kc);
/* Make K(xphys) the factorised matrix K0: SIMP, coarse conductivities and the
 * coarsest-grid inverse (Table 1 step 3). */
int mgar_build_hierarchy(mgar_handle* h, const double* xphys);
/* One V-cycle of Table 1 on the K0 hierarchy: x = MG(K0, b, x0); x0 may be NULL (zero). */
int mgar_vcycle(mgar_handle* h, const double* b, const double* x0, double* x);
/* b = -(K(xphys) - K0) r: the right-hand side of Eq 15/17. */
int mgar_op_dk(mgar_handle* h, const double* xphys, const double* r, double* b);
/* Densities as stored by the mixed-precision mode: out[e] = BF16 bits of x[e],
 * rounded to nearest even through FP32. out: E uint16 values (device). */
int mgar_op_bf16(mgar_handle* h, const double* x, void* out);

/* ---- Launch-shape tuning. ----------------------------------------------------
 * Every stencil launch on grid `level` in mode `mode` (0 apply, 1 apply + dot,
 * 2 residual, 3 Jacobi sweep, 4 Jacobi sweep + dot, 5 sweep from zero, 6 -dK
 * apply) of precision class `cls` (0: FP64 kernels; 1: FP32 kernels of
 * MGAR_PREC_MIXED) uses a launch shape of four ints {kind, kz, zd, ntx}:
 * kind 0 = one thread per node; kind 1 = z-marching blocks (3D) over ntx tiles
 * across x, kz node planes per block, a zd-deep (1 to 4) load queue; kind 2 =
 * as kind 1 with two node rows per thread (zd 1 or 2). Every
 * shape computes each node with the same arithmetic; only the summation order
 * of the dot products of modes 1 and 4 depends on the shape. Setup installs a
 * default shape everywhere.
 *
 * mgar_autotune times every candidate shape of each (class, level, mode) the
 * solvers launch (classes of the handle's precision, grids above the
 * single-workgroup tail), `reps` launches each on scratch data it allocates and
 * frees, and installs the fastest. best_us (host, may be NULL) receives the
 * winning average launch time in microseconds at [(cls*levels + level)*7 + mode]
 * (0 where nothing was tuned); it must hold 2*levels*7 doubles. Not to be
 * called while other work of the handle is in flight.
 * mgar_tune_get / mgar_tune_set read and install one shape (host int[4]), e.g.
 * from a cache; set returns MGAR_E_ARG for a shape the grid cannot take. */
int mgar_autotune(mgar_handle* h, int reps, double* best_us);
int mgar_tune_get(const mgar_handle* h, int cls, int level, int mode, int* shape);
int mgar_tune_set(mgar_handle* h, int cls, int level, int mode, const int* shape);

/* ||q - K(xphys) T|| / ||q|| over the free nodes, FP64, into *relres (host):
 * the criterion for any initial guess (a learned seed is used only when its
 * residual is below that of the previous temperature). */
int mgar_residual(mgar_handle* h, const double* xphys, const double* q, const double* T, double* relres);

/* For callers that cannot allocate device memory (work under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the criterion of
 * mgar_residual without a handle. *relres (DEVICE, one double) receives
 * ||q - K(xphys) T|| / ||q|| over the free nodes of the grid that p
 * describes (dim, nelx, nely, nelz, fix_lo/fix_hi, k0, kmin, penal; the
 * other fields are ignored), T and q read as 0 on Dirichlet nodes; 0 when q
 * is 0 there. Enqueued on `stream` (hipStream_t, NULL = default) without a
 * host synchronisation; it calls no allocating routine. Its block partial
 * sums live in a static device array of 4096 x 2 doubles (64 KiB, held on
 * every GPU the library runs on until the process ends): calls of one
 * process that overlap on the same GPU race on it. Grids of more than
 * 2^31 - 1 nodes are rejected with MGAR_E_ARG; equal to mgar_residual up to
 * the summation order. */
int mgar_residual_noalloc(const mgar_params* p, const double* xphys, const double* q, const double* T,
                          double* relres, void* stream);

/* ---- Learned initial guess (3D). -------------------------------------------
 * A convolutional U-Net on the element grid with `levels` levels of
 * channels[0..levels-1] channels (each a multiple of 16, at most 128; every
 * axis a multiple of 2^(levels-1)). Input: three channels per element
 * (physical density, fraction of the element's 8 corner nodes that are
 * Dirichlet nodes, heat source divided by its max-norm: 1 until
 * mgar_net_set_source). Encoder: per level two 3x3x3 convolutions with ReLU
 * (zero padding), 2x average pooling between levels. Decoder from level
 * levels-2 down to 0: trilinear 2x upsampling of cell-centred values
 * (clamped at the boundary), concatenation [upsampled, encoder output of the
 * level], two 3x3x3 convolutions with ReLU. Head: 1x1x1 convolution to one
 * output u per element. Parameters: one FP32 vector, per layer the weights
 * [co][ci][k][k][k] then the co biases, layers in the order encoder (level 0
 * first), decoder (level levels-2 first), head (mgar_net_sizes gives the
 * count). Created with zero parameters; the caller installs initial values
 * (mgar_net_set_params, which also resets Adam). Activations and their
 * gradients are stored in BF16, convolutions run on the matrix cores with
 * FP32 sums; weight gradients and the loss are summed in FP64.
 * Prediction on the finest nodes: scale * mean of u over the elements that
 * touch the node, 0 on Dirichlet nodes. Training pair (xphys, T, scale): loss
 * = mean over the free nodes of (prediction/scale - T/scale)^2, one Adam step
 * (0.9, 0.999, 1e-8) with learning rate lr. xphys, qe: E-vectors, T: N-vector
 * (device, FP64); theta, u: host FP32 arrays of nparams / E values; grad:
 * host FP64 array of nparams values. Every call enqueues on the stream given
 * at creation; mgar_net_train_step waits for it only when loss is non-null,
 * mgar_net_set_source, mgar_net_set_params, mgar_net_get_params, mgar_net_grad
 * and mgar_net_destroy always. */
typedef struct mgar_net mgar_net;
int mgar_net_create(const mgar_params* p, int levels, const int* channels, void* stream, mgar_net** out);
void mgar_net_destroy(mgar_net* n);
int mgar_net_sizes(const mgar_net* n, long long* nparams);
int mgar_net_set_source(mgar_net* n, const double* qe);
int mgar_net_set_params(mgar_net* n, const float* theta);
int mgar_net_get_params(const mgar_net* n, float* theta);
int mgar_net_infer(mgar_net* n, const double* xphys, double scale, double* T_seed);
int mgar_net_output(const mgar_net* n, float* u);
int mgar_net_grad(mgar_net* n, const double* xphys, const double* T, double scale, double* grad, double* loss);
int mgar_net_train_step(mgar_net* n, const double* xphys, const double* T, double scale, double lr,
                        double* loss);

/* ---- Batched solves (many independent designs at once). --------------------
 * A batch holds `ndesigns` designs of uneven grids (2D and 3D may be mixed),
 * each described by its own mgar_params (n_basis, omega, eps_accept, cg_max,
 * basis_x0_zero, precision, k0, kmin, penal and, for MGAR_PREC_MIXED,
 * inner_tol must agree across designs, else MGAR_E_ARG; levels >= 2).
 * The designs' K(xphys) t = q are solved together: every stage of the V-cycle
 * and of the PCG iteration is one launch per dimension over all designs'
 * grids, with per-design PCG state on the device, so converged designs drop
 * out and one PCG iteration is captured once as a hipGraph and replayed until
 * every design stopped. In FP64 each design gets the same solution as its own
 * mgcg_solve / mgar_solve up to the summation order of dot products. With
 * MGAR_PREC_MIXED the preconditioner and the reanalysis V-cycles are those of
 * the single-design mixed form (FP32 over BF16 densities), and each PCG is
 * plain iterative refinement: FP32 inner runs that reduce their residual by
 * inner_tol, each followed by an FP64 residual replacement, until the FP64
 * residual meets tol (at most cg_max inner iterations in total, 40
 * replacements); stats report the inner iterations and the replacements.
 * Arrays are concatenations over designs in params order: design d's nodes
 * start at node_off[d] and its elements at elem_off[d] (mgar_batch_layout;
 * both host arrays of ndesigns + 1 entries, the last = totals). stats: host
 * array of ndesigns reports (may be NULL). stream NULL: the batch works on a
 * stream of its own, ordered after the caller's default stream; every call
 * returns with its work complete. */
typedef struct mgar_batch mgar_batch;
int mgar_batch_setup(const mgar_params* p, int ndesigns, void* stream, mgar_batch** out);
void mgar_batch_destroy(mgar_batch* b);
int mgar_batch_layout(const mgar_batch* b, long long* node_off, long long* elem_off);
/* 1 (default): replay the captured PCG iteration graph; 0: launch eagerly. */
int mgar_batch_set_graph(mgar_batch* b, int use_graph);
/* Per design, as mgar_load_vector. */
int mgar_batch_load_vector(mgar_batch* b, const double* Qe, double* q);
/* Threads per block of every node-parallel launch of the batch (64, 128 or
 * 256; 256 after setup): the work lists are rebuilt (the call waits for the
 * batch's stream) and captured iterations are dropped. The arithmetic of every
 * node is the same for every block size; the order in which block partials
 * of a dot product are summed differs. */
int mgar_batch_set_block(mgar_batch* b, int bs);
int mgar_batch_get_block(const mgar_batch* b, int* bs);
/* Autotuner of the batched launches: times a batched MGCG solve from T0 = 0
 * of (xphys, q) to tol (reps times after one warm-up, HIP events on the
 * batch's stream) for blocks of 256, 128 and 64 threads and keeps the fastest
 * (*bs_out; us_out, if not NULL, receives the three mean times in
 * microseconds in that order). Allocates one N-vector for its own solves. */
int mgar_batch_autotune(mgar_batch* b, const double* xphys, const double* q, double tol, int reps, int* bs_out,
                        float* us_out);
/* Per design, as mgcg_solve (T0 may be NULL = 0) and mgar_solve (requires a
 * previous mgcg_batch_solve: MGAR_E_STATE otherwise). Returns MGAR_OK,
 * MGAR_W_NOT_CONVERGED if any design hit cg_max, or an error. In the batched
 * reanalysis only designs whose reduced solution is rejected renew K0. */
int mgcg_batch_solve(mgar_batch* b, const double* xphys, const double* q, const double* T0,
                     double tol, double* T, mgar_stats* stats);
int mgar_batch_solve(mgar_batch* b, const double* xphys, const double* q, const double* T0,
                     double tol, double* T, mgar_stats* stats);

/* PCG iterations are captured once as HIP graphs (chunks of 1, 2, 4 and 8
 * iterations, per tolerance) and replayed on a stream the handle owns, ordered
 * after and before the handle's stream; the iteration index lives on the
 * device, so replays are exact repeats of eager launches. on = 0 launches every
 * kernel eagerly instead (kernel timing via mgar_profile always does). */
int mgar_set_graphs(mgar_handle* h, int on);

/* ---- Instrumentation. ------------------------------------------------------
 * Kernel timing for roofline reports: while enabled, every launch of a
 * finest-grid stencil kernel whose mode bit is set in `mode_mask` is bracketed
 * by two HIP events on the handle's stream (bit i = mode i: 0 apply, 1 apply +
 * dot, 2 residual, 3 Jacobi sweep, 4 Jacobi sweep + dot, 5 sweep from zero,
 * 6 -dK apply). mgar_profile_read returns, and resets, the number of such
 * launches, their summed event time in milliseconds and their summed
 * algorithmic HBM bytes (every operand vector read once, every result written
 * once). mode_mask = 0 disables timing. */
int mgar_profile(mgar_handle* h, unsigned mode_mask);
int mgar_profile_read(mgar_handle* h, long long* launches, double* total_ms, double* total_bytes);

#ifdef __cplusplus
}
#endif
#endif /* MGAR_H */
