/*
 * stmg.h - C ABI of the MI355X space-time multigrid library (libstmg.so).
 *
 * The library solves one all-at-once time-slab system S u = b of a space-time
 * finite element discretisation of the heat equation or of the acoustic wave
 * equation (Margenberg & Munch, "A Space-Time Multigrid Method for Space-Time
 * Finite Element Discretizations of Parabolic and Hyperbolic PDEs"):
 *   - spatial continuous Q_p on a structured hexahedral (d = 3) or
 *     quadrilateral (d = 2) mesh of [lo, hi], Cartesian or with displaced
 *     vertices (multilinear cells), homogeneous Dirichlet data on the boundary
 *     (Sections 1.1 and 2, eqs. fespace and space-matrices);
 *   - dG(k) or cGP(k) in time, c time cells batched into one slab
 *     (Sections 2.1-2.2, eqs. heat-cg-dg-at-once, wave-cg-dg-at-once,
 *     heat-cg-cg-at-once, wave-cg-cg-at-once).  For every pair the slab matrix
 *     is S = M_T (x) A_h + N_T (x) M_h with small dense temporal factors M_T, N_T
 *     (N_T = A_T for heat, A_T M_T^{-1} A_T for the condensed wave system);
 *   - solver: flexible GMRES in FP64, preconditioned by one space-time multigrid
 *     V-cycle per iteration (Section 3, Alg. stmg) with the space-time cell-wise
 *     additive Schwarz smoother (eqs. vanka0 and vanka), spatial h/p transfers
 *     and, optionally, k- and tau-levels in time below the spatial ones
 *     (Section 3.2, Alg. mg-sequence).
 *
 * Vector layout (every device vector argument): time-major [n_t][N_x], where
 * N_x = prod_d (p * n_cells[d] + 1) lattice nodes ordered x fastest, n_t =
 * c (k+1) for dG(k) and c k for cGP(k).  Dirichlet (boundary) nodes are part of
 * the vector; S acts as the identity on them.  Level 0 is the finest level.
 *
 * Ownership: all vector arguments are device pointers owned by the caller,
 * contiguous, of the stated dtype, on the device that was current at
 * stmg_create.  Host arrays passed to stmg_create are copied.  The library owns
 * its workspace (allocated in stmg_create, released in stmg_destroy).
 *
 * Streams: every call enqueues its kernels on the hipStream_t given at
 * creation.  stmg_vmult, stmg_smooth, stmg_vcycle, stmg_prolongate and
 * stmg_restrict are asynchronous.  stmg_create and stmg_solve synchronise.
 *
 * Host-only queries (stmg_temporal_matrices, stmg_temporal_cell_factors,
 * stmg_temporal_dof_times, stmg_temporal_prolongation, stmg_transfer_1d) need no
 * handle and no device;
 * they fill caller-owned host arrays with the set-up data the library builds.
 *
 * Errors: every function returns an stmg_status; nothing is thrown or aborted
 * across the ABI.  stmg_last_error() returns a thread-local message for the
 * last failing call on the calling thread.  A handle must not be used by two
 * host threads at the same time.
 */
#ifndef STMG_H
#define STMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STMG_ABI_VERSION 4

typedef enum {
  STMG_OK = 0,
  STMG_E_ARG = 1,          /* invalid argument (null pointer, bad level/dtype, bad config) */
  STMG_E_NOMEM = 2,        /* device or host allocation failed */
  STMG_E_HIP = 3,          /* a HIP runtime or ROCm library call failed */
  STMG_E_NOCONV = 4,       /* stmg_solve reached max_iter; info is still filled */
  STMG_E_NONFINITE = 5,    /* NaN/Inf in the right-hand side or in the iteration */
  STMG_E_UNSUPPORTED = 6,  /* configuration outside what the library implements */
  STMG_E_STATE = 7         /* call not valid for this handle's state (e.g. no CNN weights) */
} stmg_status;

typedef enum { STMG_HEAT = 0, STMG_WAVE = 1 } stmg_problem;
typedef enum { STMG_DG = 0, STMG_CGP = 1 } stmg_time_method;
typedef enum { STMG_F64 = 0, STMG_F32 = 1 } stmg_dtype;
typedef enum { STMG_PREC_FP64 = 0, STMG_PREC_FP32 = 1, STMG_PREC_LEARNED = 2 } stmg_precision;
/* How the operator (eq. lin-sys) and the smoother (eq. vanka0) sum the contributions of cells
 * that share lattice nodes; all three give the same result up to rounding order, and each is
 * bitwise reproducible.
 * DEFAULT: on 3D levels with axis-aligned cells and one coefficient per cell the operator runs on
 *   bricks of cells summed in LDS, launched in 2^3 brick colours (face nodes updated in colour
 *   order); other levels as PER_CELL.
 * PER_CELL: every cell writes its contribution to a per-cell buffer and a node gather sums them in
 *   a fixed cell order (a level whose buffer cannot be allocated falls back to COLOUR).
 * COLOUR: 2^d colour launches of cells that share no node, each adding into the vector. */
typedef enum { STMG_PATH_DEFAULT = 0, STMG_PATH_PER_CELL = 1, STMG_PATH_COLOUR = 2 } stmg_kernel_path;

/* One slab problem and its solver settings.  Fields follow the paper's notation. */
typedef struct {
  int32_t abi_version;     /* must be STMG_ABI_VERSION */
  int32_t dim;             /* 2 or 3 */
  int32_t problem;         /* stmg_problem */
  int32_t time_method;     /* stmg_time_method */
  int32_t p;               /* spatial degree, 1..4 */
  int32_t k;               /* temporal degree: dG 0..5, cGP 1..5 */
  int32_t n_time_cells;    /* c >= 1, time cells in the slab */
  int32_t n_cells[3];      /* cells per direction (n_cells[2] ignored for dim 2) */
  double t0, tau;          /* slab start, time-cell length (> 0) */
  double lo[3], hi[3];     /* Cartesian box (only used when vertices == NULL) */
  int32_t n_smooth;        /* nu1 = nu2 smoothing steps per level, >= 1 */
  int32_t min_p;           /* p-coarsening stops at this degree (>= 1) */
  int32_t coarse_cells;    /* h-coarsening stops before a level has fewer cells per direction */
  int32_t vcycle_dtypes;   /* bit 0: build FP64 V-cycle data, bit 1: FP32; 0 = from precision */
  double omega;            /* > 0: relaxation used on every level; == 0: per level from eq. relaxation,
                              omega_l = 2 / (lambda_max + lambda_min) of ASM * S_l (15-step Arnoldi
                              estimate, clamped to (0, 1]); < 0: per level omega_l = |omega| /
                              lambda_max.  omega = -1.5 is eq. relaxation with lambda_min read as
                              lambda_max / 3: every eigenvalue in [lambda_max / 3, lambda_max] is
                              damped by at least 2, independently of h, while with the true lambda_min
                              (-> 0 as h -> 0) the top of the spectrum is hardly damped at Q4 */
  int32_t precision;       /* stmg_precision: preconditioner used by stmg_solve */
  int32_t restart;         /* FGMRES restart length m >= 1 */
  int32_t max_iter;        /* total FGMRES iterations allowed */
  int32_t gram_schmidt;    /* 0: one classical Gram-Schmidt pass, a second one only when the first
                              removes more than 7/8 of ||w||; 1: always two passes */
  double rtol;             /* stop at ||b - S x||_2 / ||b||_2 <= rtol (true residual) */
  uint64_t seed;           /* reserved for randomised setup steps */
  int32_t asm_variant;     /* 0: exact cell blocks, factored by generalised eigenvectors of the
                              probed principal submatrices; 1: separable surrogate (fast
                              diagonalisation, Cartesian meshes only); 2: separable vertex
                              patches (Section 5's extension of the cell-wise smoother: one block
                              per interior vertex on the nodes strictly inside its 2^d cells,
                              Kronecker product of the assembled 1D patch matrices with the
                              patch-mean coefficient; Cartesian meshes with at least two cells
                              per direction, at most 6 temporal DoFs per time cell) */
  int32_t time_mg;         /* 0: spatial levels only; 1: below the coarsest spatial level, coarsen in
                              time (Section 3.2): lower k by one per level to its minimum (dG 0,
                              cGP 1), then merge pairs of time cells while their number is even;
                              temporal prolongation = embedding of the coarse trial functions,
                              restriction its transpose; needs n_t <= 32 */
  int32_t kernel_path;     /* stmg_kernel_path: how operator and smoother sum the cell contributions */
} stmg_config;

typedef struct {
  int32_t iterations;      /* FGMRES iterations (one V-cycle each) */
  int32_t restarts;
  double rel_residual;     /* true relative residual ||b - S x|| / ||b|| at exit, FP64 */
  double seconds;          /* wall time of the solve (host clock, after a device sync) */
  double t_smoother;       /* event-timed buckets: ASM smoother applications */
  double t_gmg_other;      /* V-cycle work other than the smoother (operators, transfers, coarse solve) */
  double t_operator;       /* outer FP64 operator applications */
  double t_other;          /* everything else: orthogonalisation, updates, casts, CNN */
  int32_t cnn_used;        /* learned stage accepted this many times */
  int32_t cnn_fallbacks;   /* learned stage rejected (plain V-cycle used) */
} stmg_solve_info;

#define STMG_MAX_LEVELS 16
typedef struct {
  int32_t n_levels;
  int32_t n_t;                              /* finest level */
  int32_t nt_cell;                          /* temporal DoFs per time cell, finest level */
  int32_t temporal_nnz;                     /* nonzeros of M_T plus nonzeros of N_T */
  int64_t n_x[STMG_MAX_LEVELS];             /* lattice nodes per level */
  int32_t p[STMG_MAX_LEVELS];
  int32_t cells[STMG_MAX_LEVELS][3];
  double omega[STMG_MAX_LEVELS];            /* relaxation per level (0 on the coarsest) */
  int64_t coarse_unknowns;                  /* interior unknowns of the coarsest level */
  int64_t device_bytes;                     /* library-owned device memory */
  double setup_seconds;
  int32_t n_t_level[STMG_MAX_LEVELS];       /* temporal DoFs per level (differ with time_mg) */
  int32_t nt_cell_level[STMG_MAX_LEVELS];   /* temporal DoFs per time cell, per level */
  int32_t eig_resolves;                     /* batched local eigen-solves repeated because a cell's
                                               eigenpairs failed the check (0 normally) */
} stmg_info;

typedef struct stmg_handle stmg_handle;

/* Build the level hierarchy, smoother factors, relaxation parameters and the
 * coarse-level inverse (Section 3; Alg. mg-sequence: p- then h-levels, then,
 * with time_mg, k- and tau-levels on the coarsest spatial mesh).
 * vertices: host, nullable.  NULL means a Cartesian box [lo, hi]; otherwise
 *   (n_cells+1)^dim vertex positions, x fastest, dim doubles each.  Cells must
 *   not be inverted (STMG_E_ARG otherwise).
 * coeff: host, one positive coefficient per finest cell (rho of eqs. heat and
 *   wave), x fastest; NULL means 1 everywhere.
 * hip_stream: a hipStream_t (NULL = default stream).
 * The local eigenpairs of the smoother are checked after the batched solve and
 * the solve is repeated (stmg_info.eig_resolves) when a cell fails; STMG_E_HIP
 * if a cell still fails after three solves.
 * out: receives the handle; unchanged on failure. Synchronous. */
stmg_status stmg_create(const stmg_config* cfg, const double* vertices, const double* coeff,
                        void* hip_stream, stmg_handle** out);

/* y = S_level x (eq. lin-sys on that level), identity on Dirichlet nodes.
 * dtype 0: x, y double; dtype 1: float.  x and y must not alias. */
stmg_status stmg_vmult(stmg_handle* h, int level, int dtype, const void* x, void* y);

/* Bytes of the static per-device scratch used by stmg_vmult_noalloc. */
#define STMG_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): y = S_level x as stmg_vmult defines it, computed on
 * the per-cell path (each cell's contribution to its own slot, then a node gather in a fixed cell
 * order) with the slots in a static device array of STMG_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends.  The call allocates nothing.
 * Limit: the level's slots, ncells * n_t * (p+1)^dim values of dtype, must fit in
 * STMG_SCRATCH_BYTES; a larger level is rejected with STMG_E_UNSUPPORTED.
 * Every call on one GPU uses that GPU's one array: calls that overlap on a GPU (several streams or
 * host threads) race and give wrong results; calls on one stream are ordered.  x, y device
 * buffers as for stmg_vmult (must not alias).  Asynchronous on the handle's stream. */
stmg_status stmg_vmult_noalloc(stmg_handle* h, int level, int dtype, const void* x, void* y);

/* n_steps damped additive Schwarz steps (eq. vanka):
 * x <- x + omega_level * sum_T R_T^T [R_T S R_T^T]^{-1} R_T (b - S x),
 * blocks T = interior DoFs of one spatial cell x one time cell (eq. vanka0);
 * each Dirichlet DoF is its own identity block.  Requires the level's factors
 * for dtype (vcycle_dtypes); level must not be the coarsest. */
stmg_status stmg_smooth(stmg_handle* h, int level, int dtype, const void* b, void* x, int n_steps);

/* z = V(r): one V-cycle of Alg. stmg on the finest level with zero initial
 * guess, nu1 = nu2 = n_smooth, exact coarsest-level solve.  r, z must not alias. */
stmg_status stmg_vcycle(stmg_handle* h, int dtype, const void* r, void* z);

/* One iteration of the space-time multigrid method as a stationary solver (Alg. stmg applied
 * to the current residual, Section 3.1): r = b - S x, z = V r (one V-cycle, the settings of
 * stmg_vcycle), x <- x + z.  b, x, r, z: device vectors of level 0 in dtype, caller-owned,
 * pairwise distinct (STMG_E_ARG otherwise); x is updated in place, r and z are outputs (the
 * residual before the step and the correction).  dtype selects the hierarchy (FP64 or FP32)
 * the residual and the V-cycle run in.  Asynchronous on the handle's stream. */
stmg_status stmg_mg_step(stmg_handle* h, int dtype, const void* b, void* x, void* r, void* z);

/* fine = P coarse: prolongation from level+1 to level (Section 3.2): the coarse
 * Q_p function evaluated at the fine nodes (P^h (x) I on every temporal plane),
 * or, between two temporal levels, the coarse temporal trial functions at the
 * fine temporal DoF times (I (x) P^tau, stmg_info.n_t_level gives the sizes);
 * Dirichlet values of coarse are treated as zero and fine Dirichlet values are
 * written as zero. */
stmg_status stmg_prolongate(stmg_handle* h, int level, int dtype, const void* coarse, void* fine);

/* coarse = P^T fine (Section 3.2, restriction = adjoint of prolongation) on
 * interior nodes; coarse Dirichlet values are written as zero. */
stmg_status stmg_restrict(stmg_handle* h, int level, int dtype, const void* fine, void* coarse);

/* Solve S x = b with FP64 flexible GMRES(restart) right-preconditioned by one
 * V-cycle per iteration (Section 4 solver set-up; precision selects an FP64,
 * FP32 or learned+FP32 preconditioner).  b, x: device double vectors; x holds
 * the initial guess on entry.  Dirichlet entries of b and x are set to zero
 * (homogeneous data).  Returns STMG_E_NOCONV (with info filled) if rtol is
 * not reached within max_iter, STMG_E_NONFINITE for NaN/Inf.  Synchronous.
 * info may be NULL. */
stmg_status stmg_solve(stmg_handle* h, const double* b, double* x, stmg_solve_info* info);

/* Event-timed totals of the finest-level kernels, accumulated over stmg_solve calls:
 * the matrix-free operator (every finest-level operator launch: outer products,
 * residuals inside the V-cycle) and the smoother apply kernel. */
typedef struct {
  int64_t n_operator;       /* finest-level operator kernel launches */
  int64_t n_smoother;       /* finest-level smoother kernel launches */
  double t_operator;        /* summed kernel durations, seconds (hipEvents on the handle's stream) */
  double t_smoother;
} stmg_kernel_stats;

/* Copy the accumulated finest-level kernel statistics; reset != 0 clears them afterwards. */
stmg_status stmg_kernel_stats_get(stmg_handle* h, stmg_kernel_stats* out, int reset);

/* Select the preconditioner used by stmg_solve (stmg_precision); the matching
 * V-cycle data must have been built (vcycle_dtypes). */
stmg_status stmg_set_precision(stmg_handle* h, int precision);

/* Slab right-hand side (Sections 2.1-2.2; eqs. heat-cg-dg-at-once, heat-cg-cg-at-once,
 * wave-cg-dg-at-once, wave-cg-cg-at-once) with the coupling to the previous slab:
 *   heat dG : b = (M_T (x) I) F + (a (x) M_h) u0
 *   heat cGP: b = (M_T (x) I) F + (e_1 (x) beta) (x) F0 - (a (x) M_h + (e_1 (x) beta) (x) A_h) u0
 *   wave dG : b = (M_T (x) I) F + (a (x) M_h) v0 + (A_T M_T^{-1} a (x) M_h) u0
 *   wave cGP: b = (M_T (x) I) F + (e_1 (x) beta) (x) F0 - (a (x) M_h) v0 - ((e_1 (x) beta) (x) A_h) u0
 *             - (A_T M_T^{-1} a (x) M_h) u0 + (A_T M_T^{-1} (e_1 (x) beta) (x) M_h) v0
 * with a = e_1 (x) alpha (first time cell), A_h and M_h restricted to interior nodes, and b = 0
 * on Dirichlet nodes.  F: device FP64 [n_t][N_x] loads (f(., t_i), phi) at the temporal DoF
 * times (NULL reads as zero); F0: device FP64 [N_x] load at the slab start (cGP only);
 * u0, v0: device FP64 [N_x] displacement and velocity at the slab start (NULL reads as zero;
 * v0 is used by the wave problem only).  b: device FP64 [n_t][N_x], must not alias F.
 * Asynchronous on the handle's stream. */
stmg_status stmg_slab_rhs(stmg_handle* h, const double* F, const double* F0, const double* u0, const double* v0,
                          double* b);

/* Coordinates of the finest-level lattice nodes (Gauss-Lobatto nodes of every cell of a
 * Cartesian mesh): xyz host [N_x][dim], x fastest like the vectors; for setting initial
 * data by nodal interpolation.  STMG_E_UNSUPPORTED on meshes with displaced vertices. */
stmg_status stmg_node_coordinates(stmg_handle* h, double* xyz);

/* Point values of the Q_p interpolant of the first n_planes temporal planes of U (device
 * FP64 [n_t][N_x], finest level) at npts points pts (host [npts][dim]); out: host
 * [n_planes][npts].  Used for point goal quantities (Section 4.2).  Synchronises.
 * STMG_E_ARG for points outside the domain or n_planes outside 1..n_t; STMG_E_UNSUPPORTED on
 * meshes with displaced vertices. */
stmg_status stmg_point_values(stmg_handle* h, const double* U, int n_planes, int npts, const double* pts,
                              double* out);

/* Velocity of the wave slab from its displacement (Sections 2.1.2 and 2.2.2, eqs.
 * wave-cg-dg-ade and wave-cg-cg-ade; the second equation of the first-order system):
 *   dG(k):  V = M_T^{-1} (A_T U - a u0),    cGP(k): V = M_T^{-1} (A_T U + a u0 - b v0),
 * a = e_1 (x) alpha, b = e_1 (x) beta (first time cell only).  U, V: device FP64 [n_t][N_x]
 * on the finest level; u0, v0: device FP64 [N_x] initial displacement and velocity of the
 * slab (NULL reads as zero; v0 is not used by dG).  Asynchronous on the handle's stream.
 * STMG_E_UNSUPPORTED for the heat problem; STMG_E_ARG for NULL U / V or U == V. */
stmg_status stmg_wave_velocity(stmg_handle* h, const double* U, const double* u0, const double* v0, double* V);

/* ---- learned preconditioning stage (not part of the paper's method) ----------------
 * Network C(r) on a finest-level residual r ([n_t][N_x], FP64, 3D only):
 *   s = sqrt(mean(r^2)); h_0 = r / s (one channel per temporal DoF);
 *   h_l = relu(conv_l(h_{l-1})) for l < L, h_L = conv_L(h_{L-1});  C(r) = s h_L, zero on
 *   Dirichlet nodes (C(0) = 0).  conv_l: 3x3x3 taps on the node lattice with zero padding,
 *   conv(h)[co][v] = b[co] + sum_{tap, ci} W[tap][co][ci] h[ci][v + off(tap)],
 *   tap = dx + 3 (dy + 3 dz), off = (dx - 1, dy - 1, dz - 1).
 * Parameters: one FP32 vector, per layer W (27 * C_out * C_in, tap, then C_out, then C_in)
 * followed by b (C_out).  Activations BF16, products on BF16 matrix cores with FP32
 * accumulation.  With precision STMG_PREC_LEARNED, stmg_solve uses for an Arnoldi vector v
 *   z = C(v) + V(v - S C(v))       (V = FP32 V-cycle)
 * when plain multigrid accepts it, else z = V(v).  The stage is rejected when
 * ||v - S C(v)|| >= ||v||, when C(v) is not finite, or when ||v - S z|| exceeds the value
 * ||v' - S V(v')|| / ||v'|| of the last plain application (the first iteration of a solve
 * is plain).  After three rejections in a row the network is not evaluated again in that
 * solve.  info->cnn_used counts accepted stages, info->cnn_fallbacks the iterations that
 * used the plain V-cycle. */

/* Create (or replace) the network: n_layers in 1..6 convolutions, channels[0..n_layers]
 * with channels[0] = channels[n_layers] = n_t and every entry in 1..32.  Parameters start at 0. */
stmg_status stmg_cnn_create(stmg_handle* h, int n_layers, const int32_t* channels);
/* Number of FP32 parameters of the network. */
stmg_status stmg_cnn_param_count(stmg_handle* h, int64_t* n);
/* Copy n host FP32 parameters in (resets the Adam state) / out. Synchronous. */
stmg_status stmg_cnn_set_params(stmg_handle* h, const float* params, int64_t n);
stmg_status stmg_cnn_get_params(stmg_handle* h, float* params, int64_t n);
/* z = C(r) (device FP64 vectors of the finest level).  Synchronous (reads rms(r)). */
stmg_status stmg_cnn_forward(stmg_handle* h, const double* r, double* z);
/* grad (host, n floats) = d/dtheta sum(dz * C(r)) with s = rms(r) held fixed. Synchronous. */
stmg_status stmg_cnn_param_grad(stmg_handle* h, const double* r, const double* dz, float* grad, int64_t n);
/* One Adam step (beta = 0.9, 0.999, eps = 1e-8, rate lr) on L = ||C(r) - e||^2 / ||e||^2;
 * *loss receives L before the step (may be NULL).  Synchronous. */
stmg_status stmg_cnn_train_step(stmg_handle* h, const double* r, const double* e, double lr, double* loss);

/* Override the relaxation parameter of one level (omega > 0). */
stmg_status stmg_set_omega(stmg_handle* h, int level, double omega);

/* Sizes and parameters of the hierarchy. */
stmg_status stmg_query(stmg_handle* h, stmg_info* info);

/* Release all device memory of the handle; NULL is ignored. */
void stmg_destroy(stmg_handle* h);

/* Message of the last failing call on this thread ("" if none). */
const char* stmg_last_error(void);

/* Host only (no device work, no handle): the slab temporal matrices the library
 * builds (Sections 2.1-2.2; dG on right-Radau nodes, eq. dg-time-weights; cGP on
 * Gauss-Lobatto nodes with the last k test functions, eq. cg-time-weights).
 * problem 0 heat / 1 wave, method 0 dG / 1 cGP, k as in stmg_config, n_time_cells
 * time cells of length tau > 0.  n_t receives n_time_cells * (k + 1) (dG) or
 * n_time_cells * k (cGP).  M_T, A_T, N_T: host, row-major n_t x n_t, each written
 * when non-NULL (N_T = A_T for heat, A_T M_T^{-1} A_T for wave); cap is the
 * capacity of each in doubles.  STMG_E_ARG / STMG_E_UNSUPPORTED for invalid
 * parameters or cap < n_t * n_t (nothing written then). */
stmg_status stmg_temporal_matrices(int problem, int method, int k, int n_time_cells, double tau, int64_t cap,
                                   int32_t* n_t, double* M_T, double* A_T, double* N_T);

/* Host only: the 1D factor of the spatial prolongation along one axis (Section
 * 3.2: the coarse Q_p function evaluated at the fine Gauss-Lobatto nodes; the
 * prolongation on a tensor lattice is the Kronecker product of the axis factors,
 * applied to every temporal plane), from p_coarse on n_coarse cells to p_fine on
 * n_fine cells of the same interval, as the level transfers use it: rows and
 * columns of the two Dirichlet end nodes are zero.  Requires p_coarse <= p_fine
 * and n_coarse dividing n_fine.  rows, cols receive p_fine n_fine + 1 and
 * p_coarse n_coarse + 1; P (host, row-major, capacity cap doubles) is written
 * when non-NULL. */
stmg_status stmg_transfer_1d(int p_coarse, int n_coarse, int p_fine, int n_fine, int64_t cap, int32_t* rows,
                             int32_t* cols, double* P);

/* Host only: the temporal factors of the smoother's local blocks (Section 3.3,
 * eq. vanka0: every time cell of the slab has the same block M_tau (x) A_KK +
 * N~ (x) M_KK, with M_tau and N~ the diagonal time-cell blocks of M_T and N_T).
 * Arguments as for stmg_temporal_matrices, for one time cell of length tau;
 * nt_cell receives k + 1 (dG) or k (cGP); M_tau, N_tilde: host, row-major
 * nt_cell x nt_cell, written when non-NULL (capacity cap doubles each). */
stmg_status stmg_temporal_cell_factors(int problem, int method, int k, double tau, int64_t cap, int32_t* nt_cell,
                                       double* M_tau, double* N_tilde);

/* Host only: the times of a slab's temporal DoFs (Sections 2.1 and 2.2): time cell m of
 * length tau starts at t0 + m tau, and its DoFs sit at the k+1 right Radau points (dG) or at the
 * last k of the k+1 Gauss-Lobatto points (cGP) of the cell.  Arguments and checks as for
 * stmg_temporal_matrices; t0 must be finite.  n_t receives the number of DoFs; times (host,
 * capacity cap doubles, DoF order of the slab vectors) is written when non-NULL. */
stmg_status stmg_temporal_dof_times(int problem, int method, int k, int n_time_cells, double tau, double t0,
                                    int64_t cap, int32_t* n_t, double* times);

/* Host only: the temporal prolongation between two discretisations of one slab
 * of length slab_length (Section 3.2: the coarse trial functions evaluated at
 * the fine DoF times; restriction is its transpose), as used between temporal
 * levels with time_mg.  The coarse space must lie in the fine one:
 * k_coarse <= k_fine and c_coarse divides c_fine (STMG_E_ARG otherwise).  rows,
 * cols receive the fine and coarse n_t; P (host, row-major rows x cols, capacity
 * cap doubles) is written when non-NULL. */
stmg_status stmg_temporal_prolongation(int problem, int method, int k_fine, int c_fine, int k_coarse, int c_coarse,
                                       double slab_length, int64_t cap, int32_t* rows, int32_t* cols, double* P);

#ifdef __cplusplus
}
#endif
#endif /* STMG_H */
