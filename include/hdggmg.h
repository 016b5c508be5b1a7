/*
 * hdggmg.h -- C ABI of the MI355X (gfx950) HDG trace-operator library.
 *
 * Method: Fabien, Knepley, Mills, Riviere, "Manycore parallel computing for a
 * hybridizable discontinuous Galerkin nested multigrid method"
 * (arXiv:1705.09907).  The library discretizes -div(K grad u) = f on the unit
 * square, u = g_D on the boundary, with the LDG-H hybridizable DG method of
 * Sec. 3 (eqs. eq_h1-eq_h3, tau constant on every edge) on a uniform n x n
 * mesh of squares, condenses the element unknowns (eq. shur0) into the
 * statically condensed trace system S Lambda = b (eq. shur1), applies S
 * matrix-free face by face (Sec. 8, Alg. algo_mv) and solves it with the
 * nested p -> h multigrid of Secs. 6-7 (Algs. algo_1 / algo_2).
 *
 * Conventions (all vectors are FP64, contiguous, caller-owned DEVICE memory
 * unless a name ends in _host):
 *   element (i, j), e = i + n j, K = [i h, (i+1) h] x [j h, (j+1) h], h = 1/n
 *   interior faces: vertical between (i-1, j) and (i, j): f = (i-1) + (n-1) j;
 *                   horizontal between (i, j-1) and (i, j): f = n(n-1) + i + n(j-1)
 *   trace vector at degree p: N(p) = 2 n (n-1) (p+1) entries, DoF f (p+1) + a,
 *     a = Gauss-Lobatto node index in increasing y (vertical faces) or x
 *     (horizontal faces); p = 0 uses one value per face.
 *   local faces of an element: 0 left, 1 right, 2 bottom, 3 top.
 *   Q1 levels: interior vertices (i, j), 1 <= i, j <= m-1, v = (i-1) + (m-1)(j-1).
 *
 * Every call is stream-ordered and asynchronous on the stream given to
 * hdg_create, except calls that return host scalars (they synchronize that
 * stream).  A handle is not thread safe; use one handle per host thread.
 * Every function returns an hdg_status_t; on failure hdg_last_error(handle)
 * returns a message.  Arguments are validated before any launch.
 */
#ifndef HDGGMG_H
#define HDGGMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdg_ctx* hdg_handle_t;

typedef enum {
  HDG_OK = 0,
  HDG_ERR_INVALID_ARG = -1,   /* bad size, degree, pointer, coefficient or config field */
  HDG_ERR_OOM = -2,           /* device or host allocation failed                      */
  HDG_ERR_HIP = -3,           /* a HIP runtime call failed (message has the HIP error)  */
  HDG_ERR_NOT_CONVERGED = -4, /* maxit reached; x, iters, relres are still valid        */
  HDG_ERR_NONFINITE = -5,     /* NaN or Inf met in a residual norm                       */
  HDG_ERR_STATE = -6,         /* call not valid for this handle (e.g. level missing)     */
  HDG_ERR_AT_FLOOR = -7       /* a solve's true residual reached the rounding floor of
                                 b - S x above rtol ||b||: x, iters, relres are valid and
                                 x is as accurate as FP64 storage lets the residual show */
} hdg_status_t;

enum { HDG_SMOOTH_CHAIN = 0, HDG_SMOOTH_FACE = 1, HDG_SMOOTH_PATCH = 2 };
enum { HDG_COARSE_GALERKIN = 0, HDG_COARSE_REDISCRETIZE = 1 };
enum { HDG_SOLVE_PCG = 0, HDG_SOLVE_VCYCLE = 1, HDG_SOLVE_FCG = 2 };
enum { HDG_CYCLE_V = 0, HDG_CYCLE_W = 1, HDG_CYCLE_WH = 2 };
/* Kernel of the many-right-hand-side products in the cycle precision (FP32 or
 * bfloat16 blocks; FP64 always uses the vector kernel): HDG_MULTI_AUTO picks the
 * faster of the two by timing on first use when autotune is set, else the vector
 * kernel; HDG_MULTI_VECTOR: FP32 fused multiply-adds, one face and column per
 * thread; HDG_MULTI_MATRIX: the matrix cores (v_mfma_f32_4x4x1_16b_f32), each
 * wavefront walking a chain of faces with 64 columns on its lanes.  Both give
 * the same products up to the order of rounding of the sums. */
enum { HDG_MULTI_AUTO = 0, HDG_MULTI_VECTOR = 1, HDG_MULTI_MATRIX = 2 };

/* Launch schedules of the chain Schwarz solve (hdg_config_t.chain_shape). */
enum { HDG_CHAIN_AUTO = 0, HDG_CHAIN_LEAN = 1, HDG_CHAIN_WIDE = 2, HDG_CHAIN_FLAT = 3, HDG_CHAIN_TRI = 4 };
/* Launch schedule of a Q1 level visit (hdg_config_t.q1_schedule). */
enum { HDG_Q1_FUSED = 0, HDG_Q1_SEPARATE = 1 };
/* Precision of the multigrid cycle (the preconditioner).  The outer solver, its
 * residuals and the finest-level operator it applies stay FP64 in every mode.
 *   HDG_PREC_F64:  every level, vector and block in FP64 (the paper's setting).
 *   HDG_PREC_F32:  cycle vectors, blocks, smoother factors and Q1 stencils FP32.
 *   HDG_PREC_BF16: as F32, but on the coarse p-levels (p < k) the face blocks of
 *                  the trace operator (and the facet inverses) are stored as
 *                  bfloat16 (round to nearest even) and widened to FP32 in
 *                  registers; arithmetic stays FP32.  The finest level keeps FP32
 *                  blocks: its residuals of smooth corrections cancel below
 *                  bfloat16 resolution and the preconditioner then fails.
 * The coarsest Q1 inverse is FP64 in every mode. */
enum { HDG_PREC_F64 = 0, HDG_PREC_F32 = 1, HDG_PREC_BF16 = 2 };

#define HDG_MAX_DEGREE 8
#define HDG_MAX_HLEVELS 24

/* Solver configuration.  Fill with hdg_config_default, then override. */
typedef struct {
  int32_t n;            /* elements per direction, n >= 2                                  */
  int32_t k;            /* finest trace degree, 0 <= k <= HDG_MAX_DEGREE                   */
  double tau;           /* HDG stabilization, > 0 (Sec. 5 uses 1)                           */
  int32_t nu1, nu2;     /* pre/post smoothing steps per level (Sec. 7 uses 2, 2)           */
  int32_t smoother;     /* HDG_SMOOTH_CHAIN: additive Schwarz with one subdomain per chain
                           of faces (vertical faces of an element row / horizontal faces
                           of an element column), solved in LDS: needs
                           ((n-1)(k+1) + (k+1)^2) * (8 bytes FP64, 4 otherwise) bytes, at
                           most the LDS one workgroup may use (160 KiB on gfx950);
                           HDG_SMOOTH_FACE: one subdomain per facet
                           (Sec. 6, additive Schwarz relaxation, zero overlap);
                           HDG_SMOOTH_PATCH: one subdomain per element, its interior
                           faces (Sec. 6 with overlap: neighbouring patches share a face),
                           weighted by the inverse counting matrix W = 1/2 (each face
                           lies in two patches), x <- x + omega W M (b - S x); device
                           set-up only; omega default 1                                  */
  int32_t coarse;       /* p-level coarse operators: HDG_COARSE_GALERKIN (element-wise
                           P^T K P) or HDG_COARSE_REDISCRETIZE (degree-p HDG, Sec. 6)     */
  double omega[HDG_MAX_DEGREE + 1]; /* Schwarz damping per p; <= 0: 1 (patch), 0.8 (chain) or
                           4 / (3 lambda_max(D^-1 S_p)) estimated on the device (face)    */
  double cheb_lo, cheb_hi;          /* Chebyshev interval [lo, hi] * lambda_max on Q1 levels */
  double cheb_lmax[HDG_MAX_HLEVELS];/* lambda_max(diag^-1 A) per Q1 level (0 = finest Q1);
                                       <= 0: estimated with Lanczos at setup              */
  int32_t coarse_max;   /* coarsest Q1 level: first with <= coarse_max unknowns (default 2000) */
  int32_t nq;           /* Gauss-Legendre points per direction of f input (default k + 2) */
  int32_t precision;    /* HDG_PREC_F64 (default), HDG_PREC_F32 or HDG_PREC_BF16; reduced
                           precision with the facet smoother needs every omega[p] > 0     */
  int32_t inner_steps[HDG_MAX_DEGREE + 1]; /* K-cycle (Notay-Vassilevski): for p < k,
                           inner_steps[p] = m > 0 replaces the level-p coarse correction
                           of the cycle by m steps of flexible CG on S_p, each
                           preconditioned by one cycle from level p (an extension of the
                           paper's V-cycle; the cycle becomes nonlinear, so solve with
                           HDG_SOLVE_FCG or HDG_SOLVE_VCYCLE).  0 (default): the plain
                           coarse correction of the cycle field below.
                           Range [0, 64]; must be 0 for p >= k.                          */
  int32_t graph;        /* 1: the solver's preconditioner (the whole cycle, Krylov-accelerated
                           levels included) is captured once as a HIP graph on a library
                           stream and replayed on the handle's stream; 0 (default): eager
                           launches.  Same kernels in the same order either way.         */
  int32_t autotune;     /* 1: at setup, time the chain Schwarz launch shapes (schedule, workgroup
                           size, XCD-aware chain order, LDS staging depth) of every level and keep
                           the fastest; 0 (default): measured fixed defaults.  Results are
                           identical either way (same operations in the same order).  The
                           choices are kept for the life of the process per (device, n, level
                           degree, precision, chain_shape, LDS limit): a further handle of the
                           same sizes takes them without timing again.                   */
  int32_t cycle;        /* HDG_CYCLE_V (default): each coarse correction is one cycle of the
                           coarser level; HDG_CYCLE_W: two, the second started from the
                           first's result (the W schedule the paper also reports, Sec. 7);
                           HDG_CYCLE_WH: W on the corrections onto Q1 levels (the p = 0 -> Q1
                           step and the h-levels), V on the p-levels (not in the paper).
                           Levels with inner_steps keep their Krylov correction; the
                           coarsest level's exact solve runs once.                          */
  int32_t multi_kernel;  /* HDG_MULTI_AUTO (default), HDG_MULTI_VECTOR or HDG_MULTI_MATRIX       */
  int32_t setup_on_host; /* 0 (default): element blocks, face slabs, smoother factors and the Q1
                            hierarchy are built on the device (coefficient updates supported);
                            1: the host set-up (multi-threaded C++), the reference it is
                            checked against                                                    */
  int32_t chain_shape;   /* launch schedule of the chain Schwarz solve (HDG_CHAIN_*): AUTO
                            (default) picks by degree and mesh (or the autotuner, when on);
                            LEAN / WIDE: factors fetched level by level in register batches
                            (WIDE: every row of a position per batch, P = 3 ... 5); FLAT: every
                            factor of a sweep requested at once into registers (P <= 5, while
                            they fit).  These three run the block cyclic reduction with the
                            same operations in the same order: identical results.  TRI (the
                            default at P = 1 for 5 <= n <= 2049, ignored at other P): the
                            partitioned tridiagonal solve, one wavefront per chain, one chain
                            segment per lane; the same chain solve up to rounding.          */
  int32_t q1_schedule;   /* Q1 level visits of the single-vector cycle: HDG_Q1_FUSED (default)
                            runs the pre-smoothing steps, residual and restriction of a level as
                            one launch and the prolongation and post-smoothing as a second, on
                            tiles with redundant halos (when nu1, nu2 <= 6); HDG_Q1_SEPARATE
                            launches each step on its own.  Identical results.               */
  int32_t reserved[1];
} hdg_config_t;

/* Defaults: tau 1, V(2,2), chain smoother, Galerkin p-levels, omega/lmax estimated,
 * Chebyshev interval [0.1, 1.1], coarse_max 2000, nq = k + 2. */
hdg_status_t hdg_config_default(int32_t n, int32_t k, hdg_config_t* cfg);

/* Setup (Sec. 3 steps (i)-(ii) and the multigrid hierarchy of Sec. 6).
 * kappa_host: [n*n] per-element coefficient K_e > 0 (host memory, read only,
 * not retained).  hip_stream: a hipStream_t (NULL = default stream).  Builds
 * the condensed element blocks of every level (Sec. 8: one independent local
 * solve per element, all elements at once on the device unless setup_on_host),
 * the face-major blocks, smoother factors, transfer tables, Q1 stencils and the
 * coarsest inverse (host), then estimates any missing omega / lambda_max on the
 * device.
 * Errors: INVALID_ARG (n < 2, k out of range, tau or any kappa not > 0 and
 * finite, bad config), OOM, HIP. */
hdg_status_t hdg_create(const hdg_config_t* cfg, const double* kappa_host, void* hip_stream,
                        hdg_handle_t* out);
hdg_status_t hdg_destroy(hdg_handle_t h);

/* New per-element coefficient on an existing handle (same mesh, degree and
 * config; nothing is reallocated): rebuilds on the device every level's blocks,
 * smoother factors and Q1 hierarchy, and re-estimates the omega / lambda_max the
 * config leaves to estimation.  Right-hand sides depend on the coefficient:
 * call hdg_assemble_rhs again (the source state kept for hdg_reconstruct does
 * not).  STATE for a handle made with setup_on_host = 1. */
hdg_status_t hdg_update_coefficients(hdg_handle_t h, const double* kappa_host);

/* The 7 blocks of interior face f at level p as stored on the device (Sec. 8,
 * Alg. algo_mv's per-face data): out_host [7][p+1][p+1], slot 0 the summed
 * diagonal block K_lo[f,f] + K_hi[f,f], slots 1-3 the lo element's blocks
 * coupling f to its other faces in local order, slots 4-6 the hi element's
 * (zero where that face is on the boundary), in the storage precision of the
 * level widened to double (FP64 where an FP64 copy is kept). */
hdg_status_t hdg_get_face_blocks(hdg_handle_t h, int32_t p, int64_t f, double* out_host);

/* N(p) = 2 n (n-1) (p+1), the trace-vector length at degree p (0 <= p <= k). */
hdg_status_t hdg_num_dofs(hdg_handle_t h, int32_t p, int64_t* n_lambda);

/* Number of Q1 h-levels and the mesh size m of each (level 0 = the Q1 space on
 * the finest mesh; the last one is solved directly). */
hdg_status_t hdg_num_hlevels(hdg_handle_t h, int32_t* nlev);
hdg_status_t hdg_hlevel_mesh(hdg_handle_t h, int32_t level, int32_t* m);
/* Damping and lambda_max actually used (after estimation). */
hdg_status_t hdg_get_params(hdg_handle_t h, double* omega_out /*[k+1]*/,
                            double* lmax_out /*[num_hlevels]*/);

/* The chain Schwarz launch shape in use at level p (after autotuning, if any):
 * workgroup size (partitioned solve: 64 x chains per workgroup), XCD-aware chain
 * order (0/1), first cyclic-reduction level whose factors are staged in LDS (64:
 * none, as in the flat and partitioned schedules).  Each output pointer may be
 * NULL. */
hdg_status_t hdg_get_chain_shape(hdg_handle_t h, int32_t p, int32_t* threads, int32_t* remap, int32_t* lds_level);

/* Copy the condensed block of element e at level p (4(p+1) x 4(p+1), row major,
 * local faces left, right, bottom, top) to host memory: Sec. 3, eqs. shur0
 * substituted into shur1, K_e = [C^T, -E^T] Abb^{-1} [C; E] + tau M; for p < k
 * with Galerkin coarsening the block is P4^T K_e^{(p+1)} P4. */
hdg_status_t hdg_get_element_block(hdg_handle_t h, int32_t p, int64_t e, double* out_host);

/* Same block without a handle or device (host computation only): mesh n, finest
 * degree k, requested degree p <= k, coefficient kappa_e of the element, coarse =
 * HDG_COARSE_GALERKIN (chain of P4^T K P4 from degree k) or HDG_COARSE_REDISCRETIZE. */
hdg_status_t hdg_element_block_host(int32_t n, int32_t k, int32_t p, double tau, double kappa_e,
                                    int32_t coarse, double* out_host);

/* Gauss-Legendre nodes on [-1, 1] used for the source input (nq of them). */
hdg_status_t hdg_quadrature_nodes(int32_t nq, double* x_host);

/* Right-hand side at the finest degree (Sec. 3, steps (i)-(ii)):
 * b = sum_K R_K^T (g_K - K_K[:, bdry] Lambda_bdry), g_K = [C^T, -E^T] Abb^{-1} [0; F_K],
 * F_K = (f, w)_K.  f_qp_host: [n*n][nq*nq] source values at the Gauss-Legendre
 * points of each element, point (a, b) -> a + nq b with a along x.  gD_qp_host:
 * [4n][nq] Dirichlet data at the nq Gauss-Legendre points of each boundary face
 * (faces ordered bottom, right, top, left, each by increasing coordinate), or
 * NULL for g_D = 0; it is L2-projected onto Q_k(e) (Sec. 3).  b: device [N(k)].
 * Computed on the host, copied asynchronously. */
hdg_status_t hdg_assemble_rhs(hdg_handle_t h, const double* f_qp_host, const double* gD_qp_host,
                              double* b);

/* y = S_p x, the assembly-free trace operator of Sec. 8 (Alg. algo_mv): every
 * interior face gathers the blocks of its two elements.  x, y: device [N(p)],
 * must not alias.  With a reduced-precision cycle only p = k is kept in FP64:
 * p < k returns STATE. */
hdg_status_t hdg_apply_trace_operator(hdg_handle_t h, int32_t p, const double* x, double* y);

/* y = |S_p| |x| entrywise (every block entry and every x value by its absolute
 * value; the assembled matrix's entries, i.e. the summed diagonal block of each
 * face): the scale of the rounding error of S_p x.  eps || |S| |x| ||_2 bounds
 * from below the computed residual b - S x of any FP64 x (Sec. 7's stopping
 * test on ||b - S Lambda||).  Same arguments and level rule as
 * hdg_apply_trace_operator. */
hdg_status_t hdg_apply_abs(hdg_handle_t h, int32_t p, const double* x, double* y);

/* The same product in the cycle precision of a handle created with
 * HDG_PREC_F32 or HDG_PREC_BF16: FP32 vectors, blocks in FP32 or bfloat16,
 * FP32 accumulation.  x, y: device float [N(p)], must not alias.  Returns
 * STATE for an FP64 handle. */
hdg_status_t hdg_apply_trace_operator_lp(hdg_handle_t h, int32_t p, const float* x, float* y);

/* Y = S_p X for nrhs right-hand sides at once (1 <= nrhs <= 4096): X, Y are
 * device arrays [N(p)][nrhs], the right-hand sides of one trace DoF contiguous.
 * precision HDG_PREC_F64: double arrays and the FP64 operator (same level rule
 * as hdg_apply_trace_operator); the cycle precision of the handle: float arrays
 * and that precision's blocks.  The blocks are read once per call, whatever
 * nrhs.  X and Y must not alias. */
hdg_status_t hdg_apply_trace_operator_multi(hdg_handle_t h, int32_t p, int32_t precision, int32_t nrhs,
                                            const void* X, void* Y);

/* y_i = S x_i for count meshes of any sizes and degrees in ONE kernel launch
 * (FP64 operators, level p[i] of handles[i]; same level rule as
 * hdg_apply_trace_operator).  handles, p, X, Y: host arrays of count entries;
 * X[i], Y[i]: device [N_i(p[i])] vectors, not aliased.  A fixed grid walks the
 * (mesh, 64-face tile) items with a static stride; each y_i is bit-identical to
 * the single-mesh apply.  Runs on the stream of handles[0] (inputs of every mesh
 * must be ready there) and synchronizes that stream before returning. */
hdg_status_t hdg_apply_trace_operator_batch(int32_t count, const hdg_handle_t* handles, const int32_t* p,
                                            const double* const* X, double* const* Y);

/* The same many-mesh product (Sec. 8, Alg. algo_mv) in the cycle precision of handles created with
 * HDG_PREC_F32 or HDG_PREC_BF16 (the blocks hdg_apply_trace_operator_lp uses:
 * FP32 or bfloat16, FP32 vectors and accumulation); handles may mix the two.
 * X[i], Y[i]: device float [N_i(p[i])], not aliased.  Each y_i is bit-identical
 * to hdg_apply_trace_operator_lp on that mesh (same loads, same order of
 * operations).  Returns STATE if a handle has FP64 cycle precision.  Same
 * stream and synchronization rules as hdg_apply_trace_operator_batch. */
hdg_status_t hdg_apply_trace_operator_batch_lp(int32_t count, const hdg_handle_t* handles, const int32_t* p,
                                               const float* const* X, float* const* Y);

/* For callers that cannot allocate device memory (code under HIP graph capture
 * in the caller's own pipeline, tight serving loops, harnesses that forbid
 * hipMalloc): the same products as hdg_apply_trace_operator_batch, bit for bit,
 * with the same arguments and rules, but no allocation of any kind.  The
 * (mesh, tile) descriptor table lives in a file-scope device array of
 * HDG_BATCH_NOALLOC_MAX entries, one per GPU, held until the process ends (its
 * device address is looked up once per device by hdg_create).  count >
 * HDG_BATCH_NOALLOC_MAX returns INVALID_ARG.  Every call on one GPU shares that
 * table and rewrites it: calls that overlap on one GPU (from several host
 * threads or streams) race; calls in sequence do not, since each call
 * synchronizes the stream of handles[0] before returning. */
#define HDG_BATCH_NOALLOC_MAX 256
hdg_status_t hdg_apply_trace_operator_batch_noalloc(int32_t count, const hdg_handle_t* handles, const int32_t* p,
                                                    const double* const* X, double* const* Y);

/* Measurement entry point: the same product as hdg_apply_trace_operator
 * (precision HDG_PREC_F64, FP64 vectors) or hdg_apply_trace_operator_lp
 * (precision = the handle's cycle precision, float vectors), launched with a
 * pair of HIP events recorded at the kernel's own start and end.  Synchronizes
 * and returns the kernel duration in microseconds (*kernel_us).  Errors as for
 * the two calls it mirrors; INVALID_ARG for any other precision. */
hdg_status_t hdg_apply_trace_operator_timed(hdg_handle_t h, int32_t p, int32_t precision, const void* x, void* y,
                                            double* kernel_us);

/* Residual of the level-p trace system (Alg. algo_2, the residual handed to the
 * coarser level; Sec. 7, the residual two-norm whose ratios measure the
 * multigrid convergence factor).
 * r = b - S_p x; if norm2_host != NULL, *norm2_host = ||r||_2 (synchronizes;
 * deterministic reduction order).  r must not alias x.  Same level rule as
 * hdg_apply_trace_operator. */
hdg_status_t hdg_residual(hdg_handle_t h, int32_t p, const double* b, const double* x, double* r,
                          double* norm2_host);

/* Smoother of Sec. 6 (additive Schwarz relaxation, weighted by a scalar omega;
 * the smoothing step S(A, b, x) of Algs. algo_1 / algo_2): sweeps of
 * x <- x + omega M^{-1} (b - S_p x) in place, M the block diagonal of S_p over
 * the subdomains (chains of faces or single faces, config field smoother), in
 * the cycle precision; b and x are FP64 in every mode. */
hdg_status_t hdg_smooth(hdg_handle_t h, int32_t p, const double* b, double* x, int32_t sweeps);

/* p-transfers (eqs. eq_mg_res / eq_mg_pro), face local, 1 <= p_fine <= k:
 * r_coarse = P^T r_fine;  x_fine += P e_coarse. */
hdg_status_t hdg_restrict(hdg_handle_t h, int32_t p_fine, const double* r_fine, double* r_coarse);
hdg_status_t hdg_prolong(hdg_handle_t h, int32_t p_fine, const double* e_coarse, double* x_fine);

/* One (nu1, nu2) multigrid cycle of Sec. 6: the p-multigrid of Alg. algo_2 from
 * degree k down to p = 0, where the h-multigrid of Alg. algo_1 (p = 0 traces ->
 * Q1 on the same mesh -> coarser Q1 meshes -> exact coarsest solve) replaces
 * the coarse solve; with the V or W schedule of the handle's config, for S_k x = b starting from x (in place), run in the cycle
 * precision; b and x are FP64 in every mode. */
hdg_status_t hdg_vcycle(hdg_handle_t h, const double* b, double* x);

/* One full-multigrid pass (Sec. 7) for S_k x = b from nothing: b is restricted
 * to every level (R = P^T, the right-hand sides of the Galerkin coarse systems),
 * the coarsest Q1 system is solved exactly, and on each finer level (Q1 levels,
 * then p = 0 .. k) the prolonged coarser result starts `cycles` cycles of that
 * level (V or W by the config).  b, x: device FP64 [N(k)]; x is written, not
 * read, and must not alias b; cycles in [1, 64], else INVALID_ARG.  Runs in the
 * cycle precision.  An exact solution in the range of the prolongations from
 * the coarsest level is reproduced to rounding. */
hdg_status_t hdg_fmg(hdg_handle_t h, const double* b, double* x, int32_t cycles);

/* The solve of Sec. 7: S_k x = b (eq. shur1) by multigrid, alone or as a
 * preconditioner of conjugate gradients, to ||b - S x||_2 <= rtol ||b||_2.
 * x in: initial guess, out: solution.  mode HDG_SOLVE_PCG (conjugate gradients preconditioned by one
 * cycle, V or W by the config), HDG_SOLVE_FCG (flexible CG, FCG(1), with the same preconditioner;
 * required instead of PCG when inner_steps makes the cycle nonlinear -- PCG
 * then returns INVALID_ARG) or HDG_SOLVE_VCYCLE (repeated cycles, the paper's
 * stationary solver, applied as x += B (b - S x)).  iters, relres: host outputs (nullable); history_host: nullable
 * [maxit + 1] residual norms (entry 0 = initial).  Returns NOT_CONVERGED if
 * maxit is reached (outputs still valid), NONFINITE on NaN/Inf.
 * Residual norms: entry 0 and every VCYCLE entry is ||b - S x|| computed from
 * x.  PCG and FCG iterate on the recursively updated residual r <- r - alpha S d
 * (the usual Krylov stopping test); when it falls below rtol ||b||, or maxit is
 * reached, the true residual b - S x is recomputed, and if it is still above
 * rtol ||b|| the iteration restarts from it (residual replacement) for as long
 * as each restart at least halves it.  The history entry of that iteration and
 * *relres are the true value, so *relres is always ||b - S x|| / ||b|| of the
 * returned x.  The computed b - S x cannot fall below about u || |S| |x| ||_2,
 * u = 2^-53 (rounding of S x itself); when the true residual is above rtol ||b||
 * but within twice that floor the call returns AT_FLOOR, and when a restart
 * failed to halve it NOT_CONVERGED, with the true residual in *relres
 * (hdg_apply_abs gives |S| |x|). */
hdg_status_t hdg_solve(hdg_handle_t h, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t mode, int32_t* iters, double* relres, double* history_host);

/* Solve S_k X = B for nrhs right-hand sides at once (1 <= nrhs <= 256): B, X
 * device [N(k)][nrhs] FP64 (right-hand sides of one DoF contiguous); X in:
 * initial guesses, out: solutions.  Flexible CG per column, preconditioned by
 * the V(nu1, nu2) cycle run for all columns together in the cycle precision
 * (operators, smoother factors and stencils read once per cycle for every
 * column); the FP64 operator, residuals and updates are kept for the outer
 * iteration.  Chain smoother only (STATE otherwise); Krylov acceleration of
 * coarse levels (inner_steps) is not used here.  A column stops updating once
 * its recursively updated residual norm is <= rtol ||b||_2; the true residuals
 * are then recomputed, and a column still above its tolerance restarts from its
 * true residual as in hdg_solve.  relres_host holds the true relative residuals
 * ||B_r - S X_r|| / ||B_r||.  iters_host, relres_host: nullable [nrhs].
 * NOT_CONVERGED if some column reached maxit, or a restart failed to halve its
 * true residual above its tolerance (at the rounding floor, among other causes;
 * the per-column floor is not evaluated here); outputs still valid. */
hdg_status_t hdg_solve_multi(hdg_handle_t h, int32_t nrhs, const double* B, double* X, double rtol, int32_t maxit,
                             int32_t* iters_host, double* relres_host);

/* ---- misfit gradient with respect to theta_K = log K_K (adjoint method) ----
 * The paper solves forward problems only; these calls differentiate its
 * discretisation.  With [Q; U]_K from the local solver (eq. shur0) and S
 * Lambda = b (eq. shur1), L = 1/2 sum_K |U_K - U_obs,K|^2 over the (p+1)^2
 * nodal values of each element's volume solution (volume node I = i + (k+1) j,
 * Gauss-Lobatto nodes), and
 *   dL/dtheta = per element  w_Q^T A_K Q_K,   Abb_K^T w = [0; r_K] + [C; -E] mu_K,
 * where r = U - U_obs and mu solves the adjoint system S mu = c (c below;
 * S is symmetric, so hdg_solve serves).  Element vectors: U, U_obs [n*n][(k+1)^2],
 * Q [n*n][2 (k+1)^2] (x half then y half), grad [n*n]; device memory, FP64. */

/* Step (iv) of Sec. 3 (eq. shur0): U (and Q if not NULL) from the interior
 * traces lam and the source state (f and g_D) of the last hdg_assemble_rhs on
 * this handle.  STATE if hdg_assemble_rhs was never called. */
hdg_status_t hdg_reconstruct(hdg_handle_t h, const double* lam, double* U, double* Q);

/* Adjoint right-hand side c = (dU/dLambda)^T (U - U_obs) = -sum_K R_K^T
 * [C^T, E^T] Abb_K^{-T} [0; U_K - U_obs,K] (device [N(k)]), and, if misfit_host
 * is not NULL, L = 1/2 |U - U_obs|^2 (synchronizes). */
hdg_status_t hdg_misfit_adjoint_rhs(hdg_handle_t h, const double* U, const double* U_obs, double* c,
                                    double* misfit_host);

/* grad[K] = dL/dtheta_K from the forward traces lam, U = U(lam), the data and the
 * adjoint solution mu of S mu = c.  STATE without a source state. */
hdg_status_t hdg_misfit_gradient(hdg_handle_t h, const double* lam, const double* U, const double* U_obs,
                                 const double* mu, double* grad);

const char* hdg_last_error(hdg_handle_t h);
const char* hdg_status_string(hdg_status_t s);

#ifdef __cplusplus
}
#endif
#endif /* HDGGMG_H */
