/*
 * walklap.h -- C ABI of the MI355X walk-Laplacian library.
 *
 * The library evaluates, on one GPU, matrix functions of the walk generating
 * functions of Arrigo & Durastante, "Walk based Laplacians for modeling
 * diffusion on complex networks" (arXiv 2601.11338):
 *
 *   phi(A, c) = sum_k c_k q_k(A)                       (Sec. 3.2, Prop. "whe-we-converge")
 *   q_0 = I, q_1 = A, q_2 = A^2 - mu D,
 *   q_{k+1} = A q_k + mu (mu I - D) q_{k-1}            (eq. qrec; mu = 0: all walks,
 *                                                        mu = 1: nonbacktracking, eq. Br)
 *   w = phi 1              (walk degree / total communicability, Sec. 3.1)
 *   L = diag(w) - phi      (eq. f-laplacian, eq. weighted_laplacian)
 *   exp(-t L) U0           (diffusion, eq. diffusion_on_G_with_downweighted_walk)
 *   diag / trace estimates (Sec. 4.4, Alg. 1)
 *
 * with weights c_k = alpha^k (resolvent) or beta^k / k! (exponential), c_0 = 1.
 *
 * Conventions for every entry point:
 *  - Returns a wl_status; WL_OK = 0.  On failure a message is available from
 *    wl_last_error() (thread-local, valid until the next call on the thread).
 *    Arguments are validated before anything is enqueued; on a validation
 *    error nothing has been launched and no output has been written.
 *  - Pointers named d_* are DEVICE pointers on the context's device, owned by
 *    the caller, and must stay valid until the call returns (calls that return
 *    host scalars synchronise the context stream; the others are enqueued on
 *    it and complete in stream order).  Pointers without d_ are host memory.
 *  - Dense blocks are ROW-MAJOR n x b (the b values of one node contiguous),
 *    element type given by the precision of the object (float for WL_FP32,
 *    double for WL_FP64), base address 16-byte aligned.
 *  - Handles are created and destroyed by the library and reference counted: a
 *    graph or network keeps its context alive and an operator keeps its graph
 *    alive, so handles may be destroyed in any order (each exactly once).
 *  - Workspace (Krylov bases, recurrence buffers, reduction partials) is
 *    allocated by the library on the device and kept in the operator or graph
 *    for reuse; WL_ENOMEM if it cannot be allocated.  The _ws variants of the
 *    evaluation calls take caller-provided workspace instead (wl_workspace_size).
 */
#ifndef WALKLAP_H
#define WALKLAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WL_OK = 0,
  WL_EINVAL = 1,        /* invalid argument (null pointer, bad size, malformed graph) */
  WL_ERANGE = 2,        /* parameter outside the convergence region (alpha * rho(Z_mu) >= 1),
                           or a size beyond the supported range (wl_graph_check_size) */
  WL_ENOMEM = 3,        /* device allocation failed */
  WL_EDEVICE = 4,       /* HIP runtime error, or no usable device */
  WL_ENOTSPD = 5,       /* an operator that must be positive definite is not */
  WL_ENOCONV = 6,       /* an iteration did not reach its tolerance */
  WL_ENUMERIC = 7,      /* NaN or Inf in a result */
  WL_EUNSUPPORTED = 8,  /* valid request this build does not handle */
  WL_EINTERNAL = 9
} wl_status;

typedef enum { WL_F_RESOLVENT = 0, WL_F_EXP = 1, WL_F_LINEAR = 2 } wl_func;
typedef enum { WL_FP32 = 4, WL_FP64 = 8 } wl_prec;
typedef enum {
  WL_M_AUTO = 0,        /* exponential: recurrence; resolvent: block Lanczos on A_mu */
  WL_M_RECURRENCE = 1,  /* truncated series by the fused three-term recurrence (exponential) */
  WL_M_LANCZOS = 2,     /* block Lanczos (mu = 0: on A; resolvent: on A_mu(alpha)) */
  WL_M_ARNOLDI = 3,     /* exponential, any mu: block Arnoldi on the 2n x 2n linearisation Z
                           (eq. Zdef), phi X = X + [I O] beta phi_1(beta Z) [q_1 X; q_2 X]
                           (Prop. "whe-we-converge"); krylov_dim Arnoldi steps (required).
                           For beta rho(Z) large, where the series degree grows with it. */
  WL_M_AMG_CG = 4       /* resolvent, WL_FP64: phi X = (1 - mu^2 alpha^2) A_mu(alpha)^{-1} X by
                           conjugate gradients on the deformed Laplacian (eq. deformed, an
                           M-matrix) preconditioned with an aggregation multigrid V-cycle
                           (Sec. 4.2; see wl_amg_info); tol = relative residual of every
                           column (0: 1e-9, Sec. 5.3), krylov_dim = iteration limit (0: 1000;
                           WL_ENOCONV beyond it). */
} wl_method;
typedef enum { WL_PROBE_GAUSS = 0, WL_PROBE_RADEMACHER = 1 } wl_probe_law;
typedef enum {
  WL_EST_HUTCHINSON = 0,
  WL_EST_BKS = 1,
  WL_EST_XNYS = 2,
  WL_EST_SURROGATE = 3  /* wl_diag_est only: Hutchinson on phi - G, G the degree-3 series */
} wl_estimator;

/* Graph flags */
#define WL_GRAPH_COPY 1u      /* library copies the CSR arrays (else it borrows them) */
#define WL_GRAPH_VALIDATE 2u  /* check sortedness, range, loops, duplicates, symmetry on device */

typedef struct wl_ctx wl_ctx;
typedef struct wl_graph wl_graph;
typedef struct wl_op wl_op;
typedef struct wl_mlp wl_mlp;

/* Operator description.
 *   mu          backtrack downweighting in [0, 1]; each backtracking step of a walk is
 *               weighted by theta = 1 - mu (Sec. 3.2).  mu = 0 all walks, mu = 1 NBT.
 *   func        WL_F_RESOLVENT (c_k = param^k) or WL_F_EXP (c_k = param^k / k!), or
 *               WL_F_LINEAR: f(x) = x (c_1 = 1, c_k = 0 for k >= 2; c_0 = 1 as always),
 *               so phi = I + A, w = 1 + d and L = D - A, the standard graph Laplacian
 *               that the paper's Laplacians reduce to (param ignored; recurrence only).
 *   param       alpha (resolvent; must satisfy alpha * rho(Z_mu) < 1, Prop. "whe-we-converge"
 *               and its remark) or beta (exponential; inverse temperature, Sec. 4.1.2).
 *   prec        WL_FP32 or WL_FP64: element type of vectors; all Krylov / recurrence
 *               coefficients and inner products are accumulated in double.
 *   krylov_dim  recurrence degree (exponential) or number of block Lanczos steps;
 *               0 = choose from tol.
 *   tol         relative accuracy target used when krylov_dim = 0 (tail bound of the
 *               series, or Lanczos a-posteriori estimate).
 *   method      wl_method.
 *   reorth      0: three-term recurrence only; 1: second local Gram-Schmidt pass
 *               against the two previous blocks; 2: full reorthogonalisation.
 *   rho_hint    if > 0, rho(Z_mu) supplied by the caller (skips its computation);
 *               used to validate alpha.                                               */
typedef struct wl_op_desc {
  double mu;
  int32_t func;
  double param;
  int32_t prec;
  int32_t krylov_dim;
  double tol;
  int32_t method;
  int32_t reorth;
  double rho_hint;
} wl_op_desc;

/* ---------------------------------------------------------------- errors / version */
const char* wl_last_error(void);
const char* wl_status_string(wl_status s);
int32_t wl_version(void);

/* ---------------------------------------------------------------- context
 * device: HIP device ordinal.  stream: a hipStream_t to enqueue on (NULL = the null
 * stream).  The context never destroys a caller's stream.                          */
wl_status wl_ctx_create(int32_t device, void* stream, wl_ctx** out);
wl_status wl_ctx_set_stream(wl_ctx* ctx, void* stream);
wl_status wl_ctx_synchronize(wl_ctx* ctx);
wl_status wl_ctx_destroy(wl_ctx* ctx);

/* Opt-in live timing of kernel classes on the context stream (HIP events around every
 * launch of the class) with the algorithmic bytes each launch must move (CSR once,
 * the gathered block once, every row-aligned input / output block once).  Turning
 * profiling on or off clears the statistics.  Classes: 0 fused recurrence step of one
 * operator (degree >= 2, b >= 4), 1 block Lanczos operator product (b >= 4), 2 other
 * sparse products, 3 side-by-side series step (wl_multi_*, width >= 32), 4 side-by-side
 * Lanczos operator product (wl_multi_*, width >= 32), 5 finest-level products of the
 * multigrid-preconditioned CG (WL_M_AMG_CG).  Batched steps count as class 0.           */
wl_status wl_ctx_set_profiling(wl_ctx* ctx, int32_t on);
wl_status wl_ctx_kernel_stats(wl_ctx* ctx, int32_t kernel_class, int64_t* launches, double* total_ms,
                              double* alg_bytes);
/* With the environment variable WL_TRACE set (and not "0") when a context is created,
 * profiling stays on for the context's life and wl_ctx_destroy prints every class's
 * launches, time and algorithmic GB/s to stderr.                                      */

/* wl_ctx_set_checks: result checks of the context's calls.  WL_CHECK_FINITE scans the
 * outputs of wl_fdeg, wl_apply_phi, wl_apply_L and wl_expv (and their _ws / _noalloc
 * forms) for NaN or Inf once the call's work is done: WL_ENUMERIC names the count.  The
 * scan reads every output once and synchronises the stream (not for code under graph
 * capture).  Enabling it allocates a small counter; flags = 0 turns checks off.        */
#define WL_CHECK_FINITE 1u
wl_status wl_ctx_set_checks(wl_ctx* ctx, uint32_t flags);

/* wl_test_fail_alloc: test hook for the failure paths.  The k-th device allocation the
 * library makes from now on (k = 0: the next one) fails as an out-of-memory would
 * (the call returns WL_ENOMEM, the handles stay usable); one allocation fails, then
 * the hook is off again.  k < 0 turns it off.  The environment variable
 * WL_TEST_FAIL_ALLOC=k sets the same when the library first allocates.  Process-wide;
 * for tests only.                                                                       */
wl_status wl_test_fail_alloc(int64_t k);

/* ---------------------------------------------------------------- graph (Sec. 2)
 * A simple undirected unweighted graph as symmetric CSR: d_rowptr (n+1 int32),
 * d_colidx (nnz int32), columns strictly increasing within a row, no self loops,
 * every edge stored in both directions (Definition "adjacency"; simple graphs,
 * Sec. 2).  Sizes as wl_graph_check_size (WL_ERANGE beyond them).  With
 * WL_GRAPH_VALIDATE the structure is checked on the device (WL_EINVAL with the
 * first violation).  Degrees d = A 1 are computed on the device.  The row split
 * used by the SpMM kernels (rows above a degree threshold handled by whole
 * workgroups) is built here.
 *
 * Largest supported sizes of one CSR (a graph, or the concatenation of a batch):
 * n <= WL_MAX_ROWS and nnz <= WL_MAX_NNZ = 2^31 - 1 - 2^16 (int32 column indices; the
 * sparse-product kernels step a row's 32-bit index up to 2^16 past its end before the
 * loop test).  wl_graph_check_size returns WL_OK, WL_EINVAL (negative) or WL_ERANGE;
 * it is host only and runs without a device.  wl_graph_create and wl_batch_create
 * apply it before touching the device.                                           */
#define WL_MAX_ROWS 2147483646LL
#define WL_MAX_NNZ 2147418111LL
wl_status wl_graph_check_size(int64_t n, int64_t nnz);
wl_status wl_graph_create(wl_ctx* ctx, int64_t n, int64_t nnz, const int32_t* d_rowptr,
                          const int32_t* d_colidx, uint32_t flags, wl_graph** out);
wl_status wl_graph_info(const wl_graph* g, int64_t* n, int64_t* nnz, int32_t* max_degree);
wl_status wl_graph_destroy(wl_graph* g);

/* Y = A X for a row-major n x b block (b >= 1), element type by prec.  The raw
 * sparse product every Krylov step is built on (Sec. 4.1).                     */
wl_status wl_spmm(wl_graph* g, int32_t prec, const void* d_X, void* d_Y, int32_t b);

/* Choose the SpMM launch shape (lanes per row, long-row threshold) for (prec, b)
 * by timing candidates on this graph; the choice is kept in the graph.  Without
 * it a heuristic from the mean degree is used.  Enqueues and synchronises.     */
wl_status wl_autotune(wl_graph* g, int32_t prec, int32_t b);
/* The launch shape used for (prec, b): lanes per row (the kernel's row group size,
 * rounded up to a power of two >= the lanes one row segment needs) and the degree
 * above which a row gets a whole workgroup.  Either output may be NULL.           */
wl_status wl_graph_shape(wl_graph* g, int32_t prec, int32_t b, int32_t* lanes_per_row, int32_t* long_row_threshold);
/* Set the launch shape for (prec, b) explicitly (e.g. to give several graph handles
 * of one CSR the shape one of them was tuned to): lanes per row a power of two in
 * [1, 64] (raised to what one row segment needs), threshold >= 1 (raised to the
 * graph's minimum long-row degree).                                                */
wl_status wl_graph_set_shape(wl_graph* g, int32_t prec, int32_t b, int32_t lanes_per_row, int32_t long_row_threshold);

/* Largest adjacency eigenvalue lambda_max(A) = rho(A) by Lanczos (double).  Used
 * for beta ~ 1/rho(A) (Sec. 4.1.2).  tol: relative.                              */
wl_status wl_lambda_max(wl_graph* g, double tol, double* out);

/* rho(Z_mu) of the 2n x 2n linearisation Z = [[O, I], [mu (mu I - D), A]]
 * (eq. Zdef).  mu = 0 returns lambda_max(A).  For mu > 0 it is the reciprocal of
 * the smallest t > 0 at which A_mu(t) = (1 - mu^2 t^2) I - t A + t^2 mu D becomes
 * singular; located by bracketing + bisection on the smallest Lanczos Ritz value
 * of A_mu(t).  tol: relative.                                                     */
wl_status wl_spectral_radius(wl_graph* g, double mu, double tol, double* rho);

/* ---------------------------------------------------------------- operator */
wl_status wl_op_create(wl_graph* g, const wl_op_desc* desc, wl_op** out);
wl_status wl_op_destroy(wl_op* op);
/* The truncation degree (recurrence) or number of block Lanczos steps the operator
 * settled on, and its method (WL_M_RECURRENCE, WL_M_LANCZOS or WL_M_ARNOLDI).  Either output may
 * be NULL.                                                                        */
wl_status wl_op_info(const wl_op* op, int32_t* degree_or_steps, int32_t* method);

/* w = phi 1 (n values): total communicability t(f) (Sec. 3.1) and the diagonal of
 * the walk Laplacian's degree part (eq. weighted_laplacian).  Includes c_0 = 1.
 * Cached in the operator after the first call.                                   */
wl_status wl_fdeg(wl_op* op, void* d_w);

/* Y = phi X (n x b).                                                              */
wl_status wl_apply_phi(wl_op* op, const void* d_X, void* d_Y, int32_t b);

/* Y = L X = w * X - phi X (eq. f-laplacian / eq. weighted_laplacian), never
 * forming L (Sec. 4.1).                                                           */
wl_status wl_apply_L(wl_op* op, const void* d_X, void* d_Y, int32_t b);

/* Y_i = exp(-t_i L) U0 for i < nt (eq. diffusion_on_G_with_downweighted_walk; L is
 * symmetric so the row-vector form is the transpose).  One block Lanczos basis of
 * dimension outer_dim on L serves every t_i (as the parfor of Alg. 1 shares one
 * basis).  d_Y: host array of nt device pointers, each n x b.  err_est (host, nt,
 * may be NULL): a-posteriori estimate || B_K E_K^T exp(-t T) E_1 R_0 ||_F.        */
wl_status wl_expv(wl_op* op, const void* d_U0, int32_t b, const double* t, int32_t nt,
                  void* const* d_Y, int32_t outer_dim, double* err_est);

/* ---------------------------------------------------------------- caller workspace
 * The evaluation is matrix-vector products only (Sec. 4.1), so its memory is a fixed
 * set of blocks known before the call: Krylov bases ((K + 1) blocks of n x b),
 * recurrence buffers (two n x b blocks), small FP64 matrices and reduction partials.
 * A caller that plans its own device memory asks for that size and passes one region:
 *
 * wl_workspace_size: *bytes = device workspace one call of kind `call`
 * (WL_CALL_APPLY_PHI, WL_CALL_APPLY_L or WL_CALL_EXPV with outer_dim) on op with
 * block width b needs.  It depends on the operator's state: when op has not cached its
 * walk degrees w (wl_fdeg, wl_apply_L or wl_expv did not run), the Laplacian calls
 * include room to compute w (n values + one work vector + the b = 1 evaluation), and
 * they compute w again on every such call; call wl_fdeg once first to avoid that.
 * WL_EUNSUPPORTED for WL_M_ARNOLDI operators.  Host only, nothing enqueued.
 * wl_apply_phi_ws / wl_apply_L_ws / wl_expv_ws: as wl_apply_phi / wl_apply_L / wl_expv,
 * with every device buffer the call uses carved from d_work (device memory on the
 * context's device, 256-byte aligned, at least the wl_workspace_size bytes for the same
 * call, b and outer_dim; WL_EINVAL otherwise).  These calls allocate no device memory
 * and record no kernel timing.  The region must stay valid until the call's work has
 * completed on the stream; its contents need no initialisation and are undefined
 * afterwards.  Calls sharing one region must be ordered (one stream).              */
typedef enum { WL_CALL_APPLY_PHI = 0, WL_CALL_APPLY_L = 1, WL_CALL_EXPV = 2 } wl_call;
wl_status wl_workspace_size(const wl_op* op, int32_t call, int32_t b, int32_t outer_dim, size_t* bytes);
wl_status wl_apply_phi_ws(wl_op* op, const void* d_X, void* d_Y, int32_t b, void* d_work, size_t work_bytes);
wl_status wl_apply_L_ws(wl_op* op, const void* d_X, void* d_Y, int32_t b, void* d_work, size_t work_bytes);
wl_status wl_expv_ws(wl_op* op, const void* d_U0, int32_t b, const double* t, int32_t nt, void* const* d_Y,
                     int32_t outer_dim, double* err_est, void* d_work, size_t work_bytes);

/* ---------------------------------------------------------------- no allocation
 * wl_apply_L_noalloc: for callers that cannot allocate device memory at all (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  As
 * wl_apply_L (Y = L X, n x b row-major, L = diag(w) - phi), but every device buffer the
 * call uses lies in a fixed region of WL_NOALLOC_BYTES (64 MiB) that the library holds
 * on each device it runs on from its first wl_ctx_create there until the process ends.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library routine)
 * and records no kernel timing.  WL_ERANGE, with nothing enqueued, when the call would
 * need more than the region (wl_workspace_size(op, WL_CALL_APPLY_L, b) tells how much;
 * FP32 series operators need about 2 n b 4 bytes, Lanczos ones (K + 2) n b s): take
 * wl_apply_L_ws with a caller region then.  Every call on one GPU, from any context or
 * thread, shares that GPU's region, and the region keeps the last call's contents:
 * calls that overlap on one GPU (two host threads, or two streams whose work is in
 * flight together) race and give undefined results; calls ordered on one stream, or
 * separated by a synchronisation, are safe.  When the operator's walk degrees are not
 * cached they are computed in the region on every call, as in wl_apply_L_ws.         */
#define WL_NOALLOC_BYTES ((size_t)64 << 20)
wl_status wl_apply_L_noalloc(wl_op* op, const void* d_X, void* d_Y, int32_t b);

/* ---------------------------------------------------------------- machine ceiling (diagnostic)
 * wl_gather_probe: the rate at which the device gathers whole table rows at random,
 * the access pattern of every neighbour gather of a sparse product (Sec. 4.1: the
 * evaluation is matrix-vector products only).  d_table: rows x row_bytes (row_bytes =
 * 16 x 1, 2, 4, 8, 16 or 32; 16-byte aligned); d_idx: count int32 row numbers (entries
 * outside [0, rows) are skipped); d_out: blocks x 256 x 16 bytes of scratch output.
 * One warm launch, then reps launches of `blocks` workgroups on the context's stream;
 * *ms = mean time per launch (HIP events).  Nothing is allocated but two events.   */
wl_status wl_gather_probe(wl_ctx* ctx, const void* d_table, int64_t rows, int32_t row_bytes, const int32_t* d_idx,
                          int64_t count, void* d_out, int32_t blocks, int32_t reps, double* ms);

/* ---------------------------------------------------------------- multigrid-preconditioned CG
 * The hierarchy of a WL_M_AMG_CG operator (Sec. 4.2), built on the host when the
 * operator is created:
 *  - strong couplings j != i with |a_ij| >= theta sqrt(a_ii a_jj), theta = 0.01;
 *  - Vanek-Mandel-Brezina aggregation over the nodes that have a strong neighbour:
 *    roots whose strong neighbourhoods are wholly free (in node order), then every free
 *    node joins the aggregate of its most strongly coupled aggregated neighbour, then
 *    leftovers group with their free strong neighbours;
 *  - smoothed prolongator P = (I - omega D^-1 A) P_t, P_t the unit-norm piecewise
 *    constants, omega = 4 / (3 ||D^-1 A||_inf); Galerkin coarse matrix P^T A P;
 *  - levels while the coarse size stays below 0.9 of the fine one and the fine level
 *    has more than 256 rows (at most 20);
 *  - V-cycle: one l1-Jacobi sweep (M = diag(sum_j |a_ij|)) before and after the coarse
 *    correction, 30 sweeps on the coarsest level; CG on every column from zero, stopped
 *    when every column's residual is within tol of its right-hand side's norm.
 * wl_amg_info: the hierarchy (rows and stored entries per level; level 0 counts the
 * graph's nonzeros plus the diagonal), operator complexity (entries over all levels /
 * level 0), setup time, and for the last solve its iterations and largest relative
 * residual; products: sum of entries x columns over every sparse product so far.
 * wl_amg_describe (host only, no device): the same hierarchy for a host CSR graph and
 * (mu, alpha): level count, rows and entries per level (arrays of max_levels), and the
 * aggregate of every node on the finest level (n int32, -1: no strong neighbour; may be
 * NULL), for inspection and tests.                                                    */
#define WL_AMG_MAX_LEVELS 20
typedef struct {
  int32_t levels;
  int64_t rows[WL_AMG_MAX_LEVELS];
  int64_t nnz[WL_AMG_MAX_LEVELS];
  double operator_complexity;
  double setup_ms;
  int32_t iterations;
  double rel_residual;
  double products;
} wl_amg_stats;
wl_status wl_amg_info(const wl_op* op, wl_amg_stats* out);
wl_status wl_amg_describe(int64_t n, const int32_t* rowptr, const int32_t* colidx, double mu, double alpha,
                          int32_t max_levels, int32_t* levels, int64_t* rows, int64_t* nnz, int32_t* agg0);

/* ---------------------------------------------------------------- discrete-time diffusion
 * The Markov chain of a walk Laplacian (Sec. "Simulating discrete-time diffusion",
 * eq. let_there_be_markov): P = I - D^{-1} L with D = diag(w), w = phi 1 (the reading
 * that reproduces the stationary distributions printed in Fig. 1), so
 * P = diag(w)^{-1} phi is row-stochastic with stationary distribution pi = w / sum(w).
 * The chain needs w > 0 (every resolvent, the exponential at mu = 0).
 *
 * wl_markov_step: d_X (n x b, row-major) holds b distributions as columns (p_0^T);
 * d_Y receives them after `steps` >= 1 steps p_{k+1} = p_k P, each computed as
 * p_{k+1}^T = phi (p_k^T ./ w) (one phi product).  1 <= b <= 64, d_X != d_Y.
 * wl_markov_stationary: d_pi (n) = w / sum(w).
 * wl_markov_gap: lambda_2 (largest eigenvalue of P below 1), lambda_min and
 * gap = 1 - max(|lambda_2|, |lambda_min|), estimated by outer_dim (2..1000) fully
 * reorthogonalised single-vector Lanczos steps on diag(w)^{-1/2} phi diag(w)^{-1/2}
 * with the eigenvector sqrt(w) deflated, from a Gaussian start vector (Philox stream
 * `seed`); each step is one phi product.  Any output pointer may be NULL.  n >= 3.  */
wl_status wl_markov_step(wl_op* op, const void* d_X, int32_t b, int32_t steps, void* d_Y);
wl_status wl_markov_stationary(wl_op* op, void* d_pi);
wl_status wl_markov_gap(wl_op* op, int32_t outer_dim, uint64_t seed, double* lambda2, double* lambda_min,
                        double* gap);

/* ---------------------------------------------------------------- rational Krylov (Alg. 1)
 * Average return probability p(t) = tr exp(-t L) / n (eq. average_return_probabilities)
 * by the randomized estimate of Alg. 1: AAA poles of exp(-x) on [0, t_max rho(L)], the
 * block rational Krylov space of L and Omega with those poles
 * (eq. block-rational-Krylov), exp(-t T) of the projected matrix for every t, and the
 * leave-one-out Nystrom trace estimate on Y(t) = V exp(-t T) V^T Omega / n with Omega.
 *
 * wl_aaa: AAA (Nakatsukasa, Sete, Trefethen 2018) on N real samples F = f(Z) (host
 * arrays), tolerance tol relative to max |F|, at most mmax support points.  poles:
 * host array of 2 cap doubles receiving (re, im) of up to cap poles of the approximant;
 * npoles their number; max_err the largest error on Z (each may be NULL).  Host only.
 * wl_exp_poles: the poles wl_return_prob uses for exp(-x) on [0, xmax]: AAA on 1000
 * equispaced points plus 1000 points xmax 10^(-6 + 6 i / 999), real poles lying on
 * [0, xmax] (spurious pole-zero pairs) dropped.  Host only.
 *
 * wl_return_prob: d_Omega n x M (row-major, operator precision, device; e.g. Gaussian
 * probes from wl_probes), 2 <= M <= 32, n > M.  t (host, nt values >= 0); t_max > 0 the
 * end of the time window; rho > 0 the spectral radius of L to use (<= 0: for a
 * resolvent operator the bound max w - s / (s + (mu alpha^2 + alpha) d_max), s = 1 -
 * mu^2 alpha^2, which holds since phi = s A_mu(alpha)^{-1} is positive definite and
 * bounds lambda_max(A_mu(alpha)) by Gershgorin; for
 * other operators 40 Lanczos steps, the largest Ritz value plus its residual norm;
 * t_max rho <= aaa_tol, as for L = 0, leaves no poles).  Poles: the wl_exp_poles
 * poles for xmax = t_max rho, divided by pole_time (1: as the algorithm states; t_max:
 * the poles of r(t_max lambda) ~ exp(-t_max lambda), accurate for t near t_max).  Each
 * real pole adds one basis block, each conjugate pair two (the real and imaginary parts
 * of (L - xi)^{-1} U, U the last block); the shifted systems are solved by COCG to the
 * relative residual solve_tol within max_iters iterations (WL_ENOCONV otherwise).  The
 * projected matrix is V^T L V.  p_hat, e_hat (host, nt, may be NULL): the estimates and
 * their error estimates (standard error over the left-out probes).  poles (host,
 * 2 poles_cap doubles, may be NULL): the poles used.  info (may be NULL): counts and
 * residuals.  rcond: the Nystrom cores drop eigenvalues below rcond times the largest.
 * Resolvent operators solve each shifted system on its symmetrised form
 * (d A_mu d - s I) z = u / d, d = (w - xi)^{1/2}, one sparse product per iteration,
 * with the residual checked on the original system; other operators apply L itself.
 * FP32 Lanczos operators pad the blocks to Mp = 16 ceil(M / 16) columns (zero columns)
 * and evaluate every product as 16-column groups.  Memory: (1 + poles) blocks of
 * n x Mp plus four n x 2 Mp blocks, and for 16-column groups their Lanczos bases
 * ((K + 1) blocks of n x Mp); all of it stays with the operator for the next call (the
 * largest sizes seen) and is freed by wl_op_destroy.  Calls on one operator must not
 * overlap.                                                                             */
typedef struct {
  int32_t npoles;      /* finite poles used (a conjugate pair counts two) */
  int32_t nblocks;     /* basis blocks: Omega's, one per real pole, two per pair */
  int32_t solves;      /* shifted solves: one per real pole or conjugate pair */
  int32_t iters_total; /* COCG iterations over all solves */
  int32_t iters_max;   /* COCG iterations of the longest solve */
  double rho;          /* spectral radius used for the AAA interval */
  double aaa_err;      /* AAA's largest error on its sample points */
  double solve_res;    /* largest relative residual at the end of a solve */
  double products;     /* sparse products times the probe columns they acted on (work) */
} wl_rk_info;

wl_status wl_aaa(int64_t N, const double* Z, const double* F, double tol, int32_t mmax, double* poles, int32_t cap,
                 int32_t* npoles, double* max_err);
wl_status wl_exp_poles(double xmax, double tol, int32_t mmax, double* poles, int32_t cap, int32_t* npoles,
                       double* max_err);
wl_status wl_return_prob(wl_op* op, const void* d_Omega, int32_t M, const double* t, int32_t nt, double t_max,
                         double rho, double pole_time, double aaa_tol, double solve_tol, int32_t max_iters,
                         double rcond, double* p_hat, double* e_hat, double* poles, int32_t poles_cap,
                         wl_rk_info* info);

/* ---------------------------------------------------------------- block Krylov primitives
 * The tall-skinny kernels every block Lanczos step is made of (Sec. 4.1: the basis
 * Q_k and its projection H_k), exposed for callers building their own drivers.
 *
 * wl_block_gram: G = [X_0 .. X_{nblk-1}]^T Y with X_k the k-th of nblk consecutive
 * row-major n x bx blocks starting at d_X (block k at d_X + k n bx elements) and Y
 * one n x by block.  G (host, double, (nblk bx) x by row-major) is accumulated in
 * double in a fixed order (bitwise reproducible).  Synchronises the stream.
 *
 * wl_block_update: Out = alpha Yin + beta sum_k X_k C_k with X_k as above (width b),
 * C (host, double, (nblk b) x b row-major), Yin / Out n x b (Yin may be NULL; Out may
 * alias Yin or X_0 when nblk = 1).  If G (host, b x b) is not NULL it receives
 * Out^T Out.  Synchronises the stream.                                             */
wl_status wl_block_gram(wl_ctx* ctx, int32_t prec, int64_t n, int32_t nblk, int32_t bx, const void* d_X,
                        int32_t by, const void* d_Y, double* G);
wl_status wl_block_update(wl_ctx* ctx, int32_t prec, int64_t n, int32_t nblk, int32_t b, const void* d_X,
                          const double* C, const void* d_Yin, double alpha, double beta, void* d_Out, double* G);

/* ---------------------------------------------------------------- probes
 * Fill an n x M row-major block with Philox4x32-10 probes (Salmon et al., SC'11):
 * element (i, j) is word e mod 4 of Philox(counter (q lo, q hi, stream, 0),
 * key (seed lo, seed hi)), e = i*M + j, q = e div 4.  Rademacher 1 - 2 (word>>31);
 * Gaussian by Box-Muller on word pairs (0,1), (2,3), u = (word + 1/2) 2^-32,
 * evaluated in double.  These are the "iid isotropic" probes of Alg. 1.          */
wl_status wl_probes(wl_ctx* ctx, int32_t prec, int32_t law, uint64_t seed, uint32_t stream,
                    int64_t n, int32_t M, void* d_out);

/* ---------------------------------------------------------------- estimators (Sec. 4.4)
 * Given the probe block Omega (n x M) and Y = F Omega for a symmetric F:
 *   WL_EST_HUTCHINSON  d_i = (1/M) sum_j Omega_ij Y_ij
 *   WL_EST_BKS         d_i = sum_j Omega_ij Y_ij / sum_j Omega_ij^2
 *   WL_EST_XNYS        leave-one-out Nystrom estimator: for each j the Nystrom
 *                      approximation from the other probes, corrected by probe j,
 *                      averaged over j (F must be positive semidefinite).
 * d_diag (n, prec) receives the diagonal estimate; trace / trace_err (host, may be
 * NULL) the trace estimate and its error estimate (std over j / sqrt M; for the
 * Hutchinson/BKS laws the same statistic of the per-probe traces).  rcond: the
 * Nystrom core pseudo-inverse drops eigenvalues below rcond * largest.
 * d_cv (n, prec, may be NULL): control variate g for the diagonal:
 *   d_i = g_i + (1/M) sum_j Omega_ij (Y_ij - g_i Omega_ij)   (Hutchinson only).   */
wl_status wl_estimate(wl_ctx* ctx, int32_t prec, int32_t estimator, int64_t n, int32_t M,
                      const void* d_Omega, const void* d_Y, const void* d_cv, double rcond,
                      void* d_diag, double* trace, double* trace_err);

/* Convenience: diag phi (target 0) or diag exp(-t L) (target 1) estimated from M
 * probes drawn by wl_probes(seed, law), then wl_estimate.  d_diag: n values of the
 * operator's precision (device).  M in [1, 4096]; for M <= 64 the probes are one
 * n x M block of Philox stream 0.  For M > 64 (Hutchinson, BKS and the control
 * variate only; the Nystrom estimator takes M <= 64) the probes are ceil(M / 64)
 * blocks of 64 columns (the last one narrower), block c drawn from Philox stream c,
 * each pushed through the operator in turn with the per-row sums accumulated on the
 * device: the result is the M-probe estimator over those columns.
 * WL_EST_SURROGATE (target 0 only): with G = sum_{k<=3} c_k q_k(A) (eq. qrec, the
 * operator's own weights), whose diagonal is exact from the degrees and triangle
 * counts (diag q_1 = 0, diag q_2 = (1 - mu) d, diag q_3 = diag A^3 = 2 t):
 *   d_i = g_i + (1/M) sum_j Omega_ij ((phi - G) Omega)_ij + (diag G_i - g_i) s_i / M,
 *   s_i = sum_j Omega_ij^2, g = d_cv if given, else diag G.
 * Unbiased for any g: G's off-diagonal part no longer enters the probe noise.  The
 * trace estimate is tr G + the mean of the per-probe omega^T (phi - G) omega.     */
wl_status wl_diag_est(wl_op* op, int32_t target, double t, int32_t M, uint64_t seed,
                      int32_t law, int32_t estimator, const void* d_cv, int32_t outer_dim,
                      void* d_diag, double* trace, double* trace_err);

/* ---------------------------------------------------------------- several operators
 * Operators of one graph evaluated together on one wide block, operator g on columns
 * [g b, (g + 1) b), with one sparse product per step for all of them (wide rows gather
 * whole cache lines).  All operators share graph, precision and evaluation method:
 *   * WL_M_RECURRENCE: their truncated series (eq. qrec) step side by side with each
 *     group's weights of that step from a table (operators with a lower degree stop
 *     contributing after their last step).  Results equal those of the single
 *     operators up to the summation order of the sparse products.
 *   * WL_M_LANCZOS (Sec. 4.1): one block Lanczos process per operator, in lock step:
 *     the sparse product applies every group's own symmetric matrix and three-term
 *     subtraction, and the projections, CholQR factorisations and basis updates of all
 *     groups run as single passes over the wide block (with the second local pass
 *     against the previous block when any operator has reorth >= 1; with reorth 0
 *     each new block is projected against the current one only).  Each group's
 *     result uses its own number of steps; it agrees with the single operator's to the
 *     rounding level
 *     of the Krylov recurrence (the grouped kernels sum in another order).  Grouped
 *     kernels cover FP32 with b = 16 and b = 1 (nops <= 8, any precision); other
 *     shapes, and Krylov spaces so small that full reorthogonalisation is needed
 *     ((steps + 1) 2 b > n), are evaluated operator by operator into the same layout.
 * wl_multi_create: 1 <= nops <= 64 operators (WL_EUNSUPPORTED for mixed methods and for
 * WL_M_ARNOLDI operators, which are evaluated alone); the
 * handle keeps the graph alive (not the operators, whose descriptors it copies).
 * wl_multi_apply: d_X n x b (the same block for every operator), d_Y n x (nops b)
 * row-major, laplacian != 0: L_g X in group g, else phi_g X.  nops b <= 4096.  Rows of
 * nops b = 32 or 64 FP32 values are where the sharing pays most.
 * wl_multi_fdeg: d_W n x nops, column g = phi_g 1.
 * wl_multi_apply_fdeg: both in one evaluation (the walk degrees w_g = phi_g 1 of
 * eq. weighted_laplacian beside phi_g X or L_g X) for the first nx operators
 * (1 <= nx <= nops) on X and the walk degrees of all nops: d_Y n x (nx b) row-major
 * (group g < nx as wl_multi_apply), d_W n x nops as wl_multi_fdeg (three distinct
 * buffers).  The vectors of ones ride in one extra group of 16 columns, so each step
 * gathers them from the same cache lines as the blocks: truncated series for
 * nops <= 16 and any b; Lanczos operators for FP32, b = 16, nops <= 16 (the ones'
 * group then holds nops independent single-column Lanczos processes with diagonal
 * Grams).  Other shapes run wl_multi_apply, then wl_multi_fdeg (nx = nops only;
 * WL_EUNSUPPORTED otherwise).  With laplacian != 0 the finish takes the walk degrees
 * cached by an earlier call (computed first when there are none), as wl_multi_apply
 * does.                                                                              */
typedef struct wl_multi wl_multi;
wl_status wl_multi_create(wl_op* const* ops, int32_t nops, wl_multi** out);
wl_status wl_multi_apply(wl_multi* multi, const void* d_X, int32_t b, void* d_Y, int32_t laplacian);
wl_status wl_multi_fdeg(wl_multi* multi, void* d_W);
wl_status wl_multi_apply_fdeg(wl_multi* multi, const void* d_X, int32_t b, int32_t nx, void* d_Y, void* d_W,
                              int32_t laplacian);
wl_status wl_multi_destroy(wl_multi* multi);

/* ---------------------------------------------------------------- batches of graphs
 * Many graphs with their own walk variant and weights, evaluated together: the
 * graphs are concatenated into one block-diagonal CSR whose per-graph row ranges start
 * at 64-row boundaries (offsets from wl_batch_info; padding rows have no edges and
 * must hold zeros in inputs), so every sparse product, Gram and block update of a
 * Krylov step is one launch for the whole batch.  Inner phi products use each graph's
 * truncated series (eq. qrec) with degree from tol (exponential: tail bound with
 * lambda_max; resolvent: geometric bound alpha lambda_max, or the asymptotic ratio
 * alpha rho(Z_mu) plus 20 terms when alpha lambda_max >= 1).  FP32 vectors.
 *
 * wl_batch_create: 1 <= ngraphs <= 65535; descs[g] describes graph g (mu, func, param; krylov_dim > 0 fixes
 * its series degree; rho_hint as for operators).  Computes every walk degree.
 * wl_batch_info: any output may be NULL; row_offsets (int64) and series_degrees
 * (int32, the truncation degree K_g of graph g's series) are host arrays of ngraphs.
 * wl_batch_autotune: times SpMM launch shapes on the concatenated graph for b columns
 * (as wl_autotune) and keeps the fastest for the batch's sparse products; then times
 * the XCD-grouped tile order (every graph's row tiles on one XCD, so its gathered rows
 * stay in that XCD's L2) against the plain order and keeps the faster (plain until
 * tuned).  wl_batch_tile_order reports the choice (1: XCD-grouped);
 * wl_batch_set_tile_order sets it (results do not depend on it).
 * wl_batch_apply_L: Y = L_g X_g for every graph (d_X, d_Y: total_rows x b).
 * wl_batch_expv: Y_g = exp(-t_g L_g) U0_g for every graph (t: host array of ngraphs
 * times) by outer_dim block Lanczos steps per graph, the projected exponential
 * computed on the device; b in [2, 16] and 5 outer_dim b^2 doubles <= 150 KiB.
 * If p_hat / p_err (host, ngraphs) are given and U0 holds iid Gaussian probes, they
 * receive the leave-one-out Nystrom estimate of tr exp(-t_g L_g) / n_g (the average
 * return probability, eq. average_return_probabilities, Alg. 1) and its error
 * estimate, computed from the projected quantities only.                          */
typedef struct wl_batch wl_batch;
wl_status wl_batch_create(wl_ctx* ctx, int32_t ngraphs, wl_graph* const* graphs, const wl_op_desc* descs,
                          double tol, wl_batch** out);
wl_status wl_batch_info(const wl_batch* batch, int64_t* total_rows, int32_t* max_series_degree,
                        int64_t* row_offsets, int32_t* series_degrees);
wl_status wl_batch_autotune(wl_batch* batch, int32_t b);
wl_status wl_batch_tile_order(const wl_batch* batch, int32_t* xcd_grouped);
wl_status wl_batch_set_tile_order(wl_batch* batch, int32_t xcd_grouped);
wl_status wl_batch_apply_L(wl_batch* batch, const void* d_X, void* d_Y, int32_t b);
wl_status wl_batch_expv(wl_batch* batch, const void* d_U0, int32_t b, const double* t, int32_t outer_dim, void* d_Y,
                        double* p_hat, double* p_err);
wl_status wl_batch_destroy(wl_batch* batch);

/* Replayable batched diffusion for fixed buffers (serving loops): the whole device
 * part of wl_batch_expv for (d_U0, b, outer_dim, d_Y) captured once into a HIP
 * graph with scratch of its own.  wl_batch_graph_launch copies the ngraphs times t
 * (host) to the device, launches the graph on the context's stream and returns
 * without waiting unless p_hat / p_err are requested (as in wl_batch_expv; then it
 * synchronises).  d_U0 is read and d_Y written at every launch; their contents may
 * change between launches, their addresses may not.  Launches of one graph are
 * ordered on the stream; a graph must be destroyed before its batch
 * (wl_batch_destroy returns WL_EINVAL while graphs are alive).  Same limits on b
 * and outer_dim as wl_batch_expv.                                                  */
typedef struct wl_batch_graph wl_batch_graph;
wl_status wl_batch_graph_create(wl_batch* batch, const void* d_U0, int32_t b, int32_t outer_dim, void* d_Y,
                                wl_batch_graph** out);
wl_status wl_batch_graph_launch(wl_batch_graph* graph, const double* t, double* p_hat, double* p_err);
wl_status wl_batch_graph_destroy(wl_batch_graph* graph);

/* ---------------------------------------------------------------- learned control variate
 * No counterpart in the paper: a small network predicts diag(phi) from cheap local
 * features and serves as a control variate for the diagonal estimator.
 *
 * wl_features: d_feat (n x 8 float, row-major) = local features of every node, with
 * structural counts scaled by s (alpha or beta of the target operator):
 * log1p(s d), log1p(s^2 d), log1p(s^3 2t), log1p(s^2 S2), log1p(s mean_j d_j),
 * log1p(s rms_j d_j), log1p(s max_j d_j), clustering 2t / (d (d - 1)); d = degree,
 * t = triangles through the node, S2 = sum of neighbour degrees (2-walk count),
 * j over neighbours.  Synchronises the stream.
 *
 * wl_diag_exact: d_out[j] = phi[nodes[j], nodes[j]] for count device node indices,
 * from unit-vector blocks of the given width pushed through the operator (the
 * method's own exact diagonal, used as training targets).  Element type by op.
 *
 * wl_mlp_*: 8 -> 64 -> 64 -> 1 multilayer perceptron with tanh hidden units, FP32
 * parameters (4801 values: W1 64x8, b1, W2 64x64, b2, W3 1x64, b3), mean-squared-
 * error loss, Adam (beta1 0.9, beta2 0.999, eps 1e-8).  Gradients are reduced in
 * double in a fixed order.  h_params may be NULL (zeros).  wl_mlp_loss_grad returns
 * the loss and (if h_grad is not NULL) the gradient (4801 doubles) without updating.
 * wl_mlp_save / wl_mlp_load: flat binary file, 8-byte magic "WLMLP001", int32 count,
 * float parameters.                                                               */
wl_status wl_features(wl_graph* g, double scale, void* d_feat);
/* Low-order part of diag phi and the scale of the rest, per node (element type by op):
 *   base_i  = diag of sum_{k<=3} c_k q_k = 1 + c_2 (1 - mu) d_i + c_3 (A^3)_ii,
 *   scale_i = c_4 max(1, d_i^2 + S2_i),  S2_i = sum_{j in N(i)} d_j.
 * Either output may be NULL.  wl_surrogate_target: for count device node indices,
 * d_out[j] = (phi[i, i] - base_i) / scale_i with phi[i, i] from wl_diag_exact: the
 * training target of a network that predicts diag phi as base + scale * net(features).
 * wl_mlp_predict: d_out = base + scale * net(feat) (FP32; base / scale may be NULL for
 * 0 / 1): a control variate for the Hutchinson and surrogate estimators.           */
wl_status wl_surrogate_diag(wl_op* op, void* d_base, void* d_scale);
wl_status wl_surrogate_target(wl_op* op, const int32_t* d_nodes, int64_t count, int32_t width, void* d_out);
wl_status wl_diag_exact(wl_op* op, const int32_t* d_nodes, int64_t count, int32_t width, void* d_out);
int32_t wl_mlp_num_params(void);
wl_status wl_mlp_create(wl_ctx* ctx, const float* h_params, wl_mlp** out);
wl_status wl_mlp_destroy(wl_mlp* net);
wl_status wl_mlp_get_params(const wl_mlp* net, float* h_params);
wl_status wl_mlp_forward(wl_mlp* net, const void* d_feat, int64_t n, void* d_out);
wl_status wl_mlp_predict(wl_mlp* net, const void* d_feat, int64_t n, const void* d_base, const void* d_scale,
                         void* d_out);
wl_status wl_mlp_loss_grad(wl_mlp* net, const void* d_feat, const void* d_target, int64_t n, double* loss,
                           double* h_grad);
wl_status wl_mlp_train_step(wl_mlp* net, const void* d_feat, const void* d_target, int64_t n, double lr,
                            double* loss);
wl_status wl_mlp_save(const wl_mlp* net, const char* path);
wl_status wl_mlp_load(wl_ctx* ctx, const char* path, wl_mlp** out);

#ifdef __cplusplus
}
#endif
#endif /* WALKLAP_H */
