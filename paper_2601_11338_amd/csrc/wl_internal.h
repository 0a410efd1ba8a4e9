// Internal declarations of the walk-Laplacian library: handle structs, error
// helpers, device buffers and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <complex>
#include <vector>

#include "walklap.h"

// ------------------------------------------------------------------ errors
void wl_set_error(const char* fmt, ...);

#define WL_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      wl_set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,   \
                   __LINE__);                                                         \
      return (e_ == hipErrorOutOfMemory) ? WL_ENOMEM : WL_EDEVICE;                   \
    }                                                                                 \
  } while (0)

#define WL_CHECK(cond, code, ...) \
  do {                            \
    if (!(cond)) {                \
      wl_set_error(__VA_ARGS__);  \
      return code;                \
    }                             \
  } while (0)

#define WL_TRY(expr)              \
  do {                            \
    wl_status s_ = (expr);        \
    if (s_ != WL_OK) return s_;   \
  } while (0)

// Makes dev current for a scope and restores the previous device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// ------------------------------------------------------------------ device buffer
// Nonzero while a call runs on caller-provided workspace: no buffer may then grow (a
// growth would be a device allocation the caller asked not to happen).
extern thread_local int wl_no_alloc;

// Test hook for the failure paths: true when this device allocation is the one
// WL_TEST_FAIL_ALLOC=k (read at the first allocation) or wl_test_fail_alloc(k) selected,
// the k-th from then on (counting from 0); it then fails as an out-of-memory would.
bool wl_alloc_injected();

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool borrowed = false;  // p points into caller workspace (never freed here)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    // work still queued may read the old allocation: drain the device first
    if (p && !borrowed) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
    borrowed = false;
  }
  // Grow to at least nbytes (contents not preserved).
  wl_status ensure(size_t nbytes) {
    if (nbytes <= bytes && p) return WL_OK;
    if (borrowed || wl_no_alloc) {
      wl_set_error("workspace plan too small: a buffer of %zu bytes was needed (internal)", nbytes);
      return WL_EINTERNAL;
    }
    release();
    size_t want = nbytes < 256 ? 256 : nbytes;
    if (wl_alloc_injected()) {
      wl_set_error("hipMalloc(%zu) failed: out of memory (injected by the allocation-failure test hook)", want);
      return WL_ENOMEM;
    }
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      wl_set_error("hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
      return WL_ENOMEM;
    }
    bytes = want;
    return WL_OK;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------------ handles
struct SpmmShape {
  int G = 16;          // lanes per row group for rows below the long threshold
  int long_thr = 512;  // rows with more neighbours go to whole workgroups
};

// Live timing of kernel classes (opt-in): HIP events recorded around each launch
// on the context stream, algorithmic bytes counted per launch.
// Timing classes of sparse products: single-operator series steps (b >= 4), Lanczos
// operator products (b >= 4), side-by-side operator steps (width >= 32), the rest.
enum { WL_KC_RECURRENCE = 0, WL_KC_LANCZOS_OP = 1, WL_KC_OTHER_SPMM = 2, WL_KC_MULTI = 3, WL_KC_MULTI_LANCZOS = 4,
       WL_KC_AMG = 5, WL_KC_COUNT = 6 };
struct KernelStats {
  int64_t launches = 0;
  double bytes = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t used = 0;
  double folded_ms = 0.0;  // time of event pairs already read back and reused
};
// Trace mode (WL_TRACE set at context creation) keeps profiling on for the context's
// life: every WL_TRACE_FOLD launches of a class its event pairs are read back (one wait
// for the last) and reused.
constexpr size_t WL_TRACE_FOLD = 16384;
wl_status kstats_fold(KernelStats& k);
struct wl_ctx;
// Timing of one launch of class kc (profiling on): kstats_begin records the start event
// on the context's stream and returns the class's record (null when profiling is off or
// kc is not a class), kstats_end the end event and the launch's algorithmic bytes.
wl_status kstats_begin(wl_ctx* ctx, int kc, KernelStats** ks);
wl_status kstats_end(wl_ctx* ctx, KernelStats* ks, double bytes);

struct wl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  DevBuf partials;  // reduction partials
  DevBuf scratch;   // small device-side matrices
  DevBuf check_count;  // counter of the output scan (allocated when checks are enabled)
  uint32_t checks = 0;  // WL_CHECK_* flags
  bool profiling = false;
  bool trace = false;
  KernelStats kstats[WL_KC_COUNT];
  int refs = 1;  // the caller's handle + every graph / network made from it
};
void ctx_release(wl_ctx* ctx);

struct wl_graph {
  wl_ctx* ctx = nullptr;
  int64_t n = 0, nnz = 0;
  const int32_t* rowptr = nullptr;
  const int32_t* colidx = nullptr;
  DevBuf own_rowptr, own_colidx;
  int32_t max_deg = 0;
  double mean_deg = 0.0;
  std::vector<int32_t> h_degree_hist;   // not used by kernels
  // rows sorted by decreasing degree whose degree exceeds the smallest threshold
  // any launch may use; per launch only the prefix above its threshold is taken.
  DevBuf long_rows;
  std::vector<int32_t> h_long_deg;      // degrees of long_rows, decreasing
  int32_t long_min_thr = 64;
  std::map<int, SpmmShape> tuned;       // key: prec * 1000 + b
  double lam_max = -1.0;
  std::map<double, double> rho_cache;
  DevBuf degf, degd;                    // degree vector as float / double
  DevBuf tmp;
  DevBuf tri2;                          // (A^3)_ii, once computed
  bool tri2_valid = false;                           // Lanczos scratch for spectral routines
  int refs = 1;                         // the caller's handle + every operator on it
};
void graph_release(wl_graph* g);

struct wl_op {
  wl_graph* g = nullptr;
  wl_op_desc d{};
  double rho = 0.0;       // rho(Z_mu) used for validation (0 if not needed)
  double lam = 0.0;       // lambda_max(A) (exponential weights: scaling of the series)
  int K = 0;              // recurrence degree or Lanczos steps
  DevBuf w;               // cached phi 1
  bool w_valid = false;
  DevBuf bufA, bufB;      // recurrence buffers
  DevBuf basis;           // Lanczos basis (K+1) blocks of n x b
  DevBuf wbuf;            // Lanczos W block
  DevBuf coef;            // device copy of recombination coefficients
  DevBuf small;           // device FP64 small matrices (T blocks etc.)
  DevBuf outer_basis, outer_w, outer_small, outer_coef, inner_tmp;
  // discrete-time diffusion scratch, kept between calls (freeing a buffer waits for the
  // whole device, which would serialise work on other streams)
  DevBuf mk_rw, mk_tmp, mk_alt, mk_x0, mk_t1, mk_t2, mk_dd;
  struct AmgState* amg = nullptr;  // WL_M_AMG_CG: multigrid hierarchy and CG work blocks
  struct RkCache* rk = nullptr;    // return-probability work buffers, kept between calls
};
// Frees the operator's return-probability work buffers (with the stream drained).
void rk_cache_destroy(wl_op* op);

// ------------------------------------------------------------------ launch interfaces
// SpMM epilogue (per row r, on the b columns of the current tile):
//   y        = a * (A X)[r] + (b0 + b1 * d_r) * Z[r] - Z2[r, :] * C    (terms optional)
//   Y[r]     = y                                                       (if Y)
//   Sout[r]  = s0 * Sin[r] + sc * y                                    (if Sout; Sin optional)
//   if wv:     Sout[r] = wv[r] * Xw[r] - Sout[r]                       (walk-Laplacian finish)
//   if jw:     Sout[r] = jx[r] + jw[r] * Sout[r]                       (Jacobi sweep finish)
// C is b x b row-major double on the device (transC: use C^T).
template <typename T>
struct EpiArgs {
  double a = 1.0;
  const T* Z = nullptr;
  double b0 = 0.0, b1 = 0.0;
  const T* Z2 = nullptr;
  const double* C = nullptr;
  int transC = 0;
  const T* Sin = nullptr;
  T* Sout = nullptr;
  double s0 = 0.0, sc = 0.0;
  const T* wv = nullptr;
  const T* Xw = nullptr;
  // Jacobi finish (instead of the walk-Laplacian one): Sout[r] = jx[r] + jw[r] * Sout[r]
  const T* jw = nullptr;
  const T* jx = nullptr;
  int kclass = WL_KC_OTHER_SPMM;  // timing class when profiling is on
  // Batched graphs: row r belongs to graph gid[r]; gtab holds, per graph, the five
  // coefficients {a, b0, b1, sc, fin} of this launch (replacing a, b0, b1, sc; fin != 0
  // applies the walk-Laplacian finish).  Rows of graphs with a = sc = 0 are skipped.
  const int32_t* gid = nullptr;
  const double* gtab = nullptr;
  // Several operators side by side: column c belongs to operator c / cgw, whose five
  // coefficients of this launch are ctab[5 (c / cgw) ...]; the finish weight is then
  // wv[r * wld + c / cgw] (wv holds one walk-degree column per operator).
  // With C as well, C is block diagonal: operator q's cgw x cgw block sits at
  // C + q * cgs, and Z2's row segment of that operator is what multiplies it.
  const double* ctab = nullptr;
  int cgw = 0;
  int wld = 0;
  int64_t cgs = 0;
  // Per-column operators (with ctab): column c takes the coefficients ctab[5 cmap[c] ...]
  // and the finish weight wv[r * wld + cmap[c]] instead of those of c / cgw (cmap[c] < 0:
  // padding, all coefficients zero).  C stays block diagonal in cgw-wide groups.  This
  // lets one group of cgw columns hold single columns of different operators (their
  // walk degrees riding beside the wide blocks).
  const int32_t* cmap = nullptr;
  // Deferred normalisation (with ctab): the gathered-plus-diagonal part u of a row is
  // multiplied from the right by its cgw x cgw group block of Nm (row-major, group q's
  // at Nm + q * cgs) before the C term: y = u N_q - Z2 C_q.  Needs 16-byte vectors and
  // cgw = 16.
  const double* Nm = nullptr;
  // Row-tile order of the short-row blocks (host object, resolved by the launcher):
  // block s of the launch processes row tile map[s] (-1: idle), so that tiles that
  // gather from the same rows can be placed on one XCD.  Null: tile s = block s.
  const struct XcdTileMap* xmap = nullptr;
  const int32_t* tile_map = nullptr;  // device map, filled in by the launcher
  // Host-side preparation only (resolve the tile map for this shape), no launch: makes
  // a later launch of the same shape free of allocation and host copies (capture).
  int prepare_only = 0;
};

// Tiles of a block-diagonal graph (consecutive row ranges that only touch their own
// rows) assigned to XCDs: workgroups are dispatched to the 8 XCDs round-robin, so
// launch block b runs on XCD b mod 8.  Each range goes to one XCD (balanced by
// nonzeros), and the map puts its row tiles on blocks of that XCD; the rows it
// gathers then stay in that XCD's L2.  Ranges must start at multiples of 64 rows.
struct XcdTileMap {
  static constexpr int NXCD = 8;
  std::vector<int64_t> start, end;  // row range of every part
  std::vector<int> xcd;             // its XCD
  struct Entry {
    DevBuf map;
    int64_t blocks = 0;
  };
  std::map<std::pair<int, int>, Entry> cache;  // (rows per tile, blocks before the tiles)
  // Device map for tiles of rpb rows placed after lead other blocks; builds on first use.
  wl_status get(int rpb, int lead, const int32_t** map, int64_t* blocks);
};

template <typename T>
wl_status launch_spmm(wl_graph* g, const T* X, T* Y, int b, const EpiArgs<T>& ep, const SpmmShape& sh);

// tri2[i] = (A^3)_ii = twice the triangles through node i (n unsigned 64-bit counts),
// computed on first use and kept in the graph; colidx must be sorted within rows.
// *out receives the device array (valid while the graph lives).
wl_status graph_tri2(wl_graph* g, const unsigned long long** out);

// SpMM launch shape for (prec, b) on g: the autotuned one if present, else a heuristic.
SpmmShape shape_for(wl_graph* g, int prec, int b);

// Gram partials and finalisation.  X: nblk blocks of n x bx (block k at X + k*sX),
// Y: n x by.  out (double, nblk*bx x by row-major) = X^T Y, reduced in a fixed
// order (deterministic).  Partials live in ctx->partials.
template <typename T>
wl_status launch_gram(wl_ctx* ctx, int64_t n, const T* X, int bx, int64_t sX, int nblk, const T* Y, int by,
                      double* out);

// Out[r,:] = (wv ? wv[r] : alpha) * Yin[r,:] + beta * sum_k X_k[r,:] C_k
// with C (nblk*bx x by, row-major double, device).  Yin may be null; Out may
// alias Yin or X.  If gram_out is non-null, also gram_out = Out^T Out (double by x by).
template <typename T>
wl_status launch_update(wl_ctx* ctx, int64_t n, const T* X, int bx, int64_t sX, int nblk, const double* C,
                        const T* Yin, double alpha, const T* wv, double beta, T* Out, int by, double* gram_out);
// The same with device flags (may be NULL): when *skip != 0 the update is an identity
// the caller elides (the kernel returns at once); when *skip_gram != 0 the Gram of the
// output is not needed.  Only the FP32 block paths honour them (others compute).
template <typename T>
wl_status launch_update_skip(wl_ctx* ctx, int64_t n, const T* X, int bx, int64_t sX, int nblk, const double* C,
                             const T* Yin, double alpha, const T* wv, double beta, T* Out, int by, double* gram_out,
                             const double* skip, const double* skip_gram);

// Cholesky with deflation of the b x b Gram G (double, device):
//   G = R^T R, R upper; Rinv the inverse on the non-deflated columns (zero elsewhere).
// A pivot below tol * ref deflates its column, where
//   ref = max(max_i G_ii, (||Aref||_F^2 + ||Bref||_F^2) / b)  (Aref, Bref optional b x b).
// If Rprev is given, Bout = R * Rprev (else Bout = R when Bout is given).
// ngraphs workgroups run independent instances, instance g on matrices offset by g * gs.
// ref_out (one double, optional) receives ref.  With ref_in and post_tol > 0 every k
// with |Bout_kk| <= post_tol sqrt(*ref_in) is dropped (zero row k of Bout, zero column k
// of Rinv): Bout_kk is the true norm of the k-th component when G is the true Gram of
// the block (or Bout = R2 R1 after a second pass).
wl_status launch_chol(wl_ctx* ctx, int b, const double* G, double tol, const double* Aref, const double* Bref,
                      double* R, double* Rinv, const double* Rprev, double* Bout, int ngraphs = 1,
                      int64_t gs = 0, double* ref_out = nullptr, const double* ref_in = nullptr,
                      double post_tol = 0.0, double* skip_out = nullptr, double skip_ratio = 0.0,
                      const double* skip_in = nullptr, int dg = -1, const double* dref = nullptr);
// dg: index of a group (workgroup) whose columns are independent single-column
// processes: its G is taken as diagonal, each column deflated against its own scale
// (dref, optional: per-group b x b matrices whose diagonal is the column scale of the
// later check), and no second pass is asked for.
// skip_out (one double): 1 when the kept pivots satisfy min / max >= skip_ratio (a
// second CholQR pass would change nothing at working precision), else 0.  skip_in:
// when *skip_in != 0 the kernel only writes identity factors (R, Rinv) and
// Bout = Rprev, standing in for a second pass that was not needed.

// One block Lanczos projection: from P = [V_{j-1}^T W'; V_j^T W'; W'^T W'] (nbv = 2) or
// [V_j^T W'; W'^T W'] (nbv = 1) form A_j = sym(V_j^T W') (Aout), Cc = [-P1; -A_j; I] with
// W = [V_{j-1} V_j W'] Cc the projected block, and ref = max_i (W'^T W')_ii (ref_out,
// optional).  Batched like launch_chol.
wl_status launch_lanczos_proj(wl_ctx* ctx, int b, int nbv, const double* P, double* Aout, double* Cc,
                              double* ref_out = nullptr, int ngraphs = 1, int64_t gs = 0);

// Small device helpers on double matrices.
wl_status launch_dadd(wl_ctx* ctx, int count, const double* x, double* y);   // y += x
wl_status launch_dcopy(wl_ctx* ctx, int count, const double* x, double* y);  // y = x
wl_status launch_dtranspose(wl_ctx* ctx, int b, const double* x, double* y);  // y = x^T (b x b)

template <typename T>
wl_status launch_fill(wl_ctx* ctx, int64_t count, T value, T* out);
template <typename T>
wl_status launch_axpby_rows(wl_ctx* ctx, int64_t n, int b, const T* w, const T* X, double beta, const T* Y,
                            T* Out);  // Out = w (.) X + beta * Y  (w per row; w null = 1)
template <typename T>
wl_status launch_degrees(wl_graph* g, T* out);
wl_status launch_validate(wl_graph* g, int32_t* d_flags);

template <typename T>
wl_status launch_probes(wl_ctx* ctx, int law, uint64_t seed, uint32_t stream, int64_t n, int M, T* out);

// Row-wise estimator reductions: dot[r] (+)= sum_j Om[r,j] Y[r,j], sq[r] (+)= sum_j Om[r,j]^2
// (accumulate != 0 adds to the values already there); launch_sums_finish turns the
// sums over M probes into the Hutchinson (mode 0), BKS (1) or control-variate (2)
// diagonal.
template <typename T>
wl_status launch_rowdot(wl_ctx* ctx, int64_t n, int M, const T* Om, const T* Y, double* dot, double* sq,
                        int accumulate);
template <typename T>
wl_status launch_sums_finish(wl_ctx* ctx, int64_t n, int M, const double* dot, const double* sq, const T* g,
                             int mode, T* diag);
// Per-probe traces: tr[j] = sum_r Om[r,j] Y[r,j] (double M), through the Gram machinery.
// Nystrom diagonal finish: diag[r] = (y_r^T Q1 y_r + sum_j Om_rj Y_rj - y_r^T Q2 om_r) / M
template <typename T>
wl_status launch_nys_diag(wl_ctx* ctx, int64_t n, int M, const T* Om, const T* Y, const double* Q1,
                          const double* Q2, T* diag);
template <typename T>
wl_status launch_cv_finish(wl_ctx* ctx, int64_t n, int M, const T* Om, const T* Y, const T* g, int mode, T* diag);

// ------------------------------------------------------------------ host dense (FP64)
// Symmetric eigendecomposition A = U diag(lam) U^T of an m x m row-major matrix
// (Householder tridiagonalisation + implicit QL).  U row-major, column i = eigvec i.
int dense_syev(int m, const double* A, double* lam, double* U);
// The same with only the first kr rows of U (kr x m row-major).
int dense_syev_rows(int m, const double* A, int kr, double* lam, double* Ur);
// A = U diag(lam) U^T kept in factored form: the Householder reflectors of the
// tridiagonalisation and the plane rotations of the QL iteration, in the order they
// were made.  U is never formed; applying it or its transpose to an m x b block costs
// O(m^2 b) instead of the O(m^3) of accumulating U.  lam is in the QL order (unsorted).
struct SymEig {
  int m = 0;
  std::vector<double> lam;
  std::vector<std::vector<double>> vs;  // reflector k acts on indices k + 1.. (empty: none)
  std::vector<int32_t> ri;              // rotation r acts on indices ri[r], ri[r] + 1
  std::vector<double> rc, rs;
};
int sym_eig_factor(int m, const double* A, SymEig& E);
// X (m x b row-major) <- U^T X, resp. U X; columns split over host threads.
void sym_eig_apply_ut(const SymEig& E, int b, double* X);
void sym_eig_apply_u(const SymEig& E, int b, double* X);
// out (m x k) = phi_1(M) B, phi_1(x) = (e^x - 1) / x, for a general m x m M (row-major),
// from exp([[M, B], [0, 0]]) by Pade scaling and squaring.  Nonzero on failure.
int dense_phi1_times(int m, const double* M, int k, const double* B, double* out);
// Cholesky of an M x M Gram with deflation: pivots at or below tol * ref drop their
// column (zero row of R, zero column of Rinv); Rinv inverts R on the kept columns.
void host_chol_deflate(int M, const std::vector<double>& G, double tol, double ref, std::vector<double>& R,
                       std::vector<double>& Rinv, std::vector<char>& keep);
// Eigenvalues only of a symmetric tridiagonal matrix (diag a, offdiag b).
int tridiag_eigvals(int m, const double* a, const double* b, double* lam);
// Solve T X = B for block tridiagonal SPD T (K diagonal blocks Ad, K-1 off-diagonal
// blocks Bo with T_{j+1,j} = Bo_j), blocks b x b row-major; B, X are (K*b) x nrhs.
int block_tridiag_solve(int K, int b, const double* Ad, const double* Bo, const double* B, int nrhs, double* X);

// ------------------------------------------------------------------ Lanczos settings
template <typename T>
constexpr int prec_of() {
  return sizeof(T) == 4 ? WL_FP32 : WL_FP64;
}

// Deflation thresholds on squared norms (Gram pivots) of the first CholQR pass,
// relative to the block's norm before projection.  Small pivots of the first pass are
// unreliable (the basis is orthonormal only to the storage precision); they are kept
// there and judged after the second pass (post_tol), which measures them directly.
template <typename T>
inline double defl_tol() {
  return sizeof(T) == 4 ? 1e-10 : 1e-24;
}

// A second CholQR pass is skipped when the first factor's kept pivots span less than
// this ratio (orthogonality after one pass ~ u_64 kappa^2: 1e-8 for FP32 storage,
// 1e-10 for FP64).
template <typename T>
inline double skip_ratio() {
  return sizeof(T) == 4 ? 1e-8 : 1e-6;
}

// After the second CholQR pass the combined factor gives the true norm of every new
// component; components below this fraction of the block's scale before projection
// are rounding noise of the stored basis (~1e-7 FP32, ~1e-16 FP64) and are dropped.
template <typename T>
inline double post_tol() {
  return sizeof(T) == 4 ? 1e-5 : 1e-10;
}

// Device-resident layout of the small matrices of one Lanczos run (doubles).
struct SmallLayout {
  int b, K;
  size_t bb;
  size_t A(int j) const { return (size_t)j * bb; }              // K blocks
  size_t B(int j) const { return (size_t)(K + j) * bb; }        // K blocks
  size_t R0() const { return (size_t)(2 * K) * bb; }
  size_t G() const { return (size_t)(2 * K + 1) * bb; }
  size_t R1() const { return (size_t)(2 * K + 2) * bb; }
  size_t Ri1() const { return (size_t)(2 * K + 3) * bb; }
  size_t R2() const { return (size_t)(2 * K + 4) * bb; }
  size_t Ri2() const { return (size_t)(2 * K + 5) * bb; }
  size_t Cc() const { return (size_t)(2 * K + 6) * bb; }        // 3 blocks
  size_t P() const { return (size_t)(2 * K + 9) * bb; }         // up to (K+2) blocks
  size_t Ref() const { return (size_t)(3 * K + 11) * bb; }      // one double: reference scale
  size_t Skip() const { return Ref() + 1; }                     // one double: second pass not needed
  size_t total() const { return Ref() + 2; }
};

// Block Lanczos steps used for an operator's evaluation at block width b.
int lanczos_steps(const wl_op* op, int64_t n, int b);
// Outer Lanczos steps of the diffusion for outer_dim requested on n rows.
int expv_outer_steps(int outer_dim, int64_t n);
// The symmetric matrix Lanczos runs on, as a A + (b0 + b1 D): A_mu(alpha) for the
// resolvent, A for the exponential (mu = 0).
void lanczos_params(const wl_op* op, double* a, double* b0, double* b1);
// Recombination coefficients F ((Ke b) x b) of phi X = V F from the projected blocks
// A_j, B_j and X = V_0 R0 (resolvent: scale T^{-1} E_1 R0; exponential: exp(beta T) E_1 R0).
wl_status lanczos_coefficients(const wl_op* op, int Ke, int b, const std::vector<double>& hA,
                               const std::vector<double>& hB, const std::vector<double>& hR0,
                               std::vector<double>& F);

// ------------------------------------------------------------------ grouped blocks
// ng blocks of width gb side by side in one n x (ng gb) row-major block (group q owns
// columns [q gb, (q + 1) gb)); the small matrices of group q sit gs doubles apart.
// Supported: FP32 with gb = 16 (matrix cores) and gb = 1 (any precision, ng <= 8).
bool grouped_supported(int prec, int gb, int ng);
// out_q + k gb^2 = (X_k)_q^T Y_q for k < nblk (X_k at X + k sX); groups whose skip flag
// (at skip + q gs) is set are left alone.  Group dg (also in launch_gupdate's Gram)
// holds independent single columns: its off-diagonal entries are set to zero.
template <typename T>
wl_status launch_ggram(wl_ctx* ctx, int64_t n, int gb, int ng, const T* X, int64_t sX, int nblk, const T* Y,
                       double* out, int64_t gs, const double* skip = nullptr, int dg = -1);
// Out_q = (wv ? wv[:, q] : alpha) .* Yin_q + beta sum_k (X_k)_q C_{q,k}, C_{q,k} at
// C + q cs + k gb^2 (gb x gb row-major); wv is n x ng.  gram_out (optional): Out_q^T Out_q
// at gram_out + q gs.  Per-group flags: skip (the group's update is elided: in-place
// updates only) and skip_gram (its Gram is not formed).  Out may alias X_k or Yin.
template <typename T>
wl_status launch_gupdate(wl_ctx* ctx, int64_t n, int gb, int ng, const T* X, int64_t sX, int nblk,
                         const double* C, int64_t cs, const T* Yin, double alpha, const T* wv, double beta, T* Out,
                         double* gram_out, int64_t gs, const double* skip = nullptr,
                         const double* skip_gram = nullptr, int dg = -1);
// y_q = x_q (count doubles) for q < ng at stride gs
wl_status launch_dcopy_groups(wl_ctx* ctx, int ng, int count, const double* x, double* y, int64_t gs);
// Deferred normalisation of the lock-step Lanczos (16-wide groups): stored blocks W_j
// with factors N_j (V_j = W_j N_j).  N_0 = I; the projection from the stored blocks'
// Gram; the next factor and three-term coefficient N_j B_j^T after each CholQR.
wl_status launch_eye_groups(wl_ctx* ctx, int ng, double* N0, int64_t gs);
wl_status launch_lanczos_proj_deferred(wl_ctx* ctx, int ng, int nbv, const double* P, const double* Nprev,
                                       const double* Ncur, double* Aout, double* Cc, int64_t gs, double* ref_out);
wl_status launch_lanczos_next(wl_ctx* ctx, int ng, const double* skip, const double* Ri1, const double* Ri2,
                              const double* Ncur, const double* B, double* Nnext, double* Ct, int64_t gs);
// Y (n x ng b) column group q = X (n x b), or X's column group q into Y (n x b)
template <typename T>
wl_status launch_group_copy(wl_ctx* ctx, int64_t n, int b, int ng, int q, const T* X, T* Y, bool into_group);

// ------------------------------------------------------------------ discrete-time diffusion
// out = x^(-1) (mode 0), x^(-1/2) (mode 1) or x^(1/2) (mode 2), elementwise over n
template <typename T>
wl_status launch_wpow(wl_ctx* ctx, int64_t n, const T* x, int mode, T* out);
// out = x / *den with den one device double
template <typename T>
wl_status launch_div_by(wl_ctx* ctx, int64_t n, const T* x, const double* den, T* out);

// Upper bounds (bytes) of the reduction partials one Gram of nblk blocks of width b
// against a block of width b, or one block update of width b with its Gram, may use
// in ctx->partials (they follow the launch shapes of launch_gram / launch_update).
size_t gram_partials_bound(int64_t n, int prec, int b, int nblk);
size_t update_partials_bound(int64_t n, int prec, int b);

// ------------------------------------------------------------------ drivers
template <typename T>
wl_status ensure_w(wl_op* op);
template <typename T>
wl_status phi_apply_impl(wl_op* op, const T* X, T* Y, int b, const T* wv, const T* Xw);
template <typename T>
wl_status phi_arnoldi(wl_op* op, const T* X, T* Y, int b, const T* wv, const T* Xw);
template <typename T>
wl_status expv_impl(wl_op* op, const T* U0, int b, const double* t, int nt, T* const* Y, int outer_dim,
                    double* err_est);
template <typename T>
wl_status markov_gap_impl(wl_op* op, int outer_dim, uint64_t seed, double* lambda2, double* lambda_min,
                          double* gap);
wl_status lanczos_extreme(wl_graph* g, int kind, double mu, double t, int steps, double* lo, double* hi);
template <typename T>
wl_status laplacian_rho_impl(wl_op* op, int steps, uint64_t seed, double* rho);

// One Lanczos operator on a wide block split into G column groups of b columns, each
// group its own block Lanczos process, all in lock step through the grouped kernels
// (one sparse product per step for all groups).  The handle keeps its basis between
// calls.  Create after the operator's walk degrees are cached (the Laplacian finish
// needs them).  multi_groups_apply sets *done = false and launches nothing when the
// grouped kernels do not cover the shape (the caller then applies the operator itself).
wl_status multi_groups_create(wl_op* op, int G, wl_multi** out);
void multi_groups_destroy(wl_multi* m);
template <typename T>
wl_status multi_groups_apply(wl_multi* m, const T* X, int b, T* Y, bool laplacian, bool* done);

// ------------------------------------------------------------------ rational approximation (host)
// AAA on real samples F = f(Z) (N points): support points z, values f, weights w of the
// barycentric approximant; max_err its largest error on Z.  0 on success.
int aaa_real(int64_t N, const double* Z, const double* F, double tol, int mmax, std::vector<double>& z,
             std::vector<double>& f, std::vector<double>& w, double* max_err);
// Zeros of sum_j w_j / (x - z_j) (the poles of the approximant).
int aaa_poles(const std::vector<double>& z, const std::vector<double>& w, std::vector<std::complex<double>>& poles);
// The points exp(-x) is sampled on over [0, xmax], and the AAA poles of exp(-x) there
// (real poles on the interval itself dropped).
void exp_sample_points(double xmax, std::vector<double>& Z);
int exp_poles(double xmax, double tol, int mmax, std::vector<std::complex<double>>& poles, double* max_err);
// Leave-one-out Nystrom trace estimate from H = Omega^T Y and G = Y^T Y (M x M,
// row-major): the mean over j of tr F_(j) + omega_j^T (F - F_(j)) omega_j and its
// standard error.  0 on success.
int xnys_trace_host(int M, const std::vector<double>& H, const std::vector<double>& G, double rcond, double* trace,
                    double* trace_err);
