// Several walk operators of one graph evaluated together.
//
// Every operator runs on its own column group of one wide block n x (nops b):
// operator q owns columns [q b, (q+1) b).  One sparse product per step serves all of
// them, with every group's coefficients read from a small table.  Rows of b = 16 FP32
// values are half of a 128-byte cache line; two operators side by side gather one
// full line per neighbour, four gather two, so the same lines serve more work.
//
//   * truncated series (eq. qrec: P_1 = s A X, P_2 = s A P_1 - s^2 mu D X,
//     P_k = s A P_{k-1} + s^2 mu (mu - D) P_{k-2}, S = sum_k omega_k P_k): all groups
//     step together, a group whose series has ended gets zero coefficients;
//   * Lanczos (Sec. 4.1): one block Lanczos process per group on that operator's
//     symmetric matrix (A_mu(alpha) for the resolvent, A for the exponential), in
//     lock step: the sparse product carries every group's diagonal coefficients and
//     its own three-term subtraction (block-diagonal B_{j-1}^T), and the projection,
//     CholQR and basis updates of all groups run as one pass over the wide block
//     (grouped kernels) with one small-matrix launch for all groups.  Each group's
//     coefficients come from its own projected matrix, truncated to that operator's
//     number of steps.
#include <algorithm>
#include <cmath>
#include <vector>

#include "wl_internal.h"

struct wl_multi {
  wl_graph* g = nullptr;
  int nops = 0;
  int prec = WL_FP32;
  int method = WL_M_RECURRENCE;
  int Kmax = 0;
  std::vector<int> K;
  std::vector<wl_op_desc> desc;  // Lanczos groups: each operator's description
  std::vector<char> fin_at;  // fin_at[k]: some operator's series ends at step k
  DevBuf tab;      // [Kmax][nops][5] {a, b0, b1, omega, finish}
  DevBuf tab_phi;  // the same without the finish flags
  DevBuf W;        // walk degrees, n x nops
  bool w_valid = false;
  DevBuf Xrep, A, B, ones;
  DevBuf ltab;                      // Lanczos groups: [nops][5] {a, b0, b1, 0, 0}
  DevBuf basis, small, coef, tmpX, tmpY, tmpW;
  // walk degrees riding beside the blocks (wl_multi_apply_fdeg): one extra group of 16
  // columns whose column q < nops is operator q's vector of ones
  DevBuf tab_pk, tab_pk_phi;  // series: [Kmax][2 nops][5], entries nops + q without finish
  DevBuf cmap;                // operator of each column of the packed block
  int cmap_b = 0;
  DevBuf Xpk, Ypk, Wg;
};

namespace {

template <typename T>
__global__ void k_replicate(int64_t n, int b, int nops, const T* __restrict__ X, T* __restrict__ Xr) {
  const int64_t wd = (int64_t)b * nops;
  const int64_t total = n * wd;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / wd;
    const int c = (int)(i - r * wd) % b;
    Xr[i] = X[r * b + c];
  }
}

// Packed block: X in each of the nops groups of b columns, then a group of 16 columns
// whose column q < nops is a vector of ones (operator q's walk degrees), zero beyond.
template <typename T>
__global__ void k_pack_fdeg(int64_t n, int b, int nx, int nops, const T* __restrict__ X, T* __restrict__ Xp) {
  const int xw = b * nx;
  const int64_t wd = (int64_t)xw + 16;
  const int64_t total = n * wd;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / wd;
    const int c = (int)(i - r * wd);
    Xp[i] = c < xw ? X[r * b + c % b] : (c - xw < nops ? T(1) : T(0));
  }
}

// Y (n x nx b) and W (n x nops) out of the packed block
template <typename T>
__global__ void k_unpack_fdeg(int64_t n, int b, int nx, int nops, const T* __restrict__ Yp, T* __restrict__ Y,
                              T* __restrict__ W) {
  const int xw = b * nx;
  const int64_t wd = (int64_t)xw + 16;
  const int64_t ow = (int64_t)xw + nops;
  const int64_t total = n * ow;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ow;
    const int c = (int)(i - r * ow);
    if (c < xw)
      Y[r * xw + c] = Yp[r * wd + c];
    else
      W[r * nops + (c - xw)] = Yp[r * wd + c];
  }
}

// Wg (n x (nx + 1)) = [W_0 .. W_{nx-1} | 0]: group-indexed finish weights of the packed
// Lanczos recombination (W is n x nops; the walk-degree group takes no finish)
template <typename T>
__global__ void k_wg(int64_t n, int nx, int nops, const T* __restrict__ W, T* __restrict__ Wg) {
  const int64_t total = n * (nx + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / (nx + 1);
    const int c = (int)(i - r * (nx + 1));
    Wg[i] = c < nx ? W[r * nops + c] : T(0);
  }
}

int elem_grid(int64_t count) { return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (count + 255) / 256)); }

template <typename T>
wl_status multi_apply(wl_multi* m, const T* X, int b, T* Y, bool laplacian) {
  wl_graph* g = m->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  if (n == 0) return WL_OK;
  const int wd = b * m->nops;
  const size_t bytes = (size_t)n * wd * sizeof(T);
  WL_TRY(m->Xrep.ensure(bytes));
  WL_TRY(m->A.ensure(bytes));
  WL_TRY(m->B.ensure(bytes));
  T* Xr = m->Xrep.as<T>();
  T* A = m->A.as<T>();
  T* Bf = m->B.as<T>();
  const int grid = (int)std::min<int64_t>(8192, (n * wd + 255) / 256);
  hipLaunchKernelGGL(k_replicate<T>, dim3(grid), dim3(256), 0, ctx->stream, n, b, m->nops, X, Xr);
  WL_HIP(hipGetLastError());
  const double* tab = (laplacian ? m->tab : m->tab_phi).as<double>();
  const int64_t ts = (int64_t)m->nops * 5;
  const SpmmShape sh = shape_for(g, m->prec, wd);
  auto base = [&](int k) {
    EpiArgs<T> ep;
    ep.ctab = tab + (int64_t)(k - 1) * ts;
    ep.cgw = b;
    ep.Sin = k == 1 ? Xr : Y;
    ep.Sout = Y;
    ep.s0 = 1.0;
    if (laplacian && m->fin_at[k]) {  // only steps where some group finishes read w and X
      ep.wv = m->W.as<T>();
      ep.wld = m->nops;
      ep.Xw = Xr;
    }
    ep.kclass = wd >= 32 ? WL_KC_MULTI : WL_KC_OTHER_SPMM;
    return ep;
  };
  // step 1: P_1 = s A X in every group; S = X + omega_1 P_1
  WL_TRY(launch_spmm<T>(g, Xr, m->Kmax == 1 ? nullptr : A, wd, base(1), sh));
  const T* Pm2 = Xr;
  T* Pm1 = A;
  for (int k = 2; k <= m->Kmax; ++k) {
    EpiArgs<T> ep = base(k);
    ep.Z = Pm2;
    // P_k overwrites P_{k-2} row by row (same lanes read and write a row); P_0 = Xrep
    // is kept for the finish
    T* out = (k == 2) ? Bf : const_cast<T*>(Pm2);
    WL_TRY(launch_spmm<T>(g, Pm1, k == m->Kmax ? nullptr : out, wd, ep, sh));
    Pm2 = Pm1;
    Pm1 = out;
  }
  return WL_OK;
}

// A stand-in operator with group q's description (no buffers of the caller's op).
void group_op(const wl_multi* m, int q, wl_op* op) {
  op->g = m->g;
  op->d = m->desc[q];
  op->K = m->K[q];
}

// Where a group's small matrices sit: SmallLayout Ly from the group's base (groups gs
// doubles apart), then the deferred-normalisation factors N_j (j = 0..K) and the
// three-term coefficient of the next product.
struct LockLayout {
  SmallLayout Ly;
  int64_t noff, ctoff, gs;
  explicit LockLayout(int K) : Ly{16, K, (size_t)256} {
    noff = (int64_t)((Ly.total() + 1) / 2 * 2);
    ctoff = noff + (int64_t)(K + 1) * 256;
    gs = ctoff + 256;
  }
  int64_t N(int j) const { return noff + (int64_t)j * 256; }
};

// K steps of G block Lanczos processes of 16 columns in lock step on Xr (n x 16 G), one
// sparse product per step for all (Sec. 4.1): the three-term subtraction in the product's
// epilogue, the projection against the current block (with a second local pass
// against the previous one when any operator asks for reorth >= 1) and CholQR with
// deflation.
// Deferred normalisation: slot j of
// the basis holds W_j with V_j = W_j N_j orthonormal (N_j from the step's CholQR), and
// the products, Grams and updates that read W_j apply N_j on the small side, so the
// normalising pass over the block is made only where a second CholQR pass is needed.
// Group dg (or -1) holds independent single-column processes (diagonal Grams); cmap
// (or null) maps columns to the operators of ltab.
template <typename T>
wl_status lockstep_lanczos(wl_multi* m, const T* Xr, int G, int dg, int K, const LockLayout& L, T* basis,
                           double* S, const int32_t* cmap) {
  wl_graph* g = m->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  const SmallLayout& Ly = L.Ly;
  const int64_t gs = L.gs;
  const int wd = G * 16;
  const int64_t blk = n * wd;
  const double tol = defl_tol<T>(), ptol = post_tol<T>();
  bool local2 = false;
  for (const auto& d : m->desc) local2 = local2 || d.reorth >= 1;
  // V_0 R0 = Xr per group by CholQR2 (the walk-degree group: each column normalised)
  WL_TRY(launch_ggram<T>(ctx, n, 16, G, Xr, 0, 1, Xr, S + Ly.G(), gs, nullptr, dg));
  WL_TRY(launch_chol(ctx, 16, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R1(), S + Ly.Ri1(), nullptr, nullptr, G, gs,
                     S + Ly.Ref(), nullptr, 0.0, nullptr, 0.0, nullptr, dg));
  WL_TRY(launch_gupdate<T>(ctx, n, 16, G, Xr, 0, 1, S + Ly.Ri1(), gs, nullptr, 0.0, nullptr, 1.0, basis, S + Ly.G(),
                           gs, nullptr, nullptr, dg));
  WL_TRY(launch_chol(ctx, 16, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(), S + Ly.R0(),
                     G, gs, nullptr, S + Ly.Ref(), ptol, nullptr, 0.0, nullptr, dg));
  WL_TRY(launch_gupdate<T>(ctx, n, 16, G, basis, 0, 1, S + Ly.Ri2(), gs, nullptr, 0.0, nullptr, 1.0, basis, nullptr,
                           gs));
  WL_TRY(launch_eye_groups(ctx, G, S + L.N(0), gs));
  const SpmmShape sh = shape_for(g, m->prec, wd);
  for (int j = 0; j < K; ++j) {
    T* Vj = basis + (size_t)j * blk;
    T* Vn = Vj + blk;
    const T* Vp = j > 0 ? Vj - blk : nullptr;
    // W' = Op_q(V_j) - V_{j-1} B_{j-1,q}^T = Op_q(W_j) N_j - W_{j-1} (N_{j-1} B_{j-1}^T)
    EpiArgs<T> ep;
    ep.ctab = m->ltab.as<double>();
    ep.cgw = 16;
    ep.cmap = cmap;
    ep.cgs = gs;
    ep.Z = Vj;
    if (j > 0) ep.Nm = S + L.N(j);  // N_0 = I: V_0 is stored normalised
    if (Vp) {
      ep.Z2 = Vp;
      ep.C = S + L.ctoff;
      ep.transC = 0;
    }
    ep.kclass = wd >= 32 ? WL_KC_MULTI_LANCZOS : WL_KC_OTHER_SPMM;
    WL_TRY(launch_spmm<T>(g, Vj, Vn, wd, ep, sh));
    // projection against V_j (reorth 0: the epilogue's three-term subtraction has taken
    // V_{j-1} out), or a second local pass against V_{j-1} too (reorth 1)
    const int nbv = j > 0 && local2 ? 2 : 1;
    const T* Vlo = nbv == 2 ? Vp : Vj;
    WL_TRY(launch_ggram<T>(ctx, n, 16, G, Vlo, blk, nbv + 1, Vn, S + Ly.P(), gs, nullptr, dg));
    WL_TRY(launch_lanczos_proj_deferred(ctx, G, nbv, S + Ly.P(), nbv == 2 ? S + L.N(j - 1) : nullptr, S + L.N(j),
                                        S + Ly.A(j), S + Ly.Cc(), gs, S + Ly.Ref()));
    WL_TRY(launch_gupdate<T>(ctx, n, 16, G, Vlo, blk, nbv + 1, S + Ly.Cc(), gs, nullptr, 0.0, nullptr, 1.0, Vn,
                             S + Ly.G(), gs, nullptr, nullptr, dg));
    // the walk-degree columns are judged against their own scale before projection
    // (the diagonal of W'^T W', the last block of P)
    WL_TRY(launch_chol(ctx, 16, S + Ly.G(), tol, nullptr, nullptr, nullptr, S + Ly.Ri1(), nullptr, S + Ly.R1(), G,
                       gs, nullptr, S + Ly.Ref(), ptol, S + Ly.Skip(), skip_ratio<T>(), nullptr, dg,
                       S + Ly.P() + (size_t)nbv * 256));
    if (j + 1 == K) {
      WL_TRY(launch_dcopy_groups(ctx, G, 256, S + Ly.R1(), S + Ly.B(j), gs));
      break;
    }
    // only groups whose first factor was ill conditioned normalise the block now (and
    // take a second CholQR pass); the others keep W with N_{j+1} = R1^{-1}
    WL_TRY(launch_gupdate<T>(ctx, n, 16, G, Vn, 0, 1, S + Ly.Ri1(), gs, nullptr, 0.0, nullptr, 1.0, Vn, S + Ly.G(),
                             gs, S + Ly.Skip(), S + Ly.Skip(), dg));
    WL_TRY(launch_chol(ctx, 16, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(),
                       S + Ly.B(j), G, gs, nullptr, nullptr, 0.0, nullptr, 0.0, S + Ly.Skip(), dg));
    WL_TRY(launch_lanczos_next(ctx, G, S + Ly.Skip(), S + Ly.Ri1(), S + Ly.Ri2(), S + L.N(j), S + Ly.B(j),
                               S + L.N(j + 1), S + L.ctoff, gs));
  }
  return WL_OK;
}

// Coefficients of the stored blocks from a group's true ones: C_j <- N_j C_j (16 x 16
// blocks, j < Ke; hS the group's small matrices on the host).
void apply_deferred(const double* hSq, const LockLayout& L, int Ke, std::vector<double>& F) {
  std::vector<double> t(256);
  for (int j = 0; j < Ke; ++j) {
    const double* N = hSq + L.N(j);
    double* C = F.data() + (size_t)j * 256;
    for (int r = 0; r < 16; ++r)
      for (int c = 0; c < 16; ++c) {
        double a = 0.0;
        for (int k = 0; k < 16; ++k) a += N[r * 16 + k] * C[k * 16 + c];
        t[r * 16 + c] = a;
      }
    std::copy(t.begin(), t.end(), C);
  }
}

// Per-operator evaluation into the wide output (shapes the grouped kernels do not
// cover, or a Krylov space small enough to need full reorthogonalisation).
template <typename T>
wl_status multi_lanczos_each(wl_multi* m, const T* X, int b, T* Y, const T* wv) {
  wl_graph* g = m->g;
  const int64_t n = g->n;
  WL_TRY(m->tmpY.ensure((size_t)n * b * sizeof(T)));
  if (wv) WL_TRY(m->tmpW.ensure((size_t)n * sizeof(T)));
  for (int q = 0; q < m->nops; ++q) {
    wl_op op;
    group_op(m, q, &op);
    if (wv) WL_TRY(launch_group_copy<T>(g->ctx, n, 1, m->nops, q, wv, m->tmpW.as<T>(), false));
    WL_TRY(phi_apply_impl<T>(&op, X, m->tmpY.as<T>(), b, wv ? m->tmpW.as<T>() : nullptr, wv ? X : nullptr));
    WL_TRY(launch_group_copy<T>(g->ctx, n, b, m->nops, q, m->tmpY.as<T>(), Y, true));
    WL_HIP(hipStreamSynchronize(g->ctx->stream));  // op's buffers are freed on return
  }
  return WL_OK;
}

// All groups' block Lanczos in lock step on the wide block Xr (n x nops b, every group
// holding the same X), then Y = V F per group (with the Laplacian finish
// Y_q = wv_q .* Xr_q - V F_q when wv is given); groups of single columns (any
// precision), each basis block normalised in place.
template <typename T>
wl_status multi_lanczos_plain(wl_multi* m, const T* X, const T* Xr, int b, T* Y, const T* wv) {
  wl_graph* g = m->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  const int G = m->nops;
  std::vector<int> Kq(G);
  int K = 1;
  for (int q = 0; q < G; ++q) {
    wl_op op;
    group_op(m, q, &op);
    Kq[q] = lanczos_steps(&op, n, b);
    K = std::max(K, Kq[q]);
  }
  bool local = true;
  for (int q = 0; q < G; ++q) local = local && m->desc[q].reorth <= 1;
  if (!grouped_supported(m->prec, b, G) || (int64_t)(K + 1) * b * 2 > n || !local)
    return multi_lanczos_each<T>(m, X, b, Y, wv);
  const int wd = G * b;
  const int64_t blk = n * wd;
  SmallLayout Ly{b, K, (size_t)b * b};
  const int64_t gs = (int64_t)((Ly.total() + 1) / 2 * 2);
  WL_TRY(m->small.ensure((size_t)G * gs * sizeof(double)));
  WL_TRY(m->basis.ensure((size_t)(K + 1) * blk * sizeof(T)));
  double* S = m->small.as<double>();
  T* basis = m->basis.as<T>();
  bool local2 = false;
  for (const auto& d : m->desc) local2 = local2 || d.reorth >= 1;
  const double tol = defl_tol<T>(), ptol = post_tol<T>();
  // V_0 R0 = Xr per group by CholQR2
  WL_TRY(launch_ggram<T>(ctx, n, b, G, Xr, 0, 1, Xr, S + Ly.G(), gs));
  WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R1(), S + Ly.Ri1(), nullptr, nullptr, G, gs,
                     S + Ly.Ref()));
  WL_TRY(launch_gupdate<T>(ctx, n, b, G, Xr, 0, 1, S + Ly.Ri1(), gs, nullptr, 0.0, nullptr, 1.0, basis, S + Ly.G(),
                           gs));
  WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(), S + Ly.R0(),
                     G, gs, nullptr, S + Ly.Ref(), ptol));
  WL_TRY(launch_gupdate<T>(ctx, n, b, G, basis, 0, 1, S + Ly.Ri2(), gs, nullptr, 0.0, nullptr, 1.0, basis, nullptr,
                           gs));
  const SpmmShape sh = shape_for(g, m->prec, wd);
  for (int j = 0; j < K; ++j) {
    T* Vj = basis + (size_t)j * blk;
    T* Vn = Vj + blk;
    const T* Vp = j > 0 ? Vj - blk : nullptr;
    // W' = Op_q(V_j) - V_{j-1} B_{j-1,q}^T in every group
    EpiArgs<T> ep;
    ep.ctab = m->ltab.as<double>();
    ep.cgw = b;
    ep.Z = Vj;
    if (Vp) {
      ep.Z2 = Vp;
      ep.C = S + Ly.B(j - 1);
      ep.cgs = gs;
      ep.transC = 1;
    }
    ep.kclass = wd >= 32 ? WL_KC_MULTI_LANCZOS : WL_KC_OTHER_SPMM;
    WL_TRY(launch_spmm<T>(g, Vj, Vn, wd, ep, sh));
    const int nbv = j > 0 && local2 ? 2 : 1;  // reorth 1: second local pass against V_{j-1}
    const T* Vlo = nbv == 2 ? Vp : Vj;
    WL_TRY(launch_ggram<T>(ctx, n, b, G, Vlo, blk, nbv + 1, Vn, S + Ly.P(), gs));
    WL_TRY(launch_lanczos_proj(ctx, b, nbv, S + Ly.P(), S + Ly.A(j), S + Ly.Cc(), S + Ly.Ref(), G, gs));
    WL_TRY(launch_gupdate<T>(ctx, n, b, G, Vlo, blk, nbv + 1, S + Ly.Cc(), gs, nullptr, 0.0, nullptr, 1.0, Vn,
                             S + Ly.G(), gs));
    WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, nullptr, S + Ly.Ri1(), nullptr, S + Ly.R1(), G, gs,
                       nullptr, S + Ly.Ref(), ptol, S + Ly.Skip(), skip_ratio<T>()));
    if (j + 1 == K) {
      WL_TRY(launch_dcopy_groups(ctx, G, b * b, S + Ly.R1(), S + Ly.B(j), gs));
      break;
    }
    // second CholQR pass only in groups whose first factor was ill conditioned
    WL_TRY(launch_gupdate<T>(ctx, n, b, G, Vn, 0, 1, S + Ly.Ri1(), gs, nullptr, 0.0, nullptr, 1.0, Vn, S + Ly.G(),
                             gs, nullptr, S + Ly.Skip()));
    WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(),
                       S + Ly.B(j), G, gs, nullptr, nullptr, 0.0, nullptr, 0.0, S + Ly.Skip()));
    WL_TRY(launch_gupdate<T>(ctx, n, b, G, Vn, 0, 1, S + Ly.Ri2(), gs, nullptr, 0.0, nullptr, 1.0, Vn, nullptr, gs,
                             S + Ly.Skip(), nullptr));
  }
  std::vector<double> hS((size_t)G * gs);
  WL_HIP(hipMemcpyAsync(hS.data(), S, hS.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  const size_t bb = (size_t)b * b;
  std::vector<std::vector<double>> Fq(G);
  std::vector<int> Keq(G);
  int Kr = 1;
  for (int q = 0; q < G; ++q) {
    const double* Sq = hS.data() + (size_t)q * gs;
    const int Kg = Kq[q];
    std::vector<double> hA(Sq + Ly.A(0), Sq + Ly.A(0) + Kg * bb), hB(Sq + Ly.B(0), Sq + Ly.B(0) + Kg * bb);
    std::vector<double> hR0(Sq + Ly.R0(), Sq + Ly.R0() + bb);
    int Ke = Kg;  // stop after the first block whose coupling vanished entirely
    for (int jj = 0; jj + 1 < Kg; ++jj) {
      double s2 = 0.0;
      for (size_t e = 0; e < bb; ++e) s2 += hB[jj * bb + e] * hB[jj * bb + e];
      if (s2 == 0.0) {
        Ke = jj + 1;
        break;
      }
    }
    for (double v : hA)
      if (!std::isfinite(v)) {
        wl_set_error("block Lanczos produced non-finite coefficients (operator %d)", q);
        return WL_ENUMERIC;
      }
    wl_op op;
    group_op(m, q, &op);
    WL_TRY(lanczos_coefficients(&op, Ke, b, hA, hB, hR0, Fq[q]));
    Keq[q] = Ke;
    Kr = std::max(Kr, Ke);
  }
  // C_{q,k} = rows [k b, (k+1) b) of F_q (zero past the group's own dimension)
  std::vector<double> F((size_t)G * Kr * bb, 0.0);
  for (int q = 0; q < G; ++q)
    std::copy(Fq[q].begin(), Fq[q].end(), F.begin() + (size_t)q * Kr * bb);
  WL_TRY(m->coef.ensure(F.size() * sizeof(double)));
  WL_HIP(hipMemcpyAsync(m->coef.p, F.data(), F.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  WL_TRY(launch_gupdate<T>(ctx, n, b, G, basis, blk, Kr, m->coef.as<double>(), (int64_t)Kr * bb, wv ? Xr : nullptr,
                           0.0, wv, wv ? -1.0 : 1.0, Y, nullptr, 0));
  WL_HIP(hipStreamSynchronize(ctx->stream));  // F is host memory of this call
  return WL_OK;
}

// All groups' block Lanczos in lock step on the wide block Xr (n x nops b, every group
// holding the same X), then Y = V F per group (with the Laplacian finish
// Y_q = wv_q .* Xr_q - V F_q when wv is given).
template <typename T>
wl_status multi_lanczos(wl_multi* m, const T* X, const T* Xr, int b, T* Y, const T* wv) {
  wl_graph* g = m->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  const int G = m->nops;
  std::vector<int> Kq(G);
  int K = 1;
  for (int q = 0; q < G; ++q) {
    wl_op op;
    group_op(m, q, &op);
    Kq[q] = lanczos_steps(&op, n, b);
    K = std::max(K, Kq[q]);
  }
  bool local = true;
  for (int q = 0; q < G; ++q) local = local && m->desc[q].reorth <= 1;
  if (!grouped_supported(m->prec, b, G) || (int64_t)(K + 1) * b * 2 > n || !local)
    return multi_lanczos_each<T>(m, X, b, Y, wv);
  if (b != 16) return multi_lanczos_plain<T>(m, X, Xr, b, Y, wv);
  const int wd = G * b;
  const int64_t blk = n * wd;
  const LockLayout L(K);
  const SmallLayout& Ly = L.Ly;
  const int64_t gs = L.gs;
  WL_TRY(m->small.ensure((size_t)G * gs * sizeof(double)));
  WL_TRY(m->basis.ensure((size_t)(K + 1) * blk * sizeof(T)));
  double* S = m->small.as<double>();
  T* basis = m->basis.as<T>();
  WL_TRY(lockstep_lanczos<T>(m, Xr, G, -1, K, L, basis, S, nullptr));
  std::vector<double> hS((size_t)G * gs);
  WL_HIP(hipMemcpyAsync(hS.data(), S, hS.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  const size_t bb = (size_t)b * b;
  std::vector<std::vector<double>> Fq(G);
  std::vector<int> Keq(G);
  int Kr = 1;
  for (int q = 0; q < G; ++q) {
    const double* Sq = hS.data() + (size_t)q * gs;
    const int Kg = Kq[q];
    std::vector<double> hA(Sq + Ly.A(0), Sq + Ly.A(0) + Kg * bb), hB(Sq + Ly.B(0), Sq + Ly.B(0) + Kg * bb);
    std::vector<double> hR0(Sq + Ly.R0(), Sq + Ly.R0() + bb);
    int Ke = Kg;  // stop after the first block whose coupling vanished entirely
    for (int jj = 0; jj + 1 < Kg; ++jj) {
      double s2 = 0.0;
      for (size_t e = 0; e < bb; ++e) s2 += hB[jj * bb + e] * hB[jj * bb + e];
      if (s2 == 0.0) {
        Ke = jj + 1;
        break;
      }
    }
    for (double v : hA)
      if (!std::isfinite(v)) {
        wl_set_error("block Lanczos produced non-finite coefficients (operator %d)", q);
        return WL_ENUMERIC;
      }
    wl_op op;
    group_op(m, q, &op);
    WL_TRY(lanczos_coefficients(&op, Ke, b, hA, hB, hR0, Fq[q]));
    apply_deferred(Sq, L, Ke, Fq[q]);  // for the stored blocks W_j = V_j N_j^{-1}
    Keq[q] = Ke;
    Kr = std::max(Kr, Ke);
  }
  // C_{q,k} = rows [k b, (k+1) b) of F_q (zero past the group's own dimension)
  std::vector<double> F((size_t)G * Kr * bb, 0.0);
  for (int q = 0; q < G; ++q)
    std::copy(Fq[q].begin(), Fq[q].end(), F.begin() + (size_t)q * Kr * bb);
  WL_TRY(m->coef.ensure(F.size() * sizeof(double)));
  WL_HIP(hipMemcpyAsync(m->coef.p, F.data(), F.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  WL_TRY(launch_gupdate<T>(ctx, n, b, G, basis, blk, Kr, m->coef.as<double>(), (int64_t)Kr * bb, wv ? Xr : nullptr,
                           0.0, wv, wv ? -1.0 : 1.0, Y, nullptr, 0));
  WL_HIP(hipStreamSynchronize(ctx->stream));  // F is host memory of this call
  return WL_OK;
}

template <typename T>
wl_status multi_dispatch(wl_multi* m, const T* X, int b, T* Y, bool laplacian);

template <typename T>
wl_status multi_ensure_w(wl_multi* m) {
  if (m->w_valid) return WL_OK;
  wl_graph* g = m->g;
  const int64_t n = g->n;
  WL_TRY(m->W.ensure((size_t)std::max<int64_t>(n, 1) * m->nops * sizeof(T)));
  WL_TRY(m->ones.ensure((size_t)std::max<int64_t>(n, 1) * sizeof(T)));
  WL_TRY(launch_fill<T>(g->ctx, n, T(1), m->ones.as<T>()));
  WL_TRY(multi_dispatch<T>(m, m->ones.as<T>(), 1, m->W.as<T>(), false));
  WL_HIP(hipStreamSynchronize(g->ctx->stream));
  m->w_valid = true;
  return WL_OK;
}

template <typename T>
wl_status multi_dispatch(wl_multi* m, const T* X, int b, T* Y, bool laplacian) {
  if (m->method == WL_M_RECURRENCE) return multi_apply<T>(m, X, b, Y, laplacian);
  wl_graph* g = m->g;
  const int64_t n = g->n;
  if (n == 0) return WL_OK;
  WL_TRY(m->Xrep.ensure((size_t)n * b * m->nops * sizeof(T)));
  T* Xr = m->Xrep.as<T>();
  const int grid = (int)std::min<int64_t>(8192, (n * b * m->nops + 255) / 256);
  hipLaunchKernelGGL(k_replicate<T>, dim3(grid), dim3(256), 0, g->ctx->stream, n, b, m->nops, X, Xr);
  WL_HIP(hipGetLastError());
  return multi_lanczos<T>(m, X, Xr, b, Y, laplacian ? m->W.as<T>() : nullptr);
}

// ------------------------------------------------------------------ walk degrees alongside
// The operator of every column of the packed block (width nops b + 16): group q's
// columns take operator q (series: table entry q, with its finish); walk-degree column
// q takes operator q without finish (series: entry nops + q; Lanczos: q, the same
// matrix); padding -1.
wl_status ensure_cmap(wl_multi* m, int b, int nx, bool series) {
  const int key = (series ? 1 : -1) * (b * 128 + nx);
  if (m->cmap_b == key && m->cmap.p) return WL_OK;
  const int xw = nx * b, wd = xw + 16;
  std::vector<int32_t> h(wd);
  for (int c = 0; c < wd; ++c)
    h[c] = c < xw ? c / b : (c - xw < m->nops ? (series ? m->nops : 0) + (c - xw) : -1);
  WL_TRY(m->cmap.ensure(h.size() * 4));
  WL_HIP(hipMemcpyAsync(m->cmap.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, m->g->ctx->stream));
  WL_HIP(hipStreamSynchronize(m->g->ctx->stream));  // h is host memory of this call
  m->cmap_b = key;
  return WL_OK;
}

// Truncated series of every operator on X and on the vector of ones together: one
// sparse product per step over the packed block.
template <typename T>
wl_status multi_series_fdeg(wl_multi* m, const T* X, int b, int nx, T* Y, T* W, bool laplacian) {
  wl_graph* g = m->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  const int nops = m->nops;
  const int wd = nx * b + 16;
  const size_t bytes = (size_t)n * wd * sizeof(T);
  WL_TRY(ensure_cmap(m, b, nx, true));
  WL_TRY(m->Xpk.ensure(bytes));
  WL_TRY(m->A.ensure(bytes));
  WL_TRY(m->B.ensure(bytes));
  WL_TRY(m->Ypk.ensure(bytes));
  T* Xr = m->Xpk.as<T>();
  T* A = m->A.as<T>();
  T* Bf = m->B.as<T>();
  T* Yp = m->Ypk.as<T>();
  hipLaunchKernelGGL(k_pack_fdeg<T>, dim3(elem_grid(n * wd)), dim3(256), 0, ctx->stream, n, b, nx, nops, X, Xr);
  WL_HIP(hipGetLastError());
  const double* tab = (laplacian ? m->tab_pk : m->tab_pk_phi).as<double>();
  const int64_t ts = (int64_t)2 * nops * 5;
  const SpmmShape sh = shape_for(g, m->prec, wd);
  auto base = [&](int k) {
    EpiArgs<T> ep;
    ep.ctab = tab + (int64_t)(k - 1) * ts;
    ep.cgw = b;
    ep.cmap = m->cmap.as<int32_t>();
    ep.Sin = k == 1 ? Xr : Yp;
    ep.Sout = Yp;
    ep.s0 = 1.0;
    if (laplacian && m->fin_at[k]) {
      ep.wv = m->W.as<T>();
      ep.wld = nops;
      ep.Xw = Xr;
    }
    ep.kclass = WL_KC_MULTI;
    return ep;
  };
  WL_TRY(launch_spmm<T>(g, Xr, m->Kmax == 1 ? nullptr : A, wd, base(1), sh));
  const T* Pm2 = Xr;
  T* Pm1 = A;
  for (int k = 2; k <= m->Kmax; ++k) {
    EpiArgs<T> ep = base(k);
    ep.Z = Pm2;
    T* out = (k == 2) ? Bf : const_cast<T*>(Pm2);
    WL_TRY(launch_spmm<T>(g, Pm1, k == m->Kmax ? nullptr : out, wd, ep, sh));
    Pm2 = Pm1;
    Pm1 = out;
  }
  hipLaunchKernelGGL(k_unpack_fdeg<T>, dim3(elem_grid(n * (nx * b + nops))), dim3(256), 0, ctx->stream, n, b, nx,
                     nops, Yp, Y, W);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

// Block Lanczos of every operator on X (16-column groups) and single-column Lanczos of
// every operator on the vector of ones, all in lock step: the ones ride in one more
// 16-column group whose Grams are diagonal (its columns are independent processes of
// different operators), so one sparse product and one pass of each grouped kernel per
// step serve both.  Returns false in *done when the shape is not covered.
template <typename T>
wl_status multi_lanczos_fdeg(wl_multi* m, const T* X, int b, int nx, T* Y, T* W, bool laplacian, bool* done) {
  *done = false;
  wl_graph* g = m->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  const int nops = m->nops;
  const int G = nx + 1, dgi = nx;
  if (b != 16 || nops > 16 || !grouped_supported(m->prec, 16, G)) return WL_OK;
  std::vector<int> Kq(nx), Kd(nops);
  int K = 1;
  bool local = true;
  for (int q = 0; q < nops; ++q) {
    wl_op op;
    group_op(m, q, &op);
    if (q < nx) Kq[q] = lanczos_steps(&op, n, 16);
    Kd[q] = lanczos_steps(&op, n, 1);
    K = std::max(K, std::max(q < nx ? Kq[q] : 1, Kd[q]));
    local = local && m->desc[q].reorth <= 1;
  }
  if (!local || (int64_t)(K + 1) * 16 * 2 > n) return WL_OK;
  const int wd = G * 16;
  const int64_t blk = n * wd;
  WL_TRY(ensure_cmap(m, 16, nx, false));
  WL_TRY(m->Xpk.ensure((size_t)blk * sizeof(T)));
  WL_TRY(m->Ypk.ensure((size_t)blk * sizeof(T)));
  T* Xr = m->Xpk.as<T>();
  hipLaunchKernelGGL(k_pack_fdeg<T>, dim3(elem_grid(blk)), dim3(256), 0, ctx->stream, n, 16, nx, nops, X, Xr);
  WL_HIP(hipGetLastError());
  const LockLayout L(K);
  const SmallLayout& Ly = L.Ly;
  const int64_t gs = L.gs;
  WL_TRY(m->small.ensure((size_t)G * gs * sizeof(double)));
  WL_TRY(m->basis.ensure((size_t)(K + 1) * blk * sizeof(T)));
  double* S = m->small.as<double>();
  T* basis = m->basis.as<T>();
  WL_TRY(lockstep_lanczos<T>(m, Xr, G, dgi, K, L, basis, S, m->cmap.as<int32_t>()));
  std::vector<double> hS((size_t)G * gs);
  WL_HIP(hipMemcpyAsync(hS.data(), S, hS.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  const size_t bb = 256;
  std::vector<std::vector<double>> Fq(G);
  int Kr = 1;
  auto eff_dim = [](const std::vector<double>& hB, int Kg, size_t e2) {
    for (int jj = 0; jj + 1 < Kg; ++jj) {  // stop after the first block whose coupling vanished entirely
      double s2 = 0.0;
      for (size_t e = 0; e < e2; ++e) s2 += hB[jj * e2 + e] * hB[jj * e2 + e];
      if (s2 == 0.0) return jj + 1;
    }
    return Kg;
  };
  for (int q = 0; q < nx; ++q) {
    const double* Sq = hS.data() + (size_t)q * gs;
    const int Kg = Kq[q];
    std::vector<double> hA(Sq + Ly.A(0), Sq + Ly.A(0) + Kg * bb), hB(Sq + Ly.B(0), Sq + Ly.B(0) + Kg * bb);
    std::vector<double> hR0(Sq + Ly.R0(), Sq + Ly.R0() + bb);
    for (double v : hA)
      if (!std::isfinite(v)) {
        wl_set_error("block Lanczos produced non-finite coefficients (operator %d)", q);
        return WL_ENUMERIC;
      }
    const int Ke = eff_dim(hB, Kg, bb);
    wl_op op;
    group_op(m, q, &op);
    WL_TRY(lanczos_coefficients(&op, Ke, 16, hA, hB, hR0, Fq[q]));
    apply_deferred(Sq, L, Ke, Fq[q]);  // for the stored blocks W_j = V_j N_j^{-1}
    Kr = std::max(Kr, Ke);
  }
  // the walk-degree group: column q is operator q's own scalar Lanczos process
  std::vector<std::vector<double>> Fd(nops);
  {
    const double* Sd = hS.data() + (size_t)dgi * gs;
    for (int q = 0; q < nops; ++q) {
      const int Kg = Kd[q];
      const size_t d = (size_t)q * 16 + q;
      std::vector<double> hA(Kg), hB(Kg), hR0(1, Sd[Ly.R0() + d]);
      for (int jj = 0; jj < Kg; ++jj) {
        hA[jj] = Sd[Ly.A(jj) + d];
        hB[jj] = Sd[Ly.B(jj) + d];
        if (!std::isfinite(hA[jj])) {
          wl_set_error("Lanczos produced non-finite coefficients (walk degrees of operator %d)", q);
          return WL_ENUMERIC;
        }
      }
      const int Ke = eff_dim(hB, Kg, 1);
      wl_op op;
      group_op(m, q, &op);
      WL_TRY(lanczos_coefficients(&op, Ke, 1, hA, hB, hR0, Fd[q]));
      Kr = std::max(Kr, Ke);
    }
  }
  // C_{q,k}: rows [16 k, 16 (k + 1)) of F_q; the walk-degree group's blocks are diagonal
  // (negated under the Laplacian finish, whose weight there is zero: 0 * 1 - (-V F))
  std::vector<double> F((size_t)G * Kr * bb, 0.0);
  for (int q = 0; q < nx; ++q) std::copy(Fq[q].begin(), Fq[q].end(), F.begin() + (size_t)q * Kr * bb);
  const double* Sd = hS.data() + (size_t)dgi * gs;
  for (int q = 0; q < nops; ++q)
    for (size_t k = 0; k < Fd[q].size(); ++k) {
      const double f = Sd[L.N((int)k) + q * 16 + q] * Fd[q][k];  // stored block: diagonal N_k
      F[((size_t)dgi * Kr + k) * bb + (size_t)q * 16 + q] = laplacian ? -f : f;
    }
  WL_TRY(m->coef.ensure(F.size() * sizeof(double)));
  WL_HIP(hipMemcpyAsync(m->coef.p, F.data(), F.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  T* Wg = nullptr;
  if (laplacian) {
    WL_TRY(m->Wg.ensure((size_t)n * G * sizeof(T)));
    Wg = m->Wg.as<T>();
    hipLaunchKernelGGL(k_wg<T>, dim3(elem_grid(n * G)), dim3(256), 0, ctx->stream, n, nx, nops, m->W.as<T>(), Wg);
    WL_HIP(hipGetLastError());
  }
  T* Yp = m->Ypk.as<T>();
  WL_TRY(launch_gupdate<T>(ctx, n, 16, G, basis, blk, Kr, m->coef.as<double>(), (int64_t)Kr * bb,
                           laplacian ? Xr : nullptr, 0.0, Wg, laplacian ? -1.0 : 1.0, Yp, nullptr, 0));
  hipLaunchKernelGGL(k_unpack_fdeg<T>, dim3(elem_grid(n * (nx * 16 + nops))), dim3(256), 0, ctx->stream, n, 16,
                     nx, nops, Yp, Y, W);
  WL_HIP(hipGetLastError());
  WL_HIP(hipStreamSynchronize(ctx->stream));  // F is host memory of this call
  *done = true;
  return WL_OK;
}

}  // namespace

wl_status multi_groups_create(wl_op* op, int G, wl_multi** out) {
  *out = nullptr;
  WL_CHECK(op->d.method == WL_M_LANCZOS && G >= 1 && G <= 64, WL_EINVAL, "column groups: Lanczos operators only");
  wl_graph* g = op->g;
  auto* m = new wl_multi;
  m->g = g;
  m->nops = G;
  m->prec = op->d.prec;
  m->method = WL_M_LANCZOS;
  m->K.assign(G, op->K);
  m->desc.assign(G, op->d);
  m->Kmax = std::max(op->K, 1);
  std::vector<double> lt((size_t)G * 5, 0.0);
  for (int i = 0; i < G; ++i) lanczos_params(op, &lt[i * 5], &lt[i * 5 + 1], &lt[i * 5 + 2]);
  wl_status s = m->ltab.ensure(lt.size() * 8);
  if (s == WL_OK && hipMemcpy(m->ltab.p, lt.data(), lt.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    wl_set_error("column groups: coefficient upload failed");
    s = WL_EDEVICE;
  }
  // the operator's walk degrees in every group's column (for the Laplacian finish)
  if (s == WL_OK && op->w_valid) {
    const size_t es = m->prec == WL_FP32 ? 4 : 8;
    s = m->W.ensure((size_t)std::max<int64_t>(g->n, 1) * G * es);
    for (int q = 0; q < G && s == WL_OK; ++q)
      s = m->prec == WL_FP32
              ? launch_group_copy<float>(g->ctx, g->n, 1, G, q, op->w.as<float>(), m->W.as<float>(), true)
              : launch_group_copy<double>(g->ctx, g->n, 1, G, q, op->w.as<double>(), m->W.as<double>(), true);
    m->w_valid = s == WL_OK;
  }
  if (s != WL_OK) {
    delete m;
    return s;
  }
  ++g->refs;
  *out = m;
  return WL_OK;
}

void multi_groups_destroy(wl_multi* m) {
  if (!m) return;
  wl_graph* g = m->g;
  (void)hipStreamSynchronize(g->ctx->stream);
  delete m;
  graph_release(g);
}

template <typename T>
wl_status multi_groups_apply(wl_multi* m, const T* X, int b, T* Y, bool laplacian, bool* done) {
  *done = false;
  const int64_t n = m->g->n;
  wl_op op;
  group_op(m, 0, &op);
  const int K = lanczos_steps(&op, n, b);
  if (!grouped_supported(m->prec, b, m->nops) || (int64_t)(K + 1) * b * 2 > n || m->desc[0].reorth > 1 ||
      (laplacian && !m->w_valid))
    return WL_OK;
  WL_TRY(multi_lanczos<T>(m, X, X, b, Y, laplacian ? m->W.as<T>() : nullptr));
  *done = true;
  return WL_OK;
}

template wl_status multi_groups_apply<float>(wl_multi*, const float*, int, float*, bool, bool*);
template wl_status multi_groups_apply<double>(wl_multi*, const double*, int, double*, bool, bool*);

extern "C" {

wl_status wl_multi_create(wl_op* const* ops, int32_t nops, wl_multi** out) {
  WL_CHECK(ops && out, WL_EINVAL, "wl_multi_create: null argument");
  *out = nullptr;
  WL_CHECK(nops >= 1 && nops <= 64, WL_EINVAL, "wl_multi_create: nops must lie in [1, 64]");
  for (int i = 0; i < nops; ++i) WL_CHECK(ops[i], WL_EINVAL, "wl_multi_create: operator %d is null", i);
  wl_graph* g = ops[0]->g;
  const int prec = ops[0]->d.prec;
  const int method = ops[0]->d.method;
  WL_CHECK(method != WL_M_ARNOLDI && method != WL_M_AMG_CG, WL_EUNSUPPORTED,
           "wl_multi_create: Arnoldi and multigrid operators are evaluated alone");
  for (int i = 0; i < nops; ++i) {
    WL_CHECK(ops[i]->g == g, WL_EINVAL, "wl_multi_create: operators must share one graph");
    WL_CHECK(ops[i]->d.prec == prec, WL_EINVAL, "wl_multi_create: operators must share one precision");
    WL_CHECK(ops[i]->d.method == method, WL_EUNSUPPORTED,
             "wl_multi_create: operators must share one evaluation method (operator %d differs)", i);
    if (method == WL_M_RECURRENCE)
      WL_CHECK(ops[i]->K >= 1, WL_EINVAL, "wl_multi_create: operator %d has series degree 0", i);
  }
  DeviceGuard dg(g->ctx->device);
  auto* m = new wl_multi;
  m->g = g;
  m->nops = nops;
  m->prec = prec;
  m->method = method;
  m->K.resize(nops);
  for (int i = 0; i < nops; ++i) {
    m->K[i] = ops[i]->K;
    m->desc.push_back(ops[i]->d);
    m->Kmax = std::max(m->Kmax, ops[i]->K);
  }
  m->Kmax = std::max(m->Kmax, 1);
  wl_status s = WL_OK;
  if (method == WL_M_LANCZOS) {
    // every group's Lanczos matrix a A + (b0 + b1 D)
    std::vector<double> lt((size_t)nops * 5, 0.0);
    for (int i = 0; i < nops; ++i) lanczos_params(ops[i], &lt[i * 5], &lt[i * 5 + 1], &lt[i * 5 + 2]);
    s = m->ltab.ensure(lt.size() * 8);
    if (s == WL_OK && hipMemcpy(m->ltab.p, lt.data(), lt.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      wl_set_error("wl_multi_create: coefficient upload failed");
      s = WL_EDEVICE;
    }
  } else {
    m->fin_at.assign(m->Kmax + 1, 0);
    for (int i = 0; i < nops; ++i) m->fin_at[m->K[i]] = 1;
    // step k (1-based) of operator i: a = s, b0 = s^2 mu^2 (k >= 3), b1 = -s^2 mu (k >= 2),
    // omega_k = c_k / s^k, finish at k = K_i; all zero past K_i (the group is done)
    std::vector<double> tab((size_t)m->Kmax * nops * 5, 0.0);
    for (int i = 0; i < nops; ++i) {
      // scaling s as for one operator: exponential s = min(beta, 1 / lambda_max), weights
      // (beta / s)^k / k!; resolvent s = alpha, weights 1
      const bool ex = ops[i]->d.func == WL_F_EXP;
      const double sp = ex && ops[i]->lam > 0.0 ? std::min(ops[i]->d.param, 1.0 / ops[i]->lam) : ops[i]->d.param;
      const double mu = ops[i]->d.mu, ratio = ex ? ops[i]->d.param / sp : 1.0;
      double omega = 1.0;
      for (int k = 1; k <= m->K[i]; ++k) {
        if (ex) omega *= ratio / k;
        double* c = &tab[((size_t)(k - 1) * nops + i) * 5];
        c[0] = sp;
        c[1] = k >= 3 ? sp * sp * mu * mu : 0.0;
        c[2] = k >= 2 ? -sp * sp * mu : 0.0;
        c[3] = omega;
        c[4] = k == m->K[i] ? 1.0 : 0.0;
      }
    }
    std::vector<double> tab_phi = tab;
    for (size_t e = 4; e < tab_phi.size(); e += 5) tab_phi[e] = 0.0;
    // packed evaluation with walk degrees: entries [0, nops) as above, entries
    // [nops, 2 nops) the same operators without finish (the walk-degree columns)
    std::vector<double> tpk((size_t)m->Kmax * 2 * nops * 5, 0.0), tpk_phi;
    for (int k = 0; k < m->Kmax; ++k)
      for (int i = 0; i < nops; ++i)
        for (int e = 0; e < 5; ++e) {
          const double v = tab[((size_t)k * nops + i) * 5 + e];
          tpk[((size_t)k * 2 * nops + i) * 5 + e] = v;
          tpk[((size_t)k * 2 * nops + nops + i) * 5 + e] = e == 4 ? 0.0 : v;
        }
    tpk_phi = tpk;
    for (size_t e = 4; e < tpk_phi.size(); e += 5) tpk_phi[e] = 0.0;
    s = m->tab.ensure(tab.size() * 8);
    if (s == WL_OK) s = m->tab_phi.ensure(tab.size() * 8);
    if (s == WL_OK) s = m->tab_pk.ensure(tpk.size() * 8);
    if (s == WL_OK) s = m->tab_pk_phi.ensure(tpk.size() * 8);
    if (s == WL_OK && (hipMemcpy(m->tab.p, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                       hipMemcpy(m->tab_phi.p, tab_phi.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                       hipMemcpy(m->tab_pk.p, tpk.data(), tpk.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                       hipMemcpy(m->tab_pk_phi.p, tpk_phi.data(), tpk.size() * 8, hipMemcpyHostToDevice) !=
                           hipSuccess)) {
      wl_set_error("wl_multi_create: coefficient upload failed");
      s = WL_EDEVICE;
    }
  }
  if (s != WL_OK) {
    delete m;
    return s;
  }
  ++g->refs;
  *out = m;
  return WL_OK;
}

wl_status wl_multi_destroy(wl_multi* m) {
  if (!m) return WL_OK;
  wl_graph* g = m->g;
  {
    DeviceGuard dg(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    delete m;
  }
  graph_release(g);
  return WL_OK;
}

wl_status wl_multi_apply(wl_multi* m, const void* d_X, int32_t b, void* d_Y, int32_t laplacian) {
  WL_CHECK(m, WL_EINVAL, "wl_multi_apply: handle is null");
  WL_CHECK(b >= 1 && (int64_t)b * m->nops <= 4096, WL_EINVAL, "wl_multi_apply: need 1 <= b and nops * b <= 4096");
  WL_CHECK(m->g->n == 0 || (d_X && d_Y && d_X != d_Y), WL_EINVAL, "wl_multi_apply: bad blocks");
  DeviceGuard dg(m->g->ctx->device);
  if (m->prec == WL_FP32) {
    if (laplacian) WL_TRY(multi_ensure_w<float>(m));
    return multi_dispatch<float>(m, (const float*)d_X, b, (float*)d_Y, laplacian != 0);
  }
  if (laplacian) WL_TRY(multi_ensure_w<double>(m));
  return multi_dispatch<double>(m, (const double*)d_X, b, (double*)d_Y, laplacian != 0);
}

wl_status wl_multi_apply_fdeg(wl_multi* m, const void* d_X, int32_t b, int32_t nx, void* d_Y, void* d_W,
                              int32_t laplacian) {
  WL_CHECK(m, WL_EINVAL, "wl_multi_apply_fdeg: handle is null");
  WL_CHECK(b >= 1 && (int64_t)b * m->nops <= 4096, WL_EINVAL,
           "wl_multi_apply_fdeg: need 1 <= b and nops * b <= 4096");
  WL_CHECK(nx >= 1 && nx <= m->nops, WL_EINVAL, "wl_multi_apply_fdeg: nx must lie in [1, nops]");
  WL_CHECK(m->g->n == 0 || (d_X && d_Y && d_W && d_X != d_Y && d_X != d_W && d_Y != d_W), WL_EINVAL,
           "wl_multi_apply_fdeg: bad blocks");
  DeviceGuard dg(m->g->ctx->device);
  const int64_t n = m->g->n;
  if (n == 0) return WL_OK;
  bool done = false;
  if (m->prec == WL_FP32) {
    if (laplacian) WL_TRY(multi_ensure_w<float>(m));
    if (m->method == WL_M_RECURRENCE && m->nops <= 16)
      return multi_series_fdeg<float>(m, (const float*)d_X, b, nx, (float*)d_Y, (float*)d_W, laplacian != 0);
    if (m->method == WL_M_LANCZOS)
      WL_TRY(multi_lanczos_fdeg<float>(m, (const float*)d_X, b, nx, (float*)d_Y, (float*)d_W, laplacian != 0,
                                       &done));
    if (done) return WL_OK;
  } else {
    if (laplacian) WL_TRY(multi_ensure_w<double>(m));
    if (m->method == WL_M_RECURRENCE && m->nops <= 16)
      return multi_series_fdeg<double>(m, (const double*)d_X, b, nx, (double*)d_Y, (double*)d_W, laplacian != 0);
  }
  // shapes the packed evaluation does not cover: one call after the other
  WL_CHECK(nx == m->nops, WL_EUNSUPPORTED,
           "wl_multi_apply_fdeg: nx < nops needs the packed evaluation (series, or FP32 Lanczos with b = 16)");
  if (m->prec == WL_FP32)
    WL_TRY(multi_dispatch<float>(m, (const float*)d_X, b, (float*)d_Y, laplacian != 0));
  else
    WL_TRY(multi_dispatch<double>(m, (const double*)d_X, b, (double*)d_Y, laplacian != 0));
  return wl_multi_fdeg(m, d_W);
}

wl_status wl_multi_fdeg(wl_multi* m, void* d_W) {
  WL_CHECK(m, WL_EINVAL, "wl_multi_fdeg: handle is null");
  WL_CHECK(m->g->n == 0 || d_W, WL_EINVAL, "wl_multi_fdeg: output is null");
  DeviceGuard dg(m->g->ctx->device);
  const int64_t n = m->g->n;
  if (n == 0) return WL_OK;
  const size_t es = m->prec == WL_FP32 ? 4 : 8;
  WL_TRY(m->ones.ensure((size_t)n * es));
  if (m->prec == WL_FP32) {
    WL_TRY(launch_fill<float>(m->g->ctx, n, 1.0f, m->ones.as<float>()));
    return multi_dispatch<float>(m, m->ones.as<float>(), 1, (float*)d_W, false);
  }
  WL_TRY(launch_fill<double>(m->g->ctx, n, 1.0, m->ones.as<double>()));
  return multi_dispatch<double>(m, m->ones.as<double>(), 1, (double*)d_W, false);
}

}  // extern "C"
