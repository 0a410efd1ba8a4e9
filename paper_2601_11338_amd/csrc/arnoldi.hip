// Exponential weights through the linearisation, by block Arnoldi (Prop.
// "whe-we-converge": phi X = X + [I O] f_1(Z) [q_1 X; q_2 X], f_1(x) = beta phi_1(beta x)
// for c_k = beta^k / k!, Z = [[O, I], [mu (mu I - D), A]] of eq. Zdef).
//
// When beta rho(Z) is large the truncated series needs a degree of order e beta rho(Z);
// a Krylov space of Z reaches the same accuracy with fewer products because it adapts
// to the spectrum.  Z is not symmetric, so the basis is built by block Arnoldi with
// full classical Gram-Schmidt orthogonalisation (repeated where it cancelled).  A
// block of 2n rows is stored as one (2n) x b row-major array, its top half (rows
// 0..n-1) followed by its
// bottom half, so the Gram and update kernels treat it as a tall block unchanged, and
//   Z V = [V_bot; A V_bot + (mu^2 - mu d) (.) V_top]
// is one copy and one sparse product whose epilogue adds the diagonal term.  The
// projected matrix H_K (block upper Hessenberg) gives
//   phi X ~= X + top(V_K F),  F = beta phi_1(beta H_K) E_1 R_0,
// with phi_1 of the small dense matrix by Pade scaling and squaring on the host.
#include <algorithm>
#include <cmath>
#include <vector>

#include "wl_internal.h"

namespace {

template <typename T>
struct ArnWork {
  wl_ctx* ctx;
  int64_t rows;  // 2n
  int b;
  T* basis;
  DevBuf* small;  // device doubles
};

template <typename T>
wl_status arn_gram(ArnWork<T>& W, const T* X, int nblk, const T* Y, std::vector<double>& G) {
  const int b = W.b;
  WL_TRY(launch_gram<T>(W.ctx, W.rows, X, b, W.rows * b, nblk, Y, b, W.small->template as<double>()));
  G.resize((size_t)nblk * b * b);
  WL_HIP(hipMemcpyAsync(G.data(), W.small->p, G.size() * 8, hipMemcpyDeviceToHost, W.ctx->stream));
  WL_HIP(hipStreamSynchronize(W.ctx->stream));
  return WL_OK;
}

// Out = Yin - X C, or Out = X_0 C without Yin (C host, nblk*b x b)
template <typename T>
wl_status arn_update(ArnWork<T>& W, const T* X, int nblk, const std::vector<double>& C, const T* Yin, T* Out) {
  const int b = W.b;
  WL_HIP(hipMemcpyAsync(W.small->p, C.data(), C.size() * 8, hipMemcpyHostToDevice, W.ctx->stream));
  if (Yin)
    WL_TRY(launch_update<T>(W.ctx, W.rows, X, b, W.rows * b, nblk, W.small->template as<double>(), Yin, 1.0, nullptr,
                            -1.0, Out, b, nullptr));
  else
    WL_TRY(launch_update<T>(W.ctx, W.rows, X, b, W.rows * b, nblk, W.small->template as<double>(), nullptr, 0.0,
                            nullptr, 1.0, Out, b, nullptr));
  WL_HIP(hipStreamSynchronize(W.ctx->stream));  // C is host memory of the caller
  return WL_OK;
}

// Orthogonalise Wb against basis blocks [0, nb) (classical Gram-Schmidt, a second pass
// when the first cancelled most of a column) and store it as block nb by CholQR2 with
// deflation.  H (host, (nb + 1) b x b) receives
// the coefficients: Wb = sum_i V_i H_i + V_nb H_nb.
template <typename T>
wl_status arn_append(ArnWork<T>& W, int nb, T* Wb, std::vector<double>& H) {
  const int b = W.b;
  std::vector<double> G, R1, R1i, R2, R2i, C;
  std::vector<char> k1, k2;
  H.assign((size_t)(nb + 1) * b * b, 0.0);
  WL_TRY(arn_gram<T>(W, Wb, 1, Wb, G));
  double ref = 0.0;
  for (int c = 0; c < b; ++c) ref = std::max(ref, G[(size_t)c * b + c]);
  if (nb > 0) {
    // a second classical Gram-Schmidt pass only when the first removed most of some
    // column's norm (cancellation; the "twice is enough" criterion)
    const std::vector<double> G0 = G;
    for (int pass = 0; pass < 2; ++pass) {
      WL_TRY(arn_gram<T>(W, W.basis, nb, Wb, C));
      WL_TRY(arn_update<T>(W, W.basis, nb, C, Wb, Wb));
      for (size_t e = 0; e < C.size(); ++e) H[e] += C[e];
      WL_TRY(arn_gram<T>(W, Wb, 1, Wb, G));
      bool kept = true;
      for (int c = 0; c < b; ++c)
        if (G[(size_t)c * b + c] < 0.5 * G0[(size_t)c * b + c]) kept = false;
      if (kept) break;
    }
  }
  T* slot = W.basis + (size_t)nb * W.rows * b;
  const double tol = defl_tol<T>();
  host_chol_deflate(b, G, tol, ref, R1, R1i, k1);
  WL_TRY(arn_update<T>(W, Wb, 1, R1i, nullptr, slot));
  WL_TRY(arn_gram<T>(W, slot, 1, slot, G));
  host_chol_deflate(b, G, tol, 1.0, R2, R2i, k2);
  const double ptol = post_tol<T>();
  for (int c = 0; c < b; ++c) {
    const double d = std::fabs(R2[(size_t)c * b + c] * R1[(size_t)c * b + c]);
    if (!(d > ptol * std::sqrt(ref))) {
      for (int i = 0; i < b; ++i) R2i[(size_t)i * b + c] = 0.0;
      for (int j = 0; j < b; ++j) R2[(size_t)c * b + j] = 0.0;  // the dropped component has no coupling
    }
  }
  WL_TRY(arn_update<T>(W, slot, 1, R2i, nullptr, slot));
  double* Hn = H.data() + (size_t)nb * b * b;
  for (int i = 0; i < b; ++i)
    for (int j = 0; j < b; ++j) {
      double s = 0.0;
      for (int k = 0; k < b; ++k) s += R2[(size_t)i * b + k] * R1[(size_t)k * b + j];
      Hn[(size_t)i * b + j] = s;
    }
  return WL_OK;
}

}  // namespace

template <typename T>
wl_status phi_arnoldi(wl_op* op, const T* X, T* Y, int b, const T* wv, const T* Xw) {
  wl_graph* g = op->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  const double mu = op->d.mu, beta = op->d.param;
  // the Krylov space of Z has dimension <= 2n and grows by at least one per step until
  // it is invariant (a start block of lower rank grows by its rank, not by b); the loop
  // stops at the first vanished coupling
  const int K = (int)std::max<int64_t>(1, std::min<int64_t>(op->K, 2 * n));
  const int64_t blk2 = 2 * n * b;
  WL_TRY(op->basis.ensure((size_t)(K + 1) * blk2 * sizeof(T)));
  WL_TRY(op->wbuf.ensure((size_t)blk2 * sizeof(T)));
  WL_TRY(op->small.ensure((size_t)(K + 1) * b * b * sizeof(double)));
  ArnWork<T> W{ctx, 2 * n, b, op->basis.as<T>(), &op->small};
  T* Wb = op->wbuf.as<T>();
  const SpmmShape sh = shape_for(g, prec_of<T>(), b);
  // start block [q_1 X; q_2 X]: top = A X, bottom = A (A X) - mu D X
  {
    EpiArgs<T> ep;
    WL_TRY(launch_spmm<T>(g, X, Wb, b, ep, sh));
    EpiArgs<T> e2;
    e2.Z = X;
    e2.b1 = -mu;
    WL_TRY(launch_spmm<T>(g, Wb, Wb + n * b, b, e2, sh));
  }
  std::vector<double> Hc, R0;
  WL_TRY(arn_append<T>(W, 0, Wb, Hc));
  R0.assign(Hc.begin(), Hc.begin() + (size_t)b * b);
  // H (row-major, (K+1) b x K b): column block j from step j
  const int m = K * b;
  std::vector<double> H((size_t)(K + 1) * b * m, 0.0);
  int Ke = K;
  for (int j = 0; j < K; ++j) {
    T* Vj = W.basis + (size_t)j * blk2;
    // W = Z V_j: top = bottom(V_j), bottom = A bottom(V_j) + (mu^2 - mu d) top(V_j)
    WL_HIP(hipMemcpyAsync(Wb, Vj + n * b, (size_t)n * b * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    EpiArgs<T> ep;
    ep.Z = Vj;
    ep.b0 = mu * mu;
    ep.b1 = -mu;
    ep.kclass = b >= 4 ? WL_KC_RECURRENCE : WL_KC_OTHER_SPMM;
    WL_TRY(launch_spmm<T>(g, Vj + n * b, Wb + n * b, b, ep, sh));
    WL_TRY(arn_append<T>(W, j + 1, Wb, Hc));
    for (int i = 0; i < (j + 2) * b; ++i)
      for (int c = 0; c < b; ++c) H[(size_t)i * m + j * b + c] = Hc[(size_t)i * b + c];
    // a coupling that vanished entirely: the space is invariant, stop here
    double s2 = 0.0;
    for (int e = 0; e < b * b; ++e) s2 += Hc[(size_t)(j + 1) * b * b + e] * Hc[(size_t)(j + 1) * b * b + e];
    if (s2 == 0.0) {
      Ke = j + 1;
      break;
    }
  }
  for (double v : H)
    if (!std::isfinite(v)) {
      wl_set_error("block Arnoldi produced non-finite coefficients");
      return WL_ENUMERIC;
    }
  // F = beta phi_1(beta H_Ke) E_1 R0 on the square part
  const int me = Ke * b;
  std::vector<double> Mh((size_t)me * me), B((size_t)me * b, 0.0), F((size_t)me * b);
  for (int i = 0; i < me; ++i)
    for (int c = 0; c < me; ++c) Mh[(size_t)i * me + c] = beta * H[(size_t)i * m + c];
  for (int i = 0; i < b; ++i)
    for (int c = 0; c < b; ++c) B[(size_t)i * b + c] = R0[(size_t)i * b + c];
  if (dense_phi1_times(me, Mh.data(), b, B.data(), F.data())) {
    wl_set_error("phi_1 of the projected Arnoldi matrix failed");
    return WL_ENUMERIC;
  }
  for (double& v : F) v *= beta;
  // phi X = X + top(sum_j V_j F_j): the top halves are the first n rows of each block
  WL_TRY(op->coef.ensure(F.size() * sizeof(double)));
  WL_HIP(hipMemcpyAsync(op->coef.p, F.data(), F.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  WL_TRY(launch_update<T>(ctx, n, W.basis, b, blk2, Ke, op->coef.as<double>(), X, 1.0, nullptr, 1.0, Y, b,
                          nullptr));
  if (wv) WL_TRY(launch_axpby_rows<T>(ctx, n, b, wv, Xw, -1.0, Y, Y));  // L X = w (.) X - phi X
  WL_HIP(hipStreamSynchronize(ctx->stream));  // F is host memory of this call
  return WL_OK;
}

template wl_status phi_arnoldi<float>(wl_op*, const float*, float*, int, const float*, const float*);
template wl_status phi_arnoldi<double>(wl_op*, const double*, double*, int, const double*, const double*);
