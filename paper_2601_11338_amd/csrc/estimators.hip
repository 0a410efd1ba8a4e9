// Diagonal and trace estimators (Sec. 4.4, Alg. 1).
//
// All estimators consume the probe block Omega (n x M) and Y = F Omega.
//  * Hutchinson / BKS / control variate: one row kernel.
//  * Leave-one-out Nystrom (the exchangeable XNysTrace idea of Alg. 1).  With
//    H = Omega^T Y and G = Y^T Y (M x M, double, from the device Gram kernel) and
//    P_j the pseudo-inverse of the symmetrised H without row/column j (embedded
//    back into M x M with zeros), the per-probe estimates of
//      F_(j) = Y_{-j} H_{-j,-j}^+ Y_{-j}^T,
//      t_j   = tr F_(j) + omega_j^T (F - F_(j)) omega_j
//    reduce to small matrices:
//      tr F_(j)              = tr(P_j G),
//      omega_j^T F omega_j   = H_jj,
//      omega_j^T F_(j) omega_j = h_j^T P_j h_j,  h_j = row j of H (Y^T omega_j),
//    and the averaged diagonal estimate at row r to
//      d_r = ( y_r Q1 y_r^T + sum_j Omega_rj Y_rj - y_r Q2 omega_r^T ) / M,
//      Q1 = sum_j P_j,  column j of Q2 = P_j h_j,
//    so the device work is two Gram products and one row pass.
#include <algorithm>
#include <cmath>
#include <vector>

#include "wl_internal.h"

namespace {

constexpr int DIAG_CHUNK = 64;  // probes per block in wl_diag_est

// Surrogate estimator finish: diag G_i = 1 + c2m d_i + c3 tri2_i (c2m = c_2 (1 - mu),
// tri2_i = (A^3)_ii); dot_i = sum_j Omega_ij ((phi - G) Omega)_ij, sq_i = sum_j Omega_ij^2;
// d_i = g_i + (dot_i + (diag G_i - g_i) sq_i) / M with g = cv, or diag G without one.
template <typename T>
__global__ void k_surrogate_finish(int64_t n, int M, const double* __restrict__ dot, const double* __restrict__ sq,
                                   const int32_t* __restrict__ rowptr, const unsigned long long* __restrict__ tri2,
                                   double c2m, double c3, const T* __restrict__ cv, T* __restrict__ diag) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const double gd = 1.0 + c2m * (double)(rowptr[r + 1] - rowptr[r]) + c3 * (double)tri2[r];
    const double gh = cv ? (double)cv[r] : gd;
    diag[r] = (T)(gh + (dot[r] + (gd - gh) * sq[r]) / M);
  }
}

// Gram of two n x M row-major blocks (M <= 64: one launch of the Gram kernel).
template <typename T>
wl_status gram_full(wl_ctx* ctx, int64_t n, int M, const T* X, const T* Y, std::vector<double>& out) {
  out.assign((size_t)M * M, 0.0);
  if (M <= 64) {
    DevBuf d;
    WL_TRY(d.ensure((size_t)M * M * 8));
    WL_TRY(launch_gram<T>(ctx, n, X, M, 0, 1, Y, M, d.as<double>()));
    WL_HIP(hipMemcpyAsync(out.data(), d.p, (size_t)M * M * 8, hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    return WL_OK;
  }
  wl_set_error("estimators with more than 64 probes per block are not supported by this build");
  return WL_EUNSUPPORTED;
}

// pseudo-inverse of the symmetric part of the (M-1) x (M-1) matrix H without j,
// embedded into M x M
int pinv_drop(int M, const std::vector<double>& H, int j, double rcond, std::vector<double>& P) {
  const int m = M - 1;
  std::vector<double> S((size_t)m * m), lam(m), U((size_t)m * m);
  for (int a = 0, ia = 0; a < M; ++a) {
    if (a == j) continue;
    for (int c = 0, ic = 0; c < M; ++c) {
      if (c == j) continue;
      S[(size_t)ia * m + ic] = 0.5 * (H[(size_t)a * M + c] + H[(size_t)c * M + a]);
      ++ic;
    }
    ++ia;
  }
  if (dense_syev(m, S.data(), lam.data(), U.data())) return 1;
  double lmax = 0.0;
  for (double v : lam) lmax = std::max(lmax, v);
  P.assign((size_t)M * M, 0.0);
  std::vector<int> map;
  for (int a = 0; a < M; ++a)
    if (a != j) map.push_back(a);
  for (int k = 0; k < m; ++k) {
    if (!(lam[k] > rcond * lmax)) continue;
    const double inv = 1.0 / lam[k];
    for (int a = 0; a < m; ++a) {
      const double ua = U[(size_t)a * m + k] * inv;
      if (ua == 0.0) continue;
      for (int c = 0; c < m; ++c) P[(size_t)map[a] * M + map[c]] += ua * U[(size_t)c * m + k];
    }
  }
  return 0;
}

template <typename T>
wl_status estimate_impl(wl_ctx* ctx, int estimator, int64_t n, int M, const T* Om, const T* Y, const T* cv,
                        double rcond, T* diag, double* trace, double* trace_err) {
  std::vector<double> H;
  WL_TRY(gram_full<T>(ctx, n, M, Om, Y, H));
  if (estimator != WL_EST_XNYS) {
    const int mode = cv ? 2 : (estimator == WL_EST_BKS ? 1 : 0);
    if (diag) WL_TRY(launch_cv_finish<T>(ctx, n, M, Om, Y, cv, mode, diag));
    double mean = 0.0;
    for (int j = 0; j < M; ++j) mean += H[(size_t)j * M + j];
    mean /= M;
    double var = 0.0;
    for (int j = 0; j < M; ++j) var += (H[(size_t)j * M + j] - mean) * (H[(size_t)j * M + j] - mean);
    if (trace) *trace = mean;
    if (trace_err) *trace_err = M > 1 ? std::sqrt(var / (M - 1)) / std::sqrt((double)M) : INFINITY;
    return WL_OK;
  }
  WL_CHECK(M >= 2, WL_EINVAL, "wl_estimate: the Nystrom estimator needs M >= 2");
  std::vector<double> G;
  WL_TRY(gram_full<T>(ctx, n, M, Y, Y, G));
  std::vector<double> Q1((size_t)M * M, 0.0), Q2((size_t)M * M, 0.0), P, tj(M);
  for (int j = 0; j < M; ++j) {
    if (pinv_drop(M, H, j, rcond, P)) {
      wl_set_error("wl_estimate: eigendecomposition of the Nystrom core failed");
      return WL_ENOCONV;
    }
    double trPG = 0.0, hPh = 0.0;
    std::vector<double> Ph(M, 0.0);
    for (int a = 0; a < M; ++a)
      for (int c = 0; c < M; ++c) {
        const double p = P[(size_t)a * M + c];
        trPG += p * G[(size_t)c * M + a];
        Ph[a] += p * H[(size_t)j * M + c];
      }
    for (int a = 0; a < M; ++a) hPh += H[(size_t)j * M + a] * Ph[a];
    tj[j] = trPG + H[(size_t)j * M + j] - hPh;
    for (int e = 0; e < M * M; ++e) Q1[e] += P[e];
    for (int a = 0; a < M; ++a) Q2[(size_t)a * M + j] = Ph[a];
  }
  double mean = 0.0;
  for (double v : tj) mean += v;
  mean /= M;
  double var = 0.0;
  for (double v : tj) var += (v - mean) * (v - mean);
  if (trace) *trace = mean;
  if (trace_err) *trace_err = std::sqrt(var / (M - 1)) / std::sqrt((double)M);
  if (diag) {
    DevBuf dq;
    WL_TRY(dq.ensure((size_t)2 * M * M * 8));
    WL_HIP(hipMemcpyAsync(dq.p, Q1.data(), (size_t)M * M * 8, hipMemcpyHostToDevice, ctx->stream));
    WL_HIP(hipMemcpyAsync(dq.as<double>() + (size_t)M * M, Q2.data(), (size_t)M * M * 8, hipMemcpyHostToDevice,
                          ctx->stream));
    WL_TRY(launch_nys_diag<T>(ctx, n, M, Om, Y, dq.as<double>(), dq.as<double>() + (size_t)M * M, diag));
    WL_HIP(hipStreamSynchronize(ctx->stream));
  }
  return WL_OK;
}

}  // namespace

int xnys_trace_host(int M, const std::vector<double>& H, const std::vector<double>& G, double rcond, double* trace,
                    double* trace_err) {
  // t_j = tr(Hp_j G) + H_jj - h_j^T Hp_j h_j, Hp_j the pseudo-inverse of the core
  // without probe j, h_j = row j of H: the leave-one-out estimate written with the
  // M x M Grams alone (F_(j) = Y_{-j} Hp_j Y_{-j}^T, never formed)
  if (M < 2) return -1;
  std::vector<double> P, tj(M);
  for (int j = 0; j < M; ++j) {
    if (pinv_drop(M, H, j, rcond, P)) return -1;
    double trPG = 0.0, hPh = 0.0;
    for (int a = 0; a < M; ++a) {
      double ph = 0.0;
      for (int c = 0; c < M; ++c) {
        trPG += P[(size_t)a * M + c] * G[(size_t)c * M + a];
        ph += P[(size_t)a * M + c] * H[(size_t)j * M + c];
      }
      hPh += H[(size_t)j * M + a] * ph;
    }
    tj[j] = trPG + H[(size_t)j * M + j] - hPh;
  }
  double mean = 0.0;
  for (double v : tj) mean += v;
  mean /= M;
  double var = 0.0;
  for (double v : tj) var += (v - mean) * (v - mean);
  *trace = mean;
  *trace_err = std::sqrt(var / (M - 1)) / std::sqrt((double)M);
  return 0;
}

extern "C" {

wl_status wl_estimate(wl_ctx* ctx, int32_t prec, int32_t estimator, int64_t n, int32_t M, const void* d_Omega,
                      const void* d_Y, const void* d_cv, double rcond, void* d_diag, double* trace,
                      double* trace_err) {
  WL_CHECK(ctx, WL_EINVAL, "wl_estimate: ctx is null");
  WL_CHECK(prec == WL_FP32 || prec == WL_FP64, WL_EINVAL, "wl_estimate: bad prec");
  WL_CHECK(estimator >= WL_EST_HUTCHINSON && estimator <= WL_EST_XNYS, WL_EINVAL, "wl_estimate: bad estimator");
  WL_CHECK(n >= 1 && M >= 1, WL_EINVAL, "wl_estimate: need n >= 1 and M >= 1");
  WL_CHECK(d_Omega && d_Y, WL_EINVAL, "wl_estimate: null probe or product block");
  WL_CHECK(!(d_cv && estimator != WL_EST_HUTCHINSON), WL_EINVAL,
           "wl_estimate: the control variate applies to the Hutchinson estimator");
  WL_CHECK(rcond >= 0 && std::isfinite(rcond), WL_EINVAL, "wl_estimate: bad rcond");
  int dev = ctx->device;
  (void)hipSetDevice(dev);
  if (prec == WL_FP32)
    return estimate_impl<float>(ctx, estimator, n, M, (const float*)d_Omega, (const float*)d_Y,
                                (const float*)d_cv, rcond, (float*)d_diag, trace, trace_err);
  return estimate_impl<double>(ctx, estimator, n, M, (const double*)d_Omega, (const double*)d_Y,
                               (const double*)d_cv, rcond, (double*)d_diag, trace, trace_err);
}

wl_status wl_diag_est(wl_op* op, int32_t target, double t, int32_t M, uint64_t seed, int32_t law,
                      int32_t estimator, const void* d_cv, int32_t outer_dim, void* d_diag, double* trace,
                      double* trace_err) {
  WL_CHECK(op, WL_EINVAL, "wl_diag_est: op is null");
  WL_CHECK(target == 0 || target == 1, WL_EINVAL, "wl_diag_est: target must be 0 (phi) or 1 (exp(-tL))");
  WL_CHECK(M >= 1 && M <= 4096, WL_EINVAL, "wl_diag_est: M must lie in [1, 4096]");
  WL_CHECK(estimator >= WL_EST_HUTCHINSON && estimator <= WL_EST_SURROGATE, WL_EINVAL,
           "wl_diag_est: bad estimator");
  WL_CHECK(M <= DIAG_CHUNK || estimator != WL_EST_XNYS, WL_EINVAL,
           "wl_diag_est: the Nystrom estimator takes at most %d probes", DIAG_CHUNK);
  WL_CHECK(!(d_cv && estimator != WL_EST_HUTCHINSON && estimator != WL_EST_SURROGATE), WL_EINVAL,
           "wl_diag_est: the control variate applies to the Hutchinson and surrogate estimators");
  WL_CHECK(!(estimator == WL_EST_SURROGATE && target != 0), WL_EINVAL,
           "wl_diag_est: the surrogate estimator applies to phi (target 0)");
  WL_CHECK(law == WL_PROBE_GAUSS || law == WL_PROBE_RADEMACHER, WL_EINVAL, "wl_diag_est: bad probe law");
  WL_CHECK(std::isfinite(t) && t >= 0, WL_EINVAL, "wl_diag_est: bad t");
  wl_graph* g = op->g;
  const int64_t n = g->n;
  WL_CHECK(n >= 1, WL_EINVAL, "wl_diag_est: empty graph");
  WL_CHECK(d_diag, WL_EINVAL, "wl_diag_est: d_diag is null");
  (void)hipSetDevice(g->ctx->device);
  wl_ctx* ctx = g->ctx;
  const size_t es = op->d.prec == WL_FP32 ? 4 : 8;
  const int mc = M < DIAG_CHUNK ? M : DIAG_CHUNK;
  DevBuf Om, Y;
  WL_TRY(Om.ensure((size_t)n * mc * es));
  WL_TRY(Y.ensure((size_t)n * mc * es));
  auto product = [&](int m) -> wl_status {
    if (target == 0) return wl_apply_phi(op, Om.p, Y.p, m);
    void* outs[1] = {Y.p};
    return wl_expv(op, Om.p, m, &t, 1, outs, outer_dim, nullptr);
  };
  const bool sur = estimator == WL_EST_SURROGATE;
  if (M <= DIAG_CHUNK && !sur) {
    WL_TRY(wl_probes(ctx, op->d.prec, law, seed, 0, n, M, Om.p));
    WL_TRY(product(M));
    WL_TRY(wl_estimate(ctx, op->d.prec, estimator, n, M, Om.p, Y.p, d_cv, 1e-10, d_diag, trace, trace_err));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    return WL_OK;
  }
  // more probes than one block: blocks of DIAG_CHUNK columns (block c from Philox
  // stream c), row sums accumulated on the device, per-probe traces from the Gram
  // diagonal of each block
  // (the surrogate estimator takes this path for any M: Y becomes (phi - G) Omega)
  DevBuf sums, H, Z;
  const unsigned long long* tri = nullptr;
  WL_TRY(sums.ensure((size_t)2 * n * 8));
  WL_TRY(H.ensure((size_t)DIAG_CHUNK * DIAG_CHUNK * 8));
  wl_op gop;  // the degree-3 truncation of the same series (borrows the graph)
  double c2m = 0.0, c3 = 0.0, trG = 0.0;
  if (sur) {
    gop.g = g;
    gop.d = op->d;
    gop.d.method = WL_M_RECURRENCE;
    gop.K = std::min(3, op->K);  // linear weights: the series stops after one step
    const double p = op->d.param;
    // weights of G's terms that exist (the series may stop before degree 3: linear
    // weights after one step)
    const bool ex = op->d.func == WL_F_EXP, lin = op->d.func == WL_F_LINEAR;
    c2m = lin || gop.K < 2 ? 0.0 : (ex ? p * p / 2.0 : p * p) * (1.0 - op->d.mu);
    c3 = lin || gop.K < 3 ? 0.0 : (ex ? p * p * p / 6.0 : p * p * p);
    WL_TRY(Z.ensure((size_t)n * mc * es));
    WL_TRY(graph_tri2(g, &tri));
    std::vector<unsigned long long> ht(n);
    WL_HIP(hipMemcpyAsync(ht.data(), tri, (size_t)n * 8, hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    double st = 0.0;
    for (unsigned long long v : ht) st += (double)v;
    trG = (double)n + c2m * (double)g->nnz + c3 * st;
  }
  std::vector<double> tj;
  std::vector<double> hH((size_t)DIAG_CHUNK * DIAG_CHUNK);
  const int nchunks = (M + DIAG_CHUNK - 1) / DIAG_CHUNK;
  for (int c = 0; c < nchunks; ++c) {
    const int m = std::min(DIAG_CHUNK, M - c * DIAG_CHUNK);
    WL_TRY(wl_probes(ctx, op->d.prec, law, seed, (uint32_t)c, n, m, Om.p));
    WL_TRY(product(m));
    if (sur) {  // Y <- Y - G Omega
      if (op->d.prec == WL_FP32) {
        WL_TRY(phi_apply_impl<float>(&gop, Om.as<float>(), Z.as<float>(), m, nullptr, nullptr));
        WL_TRY(launch_axpby_rows<float>(ctx, n, m, nullptr, Y.as<float>(), -1.0, Z.as<float>(), Y.as<float>()));
      } else {
        WL_TRY(phi_apply_impl<double>(&gop, Om.as<double>(), Z.as<double>(), m, nullptr, nullptr));
        WL_TRY(launch_axpby_rows<double>(ctx, n, m, nullptr, Y.as<double>(), -1.0, Z.as<double>(),
                                         Y.as<double>()));
      }
    }
    if (op->d.prec == WL_FP32) {
      WL_TRY(launch_rowdot<float>(ctx, n, m, Om.as<float>(), Y.as<float>(), sums.as<double>(),
                                  sums.as<double>() + n, c > 0));
      WL_TRY(launch_gram<float>(ctx, n, Om.as<float>(), m, 0, 1, Y.as<float>(), m, H.as<double>()));
    } else {
      WL_TRY(launch_rowdot<double>(ctx, n, m, Om.as<double>(), Y.as<double>(), sums.as<double>(),
                                   sums.as<double>() + n, c > 0));
      WL_TRY(launch_gram<double>(ctx, n, Om.as<double>(), m, 0, 1, Y.as<double>(), m, H.as<double>()));
    }
    WL_HIP(hipMemcpyAsync(hH.data(), H.p, (size_t)m * m * 8, hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    for (int j = 0; j < m; ++j) tj.push_back(hH[(size_t)j * m + j]);
  }
  const int mode = d_cv ? 2 : (estimator == WL_EST_BKS ? 1 : 0);
  const int gb = (int)std::min<int64_t>(8192, (n + 255) / 256);
  if (sur && op->d.prec == WL_FP32) {
    hipLaunchKernelGGL(k_surrogate_finish<float>, dim3(gb), dim3(256), 0, ctx->stream, n, M, sums.as<double>(),
                       sums.as<double>() + n, g->rowptr, tri, c2m, c3,
                       (const float*)d_cv, (float*)d_diag);
    WL_HIP(hipGetLastError());
  } else if (sur) {
    hipLaunchKernelGGL(k_surrogate_finish<double>, dim3(gb), dim3(256), 0, ctx->stream, n, M, sums.as<double>(),
                       sums.as<double>() + n, g->rowptr, tri, c2m, c3,
                       (const double*)d_cv, (double*)d_diag);
    WL_HIP(hipGetLastError());
  } else if (op->d.prec == WL_FP32) {
    WL_TRY(launch_sums_finish<float>(ctx, n, M, sums.as<double>(), sums.as<double>() + n, (const float*)d_cv, mode,
                                     (float*)d_diag));
  } else {
    WL_TRY(launch_sums_finish<double>(ctx, n, M, sums.as<double>(), sums.as<double>() + n, (const double*)d_cv,
                                      mode, (double*)d_diag));
  }
  double mean = 0.0, var = 0.0;
  for (double v : tj) mean += v;
  mean /= M;
  for (double v : tj) var += (v - mean) * (v - mean);
  if (trace) *trace = mean + trG;
  if (trace_err) *trace_err = std::sqrt(var / (M - 1)) / std::sqrt((double)M);
  WL_HIP(hipStreamSynchronize(ctx->stream));
  return WL_OK;
}

}  // extern "C"
