// Several walk operators of one graph evaluated together.
//
// Every operator's truncated series (eq. qrec: P_1 = s A X, P_2 = s A P_1 - s^2 mu D X,
// P_k = s A P_{k-1} + s^2 mu (mu - D) P_{k-2}, S = sum_k omega_k P_k) runs on its own
// column group of one wide block n x (nops b): operator g owns columns [g b, (g+1) b).
// One sparse product per step serves all of them, with every group's coefficients of
// that step read from a small table.  Rows of b = 16 FP32 values are half of a
// 128-byte cache line; four operators side by side gather two full lines per
// neighbour, so the same lines serve four times the work.
#include <algorithm>
#include <cmath>
#include <vector>

#include "wl_internal.h"

struct wl_multi {
  wl_graph* g = nullptr;
  int nops = 0;
  int prec = WL_FP32;
  int Kmax = 0;
  std::vector<int> K;
  std::vector<char> fin_at;  // fin_at[k]: some operator's series ends at step k
  DevBuf tab;      // [Kmax][nops][5] {a, b0, b1, omega, finish}
  DevBuf tab_phi;  // the same without the finish flags
  DevBuf W;        // walk degrees, n x nops
  bool w_valid = false;
  DevBuf Xrep, A, B, ones;
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

template <typename T>
wl_status multi_ensure_w(wl_multi* m) {
  if (m->w_valid) return WL_OK;
  wl_graph* g = m->g;
  const int64_t n = g->n;
  WL_TRY(m->W.ensure((size_t)std::max<int64_t>(n, 1) * m->nops * sizeof(T)));
  WL_TRY(m->ones.ensure((size_t)std::max<int64_t>(n, 1) * sizeof(T)));
  WL_TRY(launch_fill<T>(g->ctx, n, T(1), m->ones.as<T>()));
  WL_TRY(multi_apply<T>(m, m->ones.as<T>(), 1, m->W.as<T>(), false));
  WL_HIP(hipStreamSynchronize(g->ctx->stream));
  m->w_valid = true;
  return WL_OK;
}

}  // namespace

extern "C" {

wl_status wl_multi_create(wl_op* const* ops, int32_t nops, wl_multi** out) {
  WL_CHECK(ops && out, WL_EINVAL, "wl_multi_create: null argument");
  *out = nullptr;
  WL_CHECK(nops >= 1 && nops <= 64, WL_EINVAL, "wl_multi_create: nops must lie in [1, 64]");
  for (int i = 0; i < nops; ++i) WL_CHECK(ops[i], WL_EINVAL, "wl_multi_create: operator %d is null", i);
  wl_graph* g = ops[0]->g;
  const int prec = ops[0]->d.prec;
  for (int i = 0; i < nops; ++i) {
    WL_CHECK(ops[i]->g == g, WL_EINVAL, "wl_multi_create: operators must share one graph");
    WL_CHECK(ops[i]->d.prec == prec, WL_EINVAL, "wl_multi_create: operators must share one precision");
    WL_CHECK(ops[i]->d.method == WL_M_RECURRENCE, WL_EUNSUPPORTED,
             "wl_multi_create: operator %d is evaluated by Lanczos; only truncated-series operators combine", i);
    WL_CHECK(ops[i]->K >= 1, WL_EINVAL, "wl_multi_create: operator %d has series degree 0", i);
  }
  DeviceGuard dg(g->ctx->device);
  auto* m = new wl_multi;
  m->g = g;
  m->nops = nops;
  m->prec = prec;
  m->K.resize(nops);
  for (int i = 0; i < nops; ++i) {
    m->K[i] = ops[i]->K;
    m->Kmax = std::max(m->Kmax, ops[i]->K);
  }
  m->Kmax = std::max(m->Kmax, 1);
  m->fin_at.assign(m->Kmax + 1, 0);
  for (int i = 0; i < nops; ++i) m->fin_at[m->K[i]] = 1;
  // step k (1-based) of operator i: a = s, b0 = s^2 mu^2 (k >= 3), b1 = -s^2 mu (k >= 2),
  // omega_k = c_k / s^k, finish at k = K_i; all zero past K_i (the group is done)
  std::vector<double> tab((size_t)m->Kmax * nops * 5, 0.0);
  for (int i = 0; i < nops; ++i) {
    const double s = ops[i]->d.param, mu = ops[i]->d.mu;
    const bool ex = ops[i]->d.func == WL_F_EXP;
    double omega = 1.0;
    for (int k = 1; k <= m->K[i]; ++k) {
      if (ex) omega /= k;
      double* c = &tab[((size_t)(k - 1) * nops + i) * 5];
      c[0] = s;
      c[1] = k >= 3 ? s * s * mu * mu : 0.0;
      c[2] = k >= 2 ? -s * s * mu : 0.0;
      c[3] = omega;
      c[4] = k == m->K[i] ? 1.0 : 0.0;
    }
  }
  std::vector<double> tab_phi = tab;
  for (size_t e = 4; e < tab_phi.size(); e += 5) tab_phi[e] = 0.0;
  wl_status s = m->tab.ensure(tab.size() * 8);
  if (s == WL_OK) s = m->tab_phi.ensure(tab.size() * 8);
  if (s == WL_OK && (hipMemcpy(m->tab.p, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                     hipMemcpy(m->tab_phi.p, tab_phi.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess)) {
    wl_set_error("wl_multi_create: coefficient upload failed");
    s = WL_EDEVICE;
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
    return multi_apply<float>(m, (const float*)d_X, b, (float*)d_Y, laplacian != 0);
  }
  if (laplacian) WL_TRY(multi_ensure_w<double>(m));
  return multi_apply<double>(m, (const double*)d_X, b, (double*)d_Y, laplacian != 0);
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
    return multi_apply<float>(m, m->ones.as<float>(), 1, (float*)d_W, false);
  }
  WL_TRY(launch_fill<double>(m->g->ctx, n, 1.0, m->ones.as<double>()));
  return multi_apply<double>(m, m->ones.as<double>(), 1, (double*)d_W, false);
}

}  // extern "C"
