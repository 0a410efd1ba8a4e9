// Discrete-time diffusion on the graph (Sec. "Simulating discrete-time diffusion",
// eq. let_there_be_markov): P = I - D^{-1} L with D = diag(w), w = phi 1, i.e.
// P = diag(w)^{-1} phi, a row-stochastic matrix whose stationary distribution is
// pi = w / sum(w).  A step p_{k+1} = p_k P on distributions held as columns is
// p_{k+1}^T = phi (p_k^T ./ w): one scaling pass and one phi product.
#include <algorithm>
#include <cmath>

#include "wl_internal.h"

namespace {

// out[r] = x[r]^power for power in {-1, -1/2, 1/2}
template <typename T>
__global__ void k_wpow(int64_t n, const T* __restrict__ x, int mode, T* __restrict__ out) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)x[r];
    out[r] = (T)(mode == 0 ? 1.0 / v : (mode == 1 ? 1.0 / std::sqrt(v) : std::sqrt(v)));
  }
}

// out[r] = x[r] / *den (den a device double)
template <typename T>
__global__ void k_div_by(int64_t n, const T* __restrict__ x, const double* __restrict__ den, T* __restrict__ out) {
  const double d = *den;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    out[r] = (T)((double)x[r] / d);
}

int grid_for(int64_t n) { return (int)std::min<int64_t>(8192, std::max<int64_t>(1, (n + 255) / 256)); }

}  // namespace

template <typename T>
wl_status launch_wpow(wl_ctx* ctx, int64_t n, const T* x, int mode, T* out) {
  if (n == 0) return WL_OK;
  hipLaunchKernelGGL(k_wpow<T>, dim3(grid_for(n)), dim3(256), 0, ctx->stream, n, x, mode, out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_div_by(wl_ctx* ctx, int64_t n, const T* x, const double* den, T* out) {
  if (n == 0) return WL_OK;
  hipLaunchKernelGGL(k_div_by<T>, dim3(grid_for(n)), dim3(256), 0, ctx->stream, n, x, den, out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template wl_status launch_wpow<float>(wl_ctx*, int64_t, const float*, int, float*);
template wl_status launch_wpow<double>(wl_ctx*, int64_t, const double*, int, double*);
template wl_status launch_div_by<float>(wl_ctx*, int64_t, const float*, const double*, float*);
template wl_status launch_div_by<double>(wl_ctx*, int64_t, const double*, const double*, double*);

namespace {

template <typename T>
wl_status markov_step_impl(wl_op* op, const T* X, int b, int steps, T* Y) {
  wl_graph* g = op->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  WL_TRY(ensure_w<T>(op));
  DevBuf& rw = op->mk_rw;
  DevBuf& tmp = op->mk_tmp;
  DevBuf& alt = op->mk_alt;
  WL_TRY(rw.ensure((size_t)n * sizeof(T)));
  WL_TRY(tmp.ensure((size_t)n * b * sizeof(T)));
  if (steps > 1) WL_TRY(alt.ensure((size_t)n * b * sizeof(T)));
  WL_TRY(launch_wpow<T>(ctx, n, op->w.as<T>(), 0, rw.as<T>()));  // 1 / w
  const T* cur = X;
  for (int s = 0; s < steps; ++s) {
    // the last step lands in Y; earlier ones alternate between Y and a spare block so
    // that the input of a step is never its output
    T* out = ((steps - 1 - s) % 2 == 0) ? Y : alt.as<T>();
    WL_TRY(launch_axpby_rows<T>(ctx, n, b, rw.as<T>(), cur, 0.0, cur, tmp.as<T>()));  // p ./ w
    WL_TRY(phi_apply_impl<T>(op, tmp.as<T>(), out, b, nullptr, nullptr));
    cur = out;
  }
  WL_HIP(hipStreamSynchronize(ctx->stream));
  return WL_OK;
}

template <typename T>
wl_status markov_stationary_impl(wl_op* op, T* pi) {
  wl_graph* g = op->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  WL_TRY(ensure_w<T>(op));
  DevBuf& s = op->mk_x0;
  DevBuf& sum = op->mk_dd;
  WL_TRY(s.ensure((size_t)n * sizeof(T)));
  WL_TRY(sum.ensure(sizeof(double)));
  WL_TRY(launch_wpow<T>(ctx, n, op->w.as<T>(), 2, s.as<T>()));  // sqrt(w): sum(w) = ||sqrt(w)||^2
  WL_TRY(launch_gram<T>(ctx, n, s.as<T>(), 1, 0, 1, s.as<T>(), 1, sum.as<double>()));
  WL_TRY(launch_div_by<T>(ctx, n, op->w.as<T>(), sum.as<double>(), pi));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  return WL_OK;
}

}  // namespace

extern "C" {

wl_status wl_markov_step(wl_op* op, const void* d_X, int32_t b, int32_t steps, void* d_Y) {
  WL_CHECK(op, WL_EINVAL, "wl_markov_step: op is null");
  WL_CHECK(b >= 1 && b <= 64, WL_EINVAL, "wl_markov_step: b must lie in [1, 64]");
  WL_CHECK(steps >= 1, WL_EINVAL, "wl_markov_step: steps must be >= 1");
  WL_CHECK(op->g->n == 0 || (d_X && d_Y && d_X != d_Y), WL_EINVAL, "wl_markov_step: bad blocks");
  if (op->g->n == 0) return WL_OK;
  DeviceGuard dg(op->g->ctx->device);
  if (op->d.prec == WL_FP32) return markov_step_impl<float>(op, (const float*)d_X, b, steps, (float*)d_Y);
  return markov_step_impl<double>(op, (const double*)d_X, b, steps, (double*)d_Y);
}

wl_status wl_markov_stationary(wl_op* op, void* d_pi) {
  WL_CHECK(op, WL_EINVAL, "wl_markov_stationary: op is null");
  WL_CHECK(op->g->n == 0 || d_pi, WL_EINVAL, "wl_markov_stationary: output is null");
  if (op->g->n == 0) return WL_OK;
  DeviceGuard dg(op->g->ctx->device);
  if (op->d.prec == WL_FP32) return markov_stationary_impl<float>(op, (float*)d_pi);
  return markov_stationary_impl<double>(op, (double*)d_pi);
}

}  // extern "C"
