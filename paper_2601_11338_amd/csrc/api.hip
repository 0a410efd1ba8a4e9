// C ABI of the walk-Laplacian library and the Krylov drivers behind it.
//
// Drivers (all vector work on the device; only b x b blocks and the projected
// matrix cross to the host):
//  * fused recurrence: phi X = sum_k c_k q_k(A) X with q from eq. qrec, scaled as
//    P_k = s^k q_k X (s = alpha or beta) so that |P_k| stays O(1):
//      P_1 = s A P_0,  P_2 = s A P_1 - s^2 mu D P_0,
//      P_{k+1} = s A P_k + s^2 mu (mu I - D) P_{k-1}   (k >= 2),
//    S = sum_k (c_k / s^k) P_k accumulated in the SpMM epilogue, one launch per
//    degree (Prop. "whe-we-converge": the recurrence is the Taylor series of f_1
//    on the linearisation Z applied to [q_1; q_2]);
//  * block Lanczos (Sec. 4.1) on a symmetric operator, block CholQR2 with
//    deflation, local or full reorthogonalisation, three-term subtraction fused
//    into the SpMM epilogue.  The resolvent uses the deformed Laplacian
//    A_mu(alpha) = (1 - mu^2 alpha^2) I - alpha A + alpha^2 mu D, for which
//    phi = (1 - mu^2 alpha^2) A_mu(alpha)^{-1} (eq. deformed, extended to all mu as
//    the remark after Prop. "CGworks" states), so phi X = (1 - mu^2 a^2) V T^{-1} E_1 R_0;
//  * diffusion: outer block Lanczos on the walk Laplacian with inner phi products,
//    exp(-t T) from one eigendecomposition for every t (Alg. 1 shares one basis
//    across its parfor over t).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "wl_internal.h"
#include "wl_amg.h"

static wl_status noalloc_setup(int device);

// ------------------------------------------------------------------ errors
static thread_local char g_err[1024] = "";
thread_local int wl_no_alloc = 0;

void wl_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

// ------------------------------------------------------------------ allocation-failure hook
// Allocations left before the injected failure: -1 off, -2 the environment not read yet.
static std::atomic<int64_t> g_fail_alloc{-2};

static void wl_fail_alloc_set(int64_t k) { g_fail_alloc.store(k < 0 ? -1 : k); }

bool wl_alloc_injected() {
  int64_t k = g_fail_alloc.load();
  if (k == -2) {
    const char* e = std::getenv("WL_TEST_FAIL_ALLOC");
    int64_t v = -1;
    if (e && e[0]) {
      char* end = nullptr;
      const long long x = std::strtoll(e, &end, 10);
      if (end && *end == '\0' && x >= 0) v = x;
    }
    g_fail_alloc.compare_exchange_strong(k, v);
    k = g_fail_alloc.load();
  }
  while (k >= 0)
    if (g_fail_alloc.compare_exchange_weak(k, k == 0 ? -1 : k - 1)) return k == 0;
  return false;
}

// ------------------------------------------------------------------ output scan
namespace {

template <typename T>
__global__ void k_count_nonfinite(const T* __restrict__ p, int64_t count, unsigned long long* __restrict__ out) {
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    c += isfinite(p[i]) ? 0ull : 1ull;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0; }

}  // namespace

// WL_CHECK_FINITE: WL_ENUMERIC when any of the count values at p (an output of the
// call `who`, already enqueued) is NaN or Inf; waits for the call's work.
static wl_status scan_output(wl_ctx* ctx, int prec, const void* p, int64_t count, const char* who) {
  if (!(ctx->checks & WL_CHECK_FINITE) || count <= 0) return WL_OK;
  unsigned long long* d = ctx->check_count.as<unsigned long long>();
  WL_CHECK(d, WL_EINTERNAL, "%s: output scan without its counter", who);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (count + 255) / 256));
  k_zero_u64<<<1, 1, 0, ctx->stream>>>(d);
  if (prec == WL_FP32)
    k_count_nonfinite<float><<<grid, 256, 0, ctx->stream>>>((const float*)p, count, d);
  else
    k_count_nonfinite<double><<<grid, 256, 0, ctx->stream>>>((const double*)p, count, d);
  WL_HIP(hipGetLastError());
  unsigned long long bad = 0;
  WL_HIP(hipMemcpyAsync(&bad, d, sizeof(bad), hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  WL_CHECK(bad == 0, WL_ENUMERIC, "%s: %llu of the %lld output values are NaN or Inf", who, bad, (long long)count);
  return WL_OK;
}

namespace {


bool is_finite(double x) { return std::isfinite(x); }

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

int lanes_for(int prec, int b) {
  const int vw = prec == WL_FP32 ? 4 : 2;
  if (b % vw == 0) {
    int l = b / vw;
    if (l >= 16) return 16;
    return next_pow2(l);
  }
  return b == 1 ? 1 : std::min(16, next_pow2(b));
}

template <typename T>
T* tptr(const DevBuf& b, size_t off_elems = 0) {
  return b.as<T>() + off_elems;
}

}  // namespace

// The autotuned shape of (prec, b) if there is one, else a heuristic from the mean
// degree: enough neighbour slots per row to cover about half the mean degree.
SpmmShape shape_for(wl_graph* g, int prec, int b) {
  auto it = g->tuned.find(prec * 1000 + std::min(b, 999));
  if (it != g->tuned.end()) return it->second;
  SpmmShape s;
  const int lpn = lanes_for(prec, b);
  int ns = next_pow2(std::max(1, (int)std::ceil(g->mean_deg))) / 2;
  if (ns < 1) ns = 1;
  int G = std::max(4, std::min(64, lpn * ns));
  s.G = G;
  s.long_thr = std::max(g->long_min_thr, 32 * (G / lpn));
  return s;
}

extern "C" {

const char* wl_last_error(void) { return g_err; }

const char* wl_status_string(wl_status s) {
  switch (s) {
    case WL_OK: return "ok";
    case WL_EINVAL: return "invalid argument";
    case WL_ERANGE: return "out of range";
    case WL_ENOMEM: return "out of device memory";
    case WL_EDEVICE: return "device error";
    case WL_ENOTSPD: return "operator not positive definite";
    case WL_ENOCONV: return "no convergence";
    case WL_ENUMERIC: return "non-finite result";
    case WL_EUNSUPPORTED: return "unsupported";
    default: return "internal error";
  }
}

int32_t wl_version(void) { return 100; }

// ------------------------------------------------------------------ context
wl_status wl_test_fail_alloc(int64_t k) {
  wl_fail_alloc_set(k);
  return WL_OK;
}

wl_status wl_ctx_create(int32_t device, void* stream, wl_ctx** out) {
  WL_CHECK(out != nullptr, WL_EINVAL, "wl_ctx_create: out is null");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  WL_CHECK(e == hipSuccess && count > 0, WL_EDEVICE, "wl_ctx_create: no HIP device available");
  WL_CHECK(device >= 0 && device < count, WL_EINVAL, "wl_ctx_create: device %d out of range [0,%d)", device, count);
  DeviceGuard dg(device);
  WL_HIP(hipFree(nullptr));
  WL_TRY(noalloc_setup(device));
  auto* c = new wl_ctx;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  const char* tr = std::getenv("WL_TRACE");
  if (tr && tr[0] && std::strcmp(tr, "0") != 0) c->trace = c->profiling = true;
  *out = c;
  return WL_OK;
}

wl_status wl_ctx_set_checks(wl_ctx* ctx, uint32_t flags) {
  WL_CHECK(ctx, WL_EINVAL, "wl_ctx_set_checks: ctx is null");
  WL_CHECK((flags & ~WL_CHECK_FINITE) == 0, WL_EINVAL, "wl_ctx_set_checks: unknown flags");
  if (flags & WL_CHECK_FINITE) {
    DeviceGuard dg(ctx->device);
    WL_TRY(ctx->check_count.ensure(sizeof(unsigned long long)));
  }
  ctx->checks = flags;
  return WL_OK;
}

wl_status wl_ctx_set_stream(wl_ctx* ctx, void* stream) {
  WL_CHECK(ctx, WL_EINVAL, "wl_ctx_set_stream: ctx is null");
  ctx->stream = static_cast<hipStream_t>(stream);
  return WL_OK;
}

wl_status wl_ctx_synchronize(wl_ctx* ctx) {
  WL_CHECK(ctx, WL_EINVAL, "wl_ctx_synchronize: ctx is null");
  DeviceGuard dg(ctx->device);
  WL_HIP(hipStreamSynchronize(ctx->stream));
  return WL_OK;
}

wl_status wl_ctx_set_profiling(wl_ctx* ctx, int32_t on) {
  WL_CHECK(ctx, WL_EINVAL, "wl_ctx_set_profiling: ctx is null");
  DeviceGuard dg(ctx->device);
  WL_HIP(hipStreamSynchronize(ctx->stream));
  for (auto& k : ctx->kstats) {
    k.launches = 0;
    k.bytes = 0.0;
    k.used = 0;
    k.folded_ms = 0.0;
  }
  ctx->profiling = on != 0;
  return WL_OK;
}

wl_status wl_ctx_kernel_stats(wl_ctx* ctx, int32_t kclass, int64_t* launches, double* total_ms, double* alg_bytes) {
  WL_CHECK(ctx, WL_EINVAL, "wl_ctx_kernel_stats: ctx is null");
  WL_CHECK(kclass >= 0 && kclass < WL_KC_COUNT, WL_EINVAL, "wl_ctx_kernel_stats: unknown kernel class");
  DeviceGuard dg(ctx->device);
  WL_HIP(hipStreamSynchronize(ctx->stream));
  KernelStats& k = ctx->kstats[kclass];
  double ms = k.folded_ms;
  for (size_t i = 0; i < k.used; ++i) {
    float e = 0.f;
    WL_HIP(hipEventElapsedTime(&e, k.events[i].first, k.events[i].second));
    ms += e;
  }
  if (launches) *launches = k.launches;
  if (total_ms) *total_ms = ms;
  if (alg_bytes) *alg_bytes = k.bytes;
  return WL_OK;
}

wl_status wl_ctx_destroy(wl_ctx* ctx) {
  ctx_release(ctx);
  return WL_OK;
}

}  // extern "C"

// Handles are reference counted: a graph or network keeps its context alive and an
// operator keeps its graph alive, so the caller may destroy them in any order.
void ctx_release(wl_ctx* ctx) {
  if (!ctx || --ctx->refs > 0) return;
  {
    DeviceGuard dg(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->trace) {
      static const char* names[WL_KC_COUNT] = {"recurrence step", "Lanczos operator product", "other sparse product",
                                               "side-by-side series step", "side-by-side Lanczos product",
                                               "multigrid finest level"};
      for (int c = 0; c < WL_KC_COUNT; ++c) {
        KernelStats& k = ctx->kstats[c];
        if (!k.launches || kstats_fold(k) != WL_OK) continue;
        std::fprintf(stderr, "[walklap trace] device %d, %s: %lld launches, %.3f ms, %.1f GB/s algorithmic\n",
                     ctx->device, names[c], (long long)k.launches, k.folded_ms,
                     k.folded_ms > 0 ? k.bytes / (k.folded_ms * 1e-3) / 1e9 : 0.0);
      }
    }
    for (auto& k : ctx->kstats)
      for (auto& e : k.events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
    ctx->partials.release();
    ctx->scratch.release();
    ctx->check_count.release();
  }
  delete ctx;
}

// Reads back the timed event pairs of a kernel class into folded_ms and frees them for
// reuse (waits for the last one).
wl_status kstats_fold(KernelStats& k) {
  if (!k.used) return WL_OK;
  WL_HIP(hipEventSynchronize(k.events[k.used - 1].second));
  for (size_t i = 0; i < k.used; ++i) {
    float e = 0.f;
    WL_HIP(hipEventElapsedTime(&e, k.events[i].first, k.events[i].second));
    k.folded_ms += e;
  }
  k.used = 0;
  return WL_OK;
}

wl_status kstats_begin(wl_ctx* ctx, int kc, KernelStats** out) {
  *out = nullptr;
  if (!ctx->profiling || kc < 0 || kc >= WL_KC_COUNT) return WL_OK;
  KernelStats* ks = &ctx->kstats[kc];
  if (ctx->trace && ks->used == WL_TRACE_FOLD) WL_TRY(kstats_fold(*ks));
  if (ks->used == ks->events.size()) {
    hipEvent_t a, c;
    WL_HIP(hipEventCreate(&a));
    WL_HIP(hipEventCreate(&c));
    ks->events.emplace_back(a, c);
  }
  WL_HIP(hipEventRecord(ks->events[ks->used].first, ctx->stream));
  *out = ks;
  return WL_OK;
}

wl_status kstats_end(wl_ctx* ctx, KernelStats* ks, double bytes) {
  if (!ks) return WL_OK;
  WL_HIP(hipEventRecord(ks->events[ks->used].second, ctx->stream));
  ++ks->used;
  ++ks->launches;
  ks->bytes += bytes;
  return WL_OK;
}

void graph_release(wl_graph* g) {
  if (!g || --g->refs > 0) return;
  wl_ctx* ctx = g->ctx;
  {
    DeviceGuard dg(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    delete g;
  }
  ctx_release(ctx);
}

extern "C" {

// ------------------------------------------------------------------ graph
wl_status wl_graph_check_size(int64_t n, int64_t nnz) {
  WL_CHECK(n >= 0 && nnz >= 0, WL_EINVAL, "graph size: negative n or nnz");
  WL_CHECK(n <= WL_MAX_ROWS, WL_ERANGE, "graph size: n = %lld exceeds %lld", (long long)n, (long long)WL_MAX_ROWS);
  // the sparse-product kernels walk a row's column list with 32-bit indices that run
  // up to 2^16 past the row's end before the loop test: nnz must leave that headroom
  WL_CHECK(nnz <= WL_MAX_NNZ, WL_ERANGE, "graph size: nnz = %lld exceeds %lld (int32 CSR with index headroom)",
           (long long)nnz, (long long)WL_MAX_NNZ);
  return WL_OK;
}

wl_status wl_graph_create(wl_ctx* ctx, int64_t n, int64_t nnz, const int32_t* d_rowptr, const int32_t* d_colidx,
                          uint32_t flags, wl_graph** out) {
  WL_CHECK(ctx && out, WL_EINVAL, "wl_graph_create: null ctx or out");
  *out = nullptr;
  WL_CHECK(n >= 0 && nnz >= 0, WL_EINVAL, "wl_graph_create: negative size");
  WL_TRY(wl_graph_check_size(n, nnz));
  WL_CHECK(d_rowptr != nullptr, WL_EINVAL, "wl_graph_create: rowptr is null");
  WL_CHECK(nnz == 0 || d_colidx != nullptr, WL_EINVAL, "wl_graph_create: colidx is null");
  WL_CHECK((flags & ~(WL_GRAPH_COPY | WL_GRAPH_VALIDATE)) == 0, WL_EINVAL, "wl_graph_create: unknown flags");
  DeviceGuard dg(ctx->device);
  auto* g = new wl_graph;
  g->ctx = ctx;
  g->n = n;
  g->nnz = nnz;
  auto fail = [&](wl_status s) {
    delete g;
    return s;
  };
  if (flags & WL_GRAPH_COPY) {
    wl_status s = g->own_rowptr.ensure((size_t)(n + 1) * 4);
    if (s != WL_OK) return fail(s);
    s = g->own_colidx.ensure((size_t)std::max<int64_t>(nnz, 1) * 4);
    if (s != WL_OK) return fail(s);
    if (hipMemcpyAsync(g->own_rowptr.p, d_rowptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice, ctx->stream) !=
            hipSuccess ||
        (nnz > 0 && hipMemcpyAsync(g->own_colidx.p, d_colidx, (size_t)nnz * 4, hipMemcpyDeviceToDevice,
                                   ctx->stream) != hipSuccess)) {
      wl_set_error("wl_graph_create: copying the CSR arrays failed");
      return fail(WL_EDEVICE);
    }
    g->rowptr = g->own_rowptr.as<int32_t>();
    g->colidx = g->own_colidx.as<int32_t>();
  } else {
    g->rowptr = d_rowptr;
    g->colidx = d_colidx;
  }
  // host copy of rowptr: structural checks that protect every kernel, degree stats,
  // and the decreasing-degree list of long rows
  std::vector<int32_t> h(n + 1);
  if (hipMemcpyAsync(h.data(), g->rowptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    wl_set_error("wl_graph_create: reading rowptr failed (is it a device pointer?)");
    return fail(WL_EDEVICE);
  }
  if (h[0] != 0 || (int64_t)h[n] != nnz) {
    wl_set_error("wl_graph_create: rowptr[0] must be 0 and rowptr[n] must equal nnz (got %d, %d)", h[0], h[n]);
    return fail(WL_EINVAL);
  }
  int32_t maxd = 0;
  std::vector<std::pair<int32_t, int32_t>> longs;
  for (int64_t r = 0; r < n; ++r) {
    const int32_t d = h[r + 1] - h[r];
    if (d < 0) {
      wl_set_error("wl_graph_create: rowptr decreases at row %lld", (long long)r);
      return fail(WL_EINVAL);
    }
    maxd = std::max(maxd, d);
    if (d > g->long_min_thr) longs.emplace_back(d, (int32_t)r);
  }
  g->max_deg = maxd;
  g->mean_deg = n > 0 ? (double)nnz / (double)n : 0.0;
  std::sort(longs.begin(), longs.end(), [](const auto& a, const auto& b) {
    return a.first != b.first ? a.first > b.first : a.second < b.second;
  });
  {
    std::vector<int32_t> rows(longs.size());
    g->h_long_deg.resize(longs.size());
    for (size_t i = 0; i < longs.size(); ++i) {
      rows[i] = longs[i].second;
      g->h_long_deg[i] = longs[i].first;
    }
    wl_status s = g->long_rows.ensure(std::max<size_t>(rows.size(), 1) * 4);
    if (s != WL_OK) return fail(s);
    if (!rows.empty() &&
        hipMemcpy(g->long_rows.p, rows.data(), rows.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      wl_set_error("wl_graph_create: upload of the long-row list failed");
      return fail(WL_EDEVICE);
    }
  }
  // column range always; full structure (order, loops, symmetry) on request
  if (n > 0) {
    DevBuf flagsbuf;
    wl_status s = flagsbuf.ensure(8 * 4);
    if (s != WL_OK) return fail(s);
    if (hipMemsetAsync(flagsbuf.p, 0, 8 * 4, ctx->stream) != hipSuccess) return fail(WL_EDEVICE);
    s = launch_validate(g, flagsbuf.as<int32_t>());
    if (s != WL_OK) return fail(s);
    int32_t hf[8];
    if (hipMemcpyAsync(hf, flagsbuf.p, sizeof(hf), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return fail(WL_EDEVICE);
    if (hf[0] || hf[1]) {
      wl_set_error("wl_graph_create: column index out of range or malformed rowptr");
      return fail(WL_EINVAL);
    }
    if (flags & WL_GRAPH_VALIDATE) {
      if (hf[2]) {
        wl_set_error("wl_graph_create: self loop (graphs must be simple)");
        return fail(WL_EINVAL);
      }
      if (hf[3]) {
        wl_set_error("wl_graph_create: columns not strictly increasing (unsorted or duplicate edge)");
        return fail(WL_EINVAL);
      }
      if (hf[4]) {
        wl_set_error("wl_graph_create: adjacency not symmetric");
        return fail(WL_EINVAL);
      }
    }
  }
  wl_status s = g->degf.ensure(std::max<int64_t>(n, 1) * 4);
  if (s == WL_OK) s = g->degd.ensure(std::max<int64_t>(n, 1) * 8);
  if (s == WL_OK) s = launch_degrees<float>(g, g->degf.as<float>());
  if (s == WL_OK) s = launch_degrees<double>(g, g->degd.as<double>());
  if (s != WL_OK) return fail(s);
  ++ctx->refs;
  *out = g;
  return WL_OK;
}

wl_status wl_graph_info(const wl_graph* g, int64_t* n, int64_t* nnz, int32_t* max_degree) {
  WL_CHECK(g, WL_EINVAL, "wl_graph_info: graph is null");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (max_degree) *max_degree = g->max_deg;
  return WL_OK;
}

wl_status wl_graph_destroy(wl_graph* g) {
  graph_release(g);
  return WL_OK;
}

wl_status wl_spmm(wl_graph* g, int32_t prec, const void* d_X, void* d_Y, int32_t b) {
  WL_CHECK(g, WL_EINVAL, "wl_spmm: graph is null");
  WL_CHECK(prec == WL_FP32 || prec == WL_FP64, WL_EINVAL, "wl_spmm: prec must be WL_FP32 or WL_FP64");
  WL_CHECK(b >= 1, WL_EINVAL, "wl_spmm: b must be >= 1");
  WL_CHECK(g->n == 0 || (d_X && d_Y), WL_EINVAL, "wl_spmm: null block");
  WL_CHECK(d_X != d_Y || g->n == 0, WL_EINVAL, "wl_spmm: X and Y must not alias");
  DeviceGuard dg(g->ctx->device);
  const SpmmShape sh = shape_for(g, prec, b);
  if (prec == WL_FP32) {
    EpiArgs<float> ep;
    return launch_spmm<float>(g, (const float*)d_X, (float*)d_Y, b, ep, sh);
  }
  EpiArgs<double> ep;
  return launch_spmm<double>(g, (const double*)d_X, (double*)d_Y, b, ep, sh);
}

wl_status wl_autotune(wl_graph* g, int32_t prec, int32_t b) {
  WL_CHECK(g, WL_EINVAL, "wl_autotune: graph is null");
  WL_CHECK(prec == WL_FP32 || prec == WL_FP64, WL_EINVAL, "wl_autotune: bad prec");
  WL_CHECK(b >= 1 && b <= 4096, WL_EINVAL, "wl_autotune: b out of range");
  if (g->n == 0) return WL_OK;
  DeviceGuard dg(g->ctx->device);
  const size_t es = prec == WL_FP32 ? 4 : 8;
  DevBuf X, Y;
  WL_TRY(X.ensure((size_t)g->n * b * es));
  WL_TRY(Y.ensure((size_t)g->n * b * es));
  hipStream_t st = g->ctx->stream;
  if (prec == WL_FP32)
    WL_TRY(launch_fill<float>(g->ctx, g->n * b, 1.0f, X.as<float>()));
  else
    WL_TRY(launch_fill<double>(g->ctx, g->n * b, 1.0, X.as<double>()));
  const int lpn = lanes_for(prec, b);
  std::vector<SpmmShape> cands;
  for (int G = std::max(4, lpn); G <= 64; G <<= 1) {
    for (int mult : {8, 32, 128}) {
      SpmmShape s;
      s.G = G;
      s.long_thr = std::max(g->long_min_thr, mult * (G / lpn));
      cands.push_back(s);
    }
  }
  hipEvent_t e0, e1;
  WL_HIP(hipEventCreate(&e0));
  WL_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  SpmmShape bests = shape_for(g, prec, b);
  for (const auto& s : cands) {
    auto run = [&]() -> wl_status {
      if (prec == WL_FP32) {
        EpiArgs<float> ep;
        return launch_spmm<float>(g, X.as<float>(), Y.as<float>(), b, ep, s);
      }
      EpiArgs<double> ep;
      return launch_spmm<double>(g, X.as<double>(), Y.as<double>(), b, ep, s);
    };
    WL_TRY(run());  // warm
    // best of three timings of five launches each
    float ms = 1e30f;
    for (int trial = 0; trial < 3; ++trial) {
      WL_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < 5; ++r) WL_TRY(run());
      WL_HIP(hipEventRecord(e1, st));
      WL_HIP(hipEventSynchronize(e1));
      float t = 0.f;
      WL_HIP(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, t);
    }
    // a later candidate must win by 5% (timing noise would otherwise flip between
    // near-equal shapes from run to run)
    if (ms < 0.95f * best) {
      best = ms;
      bests = s;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g->tuned[prec * 1000 + std::min(b, 999)] = bests;
  return WL_OK;
}

wl_status wl_graph_set_shape(wl_graph* g, int32_t prec, int32_t b, int32_t lanes_per_row, int32_t long_row_threshold) {
  WL_CHECK(g, WL_EINVAL, "wl_graph_set_shape: graph is null");
  WL_CHECK(prec == WL_FP32 || prec == WL_FP64, WL_EINVAL, "wl_graph_set_shape: bad prec");
  WL_CHECK(b >= 1 && b <= 4096, WL_EINVAL, "wl_graph_set_shape: b out of range");
  WL_CHECK(lanes_per_row >= 1 && lanes_per_row <= 64 && (lanes_per_row & (lanes_per_row - 1)) == 0, WL_EINVAL,
           "wl_graph_set_shape: lanes per row must be a power of two in [1, 64]");
  WL_CHECK(long_row_threshold >= 1, WL_EINVAL, "wl_graph_set_shape: bad long-row threshold");
  SpmmShape s;
  s.G = std::max({4, lanes_for(prec, b), (int)lanes_per_row});
  s.long_thr = std::max(g->long_min_thr, (int)long_row_threshold);
  g->tuned[prec * 1000 + std::min(b, 999)] = s;
  return WL_OK;
}

wl_status wl_graph_shape(wl_graph* g, int32_t prec, int32_t b, int32_t* lanes_per_row, int32_t* long_row_threshold) {
  WL_CHECK(g, WL_EINVAL, "wl_graph_shape: graph is null");
  WL_CHECK(prec == WL_FP32 || prec == WL_FP64, WL_EINVAL, "wl_graph_shape: bad prec");
  WL_CHECK(b >= 1 && b <= 4096, WL_EINVAL, "wl_graph_shape: b out of range");
  const SpmmShape s = shape_for(g, prec, b);
  if (lanes_per_row) *lanes_per_row = s.G;
  if (long_row_threshold) *long_row_threshold = s.long_thr;
  return WL_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ block Lanczos core
namespace {

// Operator applied by the Lanczos driver to block V (n x b), result into W, with the
// three-term subtraction W -= Vprev Bprev^T fused when possible.
template <typename T>
struct LanczosOp {
  // 0: a*A + (b0 + b1 d) I (one SpMM); 1: walk Laplacian of an operator;
  // 2: the symmetrised Markov matrix of an operator, diag(w)^{-1/2} phi diag(w)^{-1/2}
  int kind = 0;
  double a = 1.0, b0 = 0.0, b1 = 0.0;
  wl_op* inner = nullptr;  // kinds 1, 2
  const T* rw = nullptr;   // kind 2: w^{-1/2}
  T* tmp1 = nullptr;       // kind 2: n x b scratch
  T* tmp2 = nullptr;       // kind 2: n x b scratch
};

template <typename T>
wl_status apply_lanczos_op(wl_graph* g, const LanczosOp<T>& L, const T* V, T* W, int b, const T* Vprev,
                           const double* Bprev, double* scratch) {
  if (L.kind == 0) {
    EpiArgs<T> ep;
    ep.a = L.a;
    if (L.b0 != 0.0 || L.b1 != 0.0) {
      ep.Z = V;
      ep.b0 = L.b0;
      ep.b1 = L.b1;
    }
    if (Vprev) {
      ep.Z2 = Vprev;
      ep.C = Bprev;
      ep.transC = 1;
    }
    ep.kclass = b >= 4 ? WL_KC_LANCZOS_OP : WL_KC_OTHER_SPMM;
    return launch_spmm<T>(g, V, W, b, ep, shape_for(g, prec_of<T>(), b));
  }
  wl_op* op = L.inner;
  if (L.kind == 2) {
    // W = D^{-1/2} phi D^{-1/2} V (the driver keeps the basis orthogonal to v)
    const int64_t n = g->n;
    WL_TRY(launch_axpby_rows<T>(g->ctx, n, b, L.rw, V, 0.0, V, L.tmp1));
    WL_TRY(phi_apply_impl<T>(op, L.tmp1, L.tmp2, b, nullptr, nullptr));
    WL_TRY(launch_axpby_rows<T>(g->ctx, n, b, L.rw, L.tmp2, 0.0, L.tmp2, W));
  } else {
    // walk Laplacian: W = w (.) V - phi V
    WL_TRY(phi_apply_impl<T>(op, V, W, b, op->w.as<T>(), V));
  }
  // then the three-term subtraction
  if (Vprev) {
    WL_TRY(launch_dtranspose(g->ctx, b, Bprev, scratch));
    WL_TRY(launch_update<T>(g->ctx, g->n, Vprev, b, 0, 1, scratch, W, 1.0, nullptr, -1.0, W, b, nullptr));
  }
  return WL_OK;
}

// Runs K block Lanczos steps from X (n x b).  basis must hold (K+1) blocks, Wb one
// block.  On return the host arrays hold A_j (K blocks), B_j (K blocks; B_{K-1}
// is the residual coupling), R0 (X = V_0 R0).
// ring = true keeps only three basis blocks (slot j mod 3) and needs reorth = 0.
template <typename T>
wl_status block_lanczos(wl_graph* g, const LanczosOp<T>& L, const T* X, int b, int K, int reorth, T* basis, T* Wb,
                        DevBuf& small, std::vector<double>& hA, std::vector<double>& hB, std::vector<double>& hR0,
                        int* K_eff, bool ring = false) {
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  const int64_t blk = n * b;
  SmallLayout Ly{b, K, (size_t)b * b};
  WL_TRY(small.ensure(Ly.total() * sizeof(double)));
  double* S = small.as<double>();
  const double tol = defl_tol<T>();
  const double ptol = post_tol<T>();
  // V_0 R0 = X by CholQR2
  WL_TRY(launch_gram<T>(ctx, n, X, b, 0, 1, X, b, S + Ly.G()));
  WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R1(), S + Ly.Ri1(), nullptr, nullptr, 1, 0,
                     S + Ly.Ref()));
  WL_TRY(launch_update<T>(ctx, n, X, b, 0, 1, S + Ly.Ri1(), nullptr, 0.0, nullptr, 1.0, basis, b, S + Ly.G()));
  WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(),
                     S + Ly.R0(), 1, 0, nullptr, S + Ly.Ref(), ptol));
  WL_TRY(launch_update<T>(ctx, n, basis, b, 0, 1, S + Ly.Ri2(), nullptr, 0.0, nullptr, 1.0, basis, b, nullptr));
  if (ring) reorth = 0;
  // A basis that will span more than half of the space loses orthogonality under local
  // reorthogonalisation as its Ritz values converge (at exhaustion the projected matrix
  // gains spurious eigenvalues); there every block is orthogonalised against all
  // earlier ones, which costs little at such sizes.
  if (!ring && (int64_t)(K + 1) * b * 2 > n) reorth = std::max(reorth, 2);
  auto slot = [&](int j) { return basis + (size_t)(ring ? j % 3 : j) * blk; };
  if (!ring && reorth <= 1) {
    // Fused step: W' lands in basis slot j+1; one Gram of [V_{j-1} V_j W'] (reorth 1;
    // [V_j W'] with reorth 0) against W' gives the projection; W = [.. W'] Cc is
    // formed in place together with its own Gram; CholQR2 on that true Gram (with the
    // deflation check of the first factor against W's scale before projection)
    // orthonormalises it in place.
    for (int j = 0; j < K; ++j) {
      T* Vj = slot(j);
      T* Vn = slot(j + 1);
      const T* Vp = j > 0 ? slot(j - 1) : nullptr;
      WL_TRY(apply_lanczos_op<T>(g, L, Vj, Vn, b, Vp, j > 0 ? S + Ly.B(j - 1) : nullptr, S + Ly.P()));
      // projection against V_j (reorth 0), or a second local pass against V_{j-1} too
      const int nbv = j > 0 && reorth >= 1 ? 2 : 1;
      const T* Vlo = nbv == 2 ? Vp : Vj;
      WL_TRY(launch_gram<T>(ctx, n, Vlo, b, blk, nbv + 1, Vn, b, S + Ly.P()));
      WL_TRY(launch_lanczos_proj(ctx, b, nbv, S + Ly.P(), S + Ly.A(j), S + Ly.Cc(), S + Ly.Ref()));
      WL_TRY(launch_update<T>(ctx, n, Vlo, b, blk, nbv + 1, S + Ly.Cc(), nullptr, 0.0, nullptr, 1.0, Vn, b,
                              S + Ly.G()));
      WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, nullptr, S + Ly.Ri1(), nullptr, S + Ly.R1(), 1, 0,
                         nullptr, S + Ly.Ref(), ptol, S + Ly.Skip(), skip_ratio<T>()));
      if (j + 1 == K) {  // residual coupling B_{K-1} (a-posteriori error estimates)
        WL_TRY(launch_dcopy(ctx, b * b, S + Ly.R1(), S + Ly.B(j)));
        break;
      }
      // the second CholQR pass runs only when the first factor was ill conditioned
      // (device flag): otherwise its Gram and update return at once and B_j = R1
      WL_TRY(launch_update_skip<T>(ctx, n, Vn, b, 0, 1, S + Ly.Ri1(), nullptr, 0.0, nullptr, 1.0, Vn, b, S + Ly.G(),
                                   nullptr, S + Ly.Skip()));
      WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(),
                         S + Ly.B(j), 1, 0, nullptr, nullptr, 0.0, nullptr, 0.0, S + Ly.Skip()));
      WL_TRY(launch_update_skip<T>(ctx, n, Vn, b, 0, 1, S + Ly.Ri2(), nullptr, 0.0, nullptr, 1.0, Vn, b, nullptr,
                                   S + Ly.Skip(), nullptr));
    }
  }
  for (int j = 0; j < K && (ring || reorth > 1); ++j) {
    T* Vj = slot(j);
    const T* Vp = j > 0 ? slot(j - 1) : nullptr;
    WL_TRY(apply_lanczos_op<T>(g, L, Vj, Wb, b, Vp, j > 0 ? S + Ly.B(j - 1) : nullptr, S + Ly.P()));
    // A_j = V_j^T W ; W -= V_j A_j
    WL_TRY(launch_gram<T>(ctx, n, Vj, b, 0, 1, Wb, b, S + Ly.A(j)));
    const bool second = reorth >= 1;
    WL_TRY(launch_update<T>(ctx, n, Vj, b, 0, 1, S + Ly.A(j), Wb, 1.0, nullptr, -1.0, Wb, b,
                            second ? nullptr : S + Ly.G()));
    if (second) {
      // reorth 3: also against the block stored just before slot 0 (a locked vector)
      const int lo = reorth >= 3 ? -1 : (reorth >= 2 ? 0 : std::max(0, j - 1));
      const int nb = j - lo + 1;
      const T* Vlo = basis + (size_t)lo * blk;
      WL_TRY(launch_gram<T>(ctx, n, Vlo, b, blk, nb, Wb, b, S + Ly.P()));
      WL_TRY(launch_update<T>(ctx, n, Vlo, b, blk, nb, S + Ly.P(), Wb, 1.0, nullptr, -1.0, Wb, b, S + Ly.G()));
      WL_TRY(launch_dadd(ctx, b * b, S + Ly.P() + (size_t)(nb - 1) * b * b, S + Ly.A(j)));
    }
    // W = V_{j+1} B_j by CholQR2
    WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, S + Ly.A(j), j > 0 ? S + Ly.B(j - 1) : nullptr, S + Ly.R1(),
                       S + Ly.Ri1(), nullptr, nullptr, 1, 0, S + Ly.Ref()));
    if (j + 1 == K) {
      WL_TRY(launch_dcopy(ctx, b * b, S + Ly.R1(), S + Ly.B(j)));
      break;
    }
    T* Vn = slot(j + 1);
    WL_TRY(launch_update<T>(ctx, n, Wb, b, 0, 1, S + Ly.Ri1(), nullptr, 0.0, nullptr, 1.0, Vn, b, S + Ly.G()));
    WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(),
                       S + Ly.B(j), 1, 0, nullptr, S + Ly.Ref(), ptol));
    WL_TRY(launch_update<T>(ctx, n, Vn, b, 0, 1, S + Ly.Ri2(), nullptr, 0.0, nullptr, 1.0, Vn, b, nullptr));
  }
  hA.assign((size_t)K * b * b, 0.0);
  hB.assign((size_t)K * b * b, 0.0);
  hR0.assign((size_t)b * b, 0.0);
  WL_HIP(hipMemcpyAsync(hA.data(), S + Ly.A(0), hA.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipMemcpyAsync(hB.data(), S + Ly.B(0), hB.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipMemcpyAsync(hR0.data(), S + Ly.R0(), hR0.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  // effective dimension: stop after the first block whose coupling vanished entirely
  int Ke = K;
  for (int j = 0; j + 1 < K; ++j) {
    double s = 0.0;
    for (int e = 0; e < b * b; ++e) s += hB[(size_t)j * b * b + e] * hB[(size_t)j * b * b + e];
    if (s == 0.0) {
      Ke = j + 1;
      break;
    }
  }
  *K_eff = Ke;
  for (double v : hA)
    if (!is_finite(v)) {
      wl_set_error("block Lanczos produced non-finite coefficients");
      return WL_ENUMERIC;
    }
  return WL_OK;
}

// Assemble the (K b) x (K b) block tridiagonal T.
std::vector<double> assemble_T(int K, int b, const std::vector<double>& hA, const std::vector<double>& hB) {
  const int m = K * b;
  std::vector<double> T((size_t)m * m, 0.0);
  for (int j = 0; j < K; ++j) {
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c) {
        T[(size_t)(j * b + r) * m + j * b + c] = hA[(size_t)j * b * b + r * b + c];
        if (j + 1 < K) {
          const double v = hB[(size_t)j * b * b + r * b + c];  // T_{j+1, j}
          T[(size_t)((j + 1) * b + r) * m + j * b + c] = v;
          T[(size_t)(j * b + c) * m + (j + 1) * b + r] = v;
        }
      }
  }
  return T;
}

// F = f(T) E_1 R0 via the eigendecomposition of T (m = K b), f applied to eigenvalues;
// T = U diag(lam) U^T kept in factored form (U applied to the b-column block only).
template <typename Fn>
int coeffs_by_eig(int K, int b, const std::vector<double>& hA, const std::vector<double>& hB,
                  const std::vector<double>& hR0, Fn f, std::vector<double>& F) {
  const int m = K * b;
  std::vector<double> T = assemble_T(K, b, hA, hB);
  SymEig E;
  if (sym_eig_factor(m, T.data(), E)) return 1;
  F.assign((size_t)m * b, 0.0);
  for (int k = 0; k < b; ++k)
    for (int c = 0; c < b; ++c) F[(size_t)k * b + c] = hR0[(size_t)k * b + c];
  sym_eig_apply_ut(E, b, F.data());
  for (int i = 0; i < m; ++i) {
    const double fi = f(E.lam[i]);
    for (int c = 0; c < b; ++c) F[(size_t)i * b + c] *= fi;
  }
  sym_eig_apply_u(E, b, F.data());
  return 0;
}

template <typename T>
wl_status recombine(wl_graph* g, const T* basis, int b, int K, const std::vector<double>& F, DevBuf& coef,
                    const T* wv, const T* Xw, T* Y) {
  WL_TRY(coef.ensure(F.size() * sizeof(double)));
  WL_HIP(hipMemcpyAsync(coef.p, F.data(), F.size() * 8, hipMemcpyHostToDevice, g->ctx->stream));
  WL_HIP(hipStreamSynchronize(g->ctx->stream));
  if (wv)
    return launch_update<T>(g->ctx, g->n, basis, b, g->n * b, K, coef.as<double>(), Xw, 0.0, wv, -1.0, Y, b, nullptr);
  return launch_update<T>(g->ctx, g->n, basis, b, g->n * b, K, coef.as<double>(), nullptr, 0.0, nullptr, 1.0, Y, b,
                          nullptr);
}

// phi X through the fused recurrence.
template <typename T>
wl_status phi_recurrence(wl_op* op, const T* X, T* Y, int b, const T* wv, const T* Xw) {
  wl_graph* g = op->g;
  const int64_t n = g->n;
  const double mu = op->d.mu;
  // P_k = s^k q_k X and weights omega_k = c_k / s^k.  Resolvent: s = alpha (alpha
  // rho(Z) < 1 keeps both bounded).  Exponential: s = min(beta, 1 / lambda_max) keeps
  // P_k bounded (q_k <= A^k entrywise) and omega_k = (beta / s)^k / k! <= e^{beta / s};
  // with s = beta the P_k would grow like (beta lambda_max)^k and leave the FP32 range.
  const bool ex = op->d.func == WL_F_EXP;
  const double s = ex && op->lam > 0.0 ? std::min(op->d.param, 1.0 / op->lam) : op->d.param;
  const double ratio = ex ? op->d.param / s : 1.0;
  const int K = op->K;
  WL_TRY(op->bufA.ensure((size_t)n * b * sizeof(T)));
  WL_TRY(op->bufB.ensure((size_t)n * b * sizeof(T)));
  T* A = op->bufA.as<T>();
  T* B = op->bufB.as<T>();
  const SpmmShape sh = shape_for(g, prec_of<T>(), b);
  auto omega = [&](int k) {
    if (!ex) return 1.0;
    double f = 1.0;
    for (int i = 1; i <= k; ++i) f *= ratio / i;
    return f;
  };
  if (K == 0) {
    // phi = c_0 I
    if (wv) return launch_axpby_rows<T>(g->ctx, n, b, wv, Xw, -1.0, X, Y);
    return launch_axpby_rows<T>(g->ctx, n, b, nullptr, X, 0.0, X, Y);
  }
  // step 1: P_1 = s A X ; S = X + omega_1 P_1
  {
    EpiArgs<T> ep;
    ep.a = s;
    ep.Sin = X;
    ep.Sout = Y;
    ep.s0 = 1.0;
    ep.sc = omega(1);
    if (K == 1) {
      ep.wv = wv;
      ep.Xw = Xw;
    }
    WL_TRY(launch_spmm<T>(g, X, K == 1 ? nullptr : A, b, ep, sh));
  }
  const T* Pm2 = X;  // P_{k-2}
  T* Pm1 = A;        // P_{k-1}
  T* spare = B;
  for (int k = 2; k <= K; ++k) {
    EpiArgs<T> ep;
    ep.a = s;
    ep.Z = Pm2;
    ep.b0 = (k == 2) ? 0.0 : s * s * mu * mu;
    ep.b1 = -s * s * mu;
    ep.Sin = Y;
    ep.Sout = Y;
    ep.s0 = 1.0;
    ep.sc = omega(k);
    const bool last = k == K;
    if (last) {
      ep.wv = wv;
      ep.Xw = Xw;
    }
    ep.kclass = b >= 4 ? WL_KC_RECURRENCE : WL_KC_OTHER_SPMM;
    // P_k overwrites the buffer of P_{k-2} (row r of P_{k-2} is read and row r of
    // P_k written by the same lanes); P_0 = X is never overwritten.
    T* out = (k == 2) ? spare : const_cast<T*>(Pm2);
    if (mu == 0.0) ep.Z = nullptr;
    WL_TRY(launch_spmm<T>(g, Pm1, last ? nullptr : out, b, ep, sh));
    Pm2 = Pm1;
    Pm1 = out;
  }
  return WL_OK;
}

}  // namespace

int expv_outer_steps(int outer_dim, int64_t n) {
  // n steps always reach an invariant space (a rank-deficient U0 grows by its rank)
  return (int)std::max<int64_t>(1, std::min<int64_t>(outer_dim, n));
}

int lanczos_steps(const wl_op* op, int64_t n, int b) {
  // The block Krylov space has dimension <= n and grows by at least one per step until
  // it is invariant, so n + 1 steps always suffice; fewer would not: a block with
  // deflated (zero or dependent) columns grows by its rank, not by b.  Steps after the
  // space is exhausted are zero blocks (the coupling vanishes and the process stops).
  (void)b;
  return (int)std::max<int64_t>(1, std::min<int64_t>(op->K, n + 1));
}

void lanczos_params(const wl_op* op, double* a, double* b0, double* b1) {
  const double mu = op->d.mu, p = op->d.param;
  if (op->d.func == WL_F_RESOLVENT) {
    // A_mu(alpha) = (1 - mu^2 a^2) I - a A + a^2 mu D
    *a = -p;
    *b0 = 1.0 - mu * mu * p * p;
    *b1 = p * p * mu;
  } else {
    *a = 1.0;  // mu = 0: phi = exp(beta A)
    *b0 = *b1 = 0.0;
  }
}

wl_status lanczos_coefficients(const wl_op* op, int Ke, int b, const std::vector<double>& hA,
                               const std::vector<double>& hB, const std::vector<double>& hR0,
                               std::vector<double>& F) {
  const double mu = op->d.mu, p = op->d.param;
  const double scale = op->d.func == WL_F_RESOLVENT ? 1.0 - mu * mu * p * p : 1.0;
  if (op->d.func == WL_F_RESOLVENT) {
    // F = scale * T^{-1} E_1 R0
    std::vector<double> rhs((size_t)Ke * b * b, 0.0), sol((size_t)Ke * b * b);
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c) rhs[(size_t)r * b + c] = hR0[(size_t)r * b + c];
    // Deflated basis columns leave rows of T that are exactly zero (and zero right-hand
    // sides): give them a unit diagonal so they decouple from the solve.
    std::vector<double> Ad(hA.begin(), hA.begin() + (size_t)Ke * b * b);
    for (int j = 0; j < Ke; ++j)
      for (int c = 0; c < b; ++c) {
        bool zero = true;
        for (int k = 0; k < b && zero; ++k) {
          zero = Ad[(size_t)j * b * b + c * b + k] == 0.0;
          if (zero && j > 0) zero = hB[(size_t)(j - 1) * b * b + c * b + k] == 0.0;   // T_{j, j-1} row c
          if (zero && j + 1 < Ke) zero = hB[(size_t)j * b * b + k * b + c] == 0.0;    // T_{j+1, j} column c
        }
        if (zero) Ad[(size_t)j * b * b + c * b + c] = 1.0;
      }
    bool ok = block_tridiag_solve(Ke, b, Ad.data(), hB.data(), rhs.data(), b, sol.data()) == 0;
    if (ok) {
      F.resize(sol.size());
      for (size_t i = 0; i < sol.size(); ++i) F[i] = scale * sol[i];
    } else {
      // deflated (singular) projection: pseudo-inverse through the eigendecomposition
      std::vector<double> lam;
      double lmax = 0.0;
      {
        std::vector<double> Tm = assemble_T(Ke, b, hA, hB);
        std::vector<double> l(Ke * b), U((size_t)Ke * b * Ke * b);
        if (dense_syev(Ke * b, Tm.data(), l.data(), U.data())) {
          wl_set_error("eigendecomposition of the projected matrix failed");
          return WL_ENOCONV;
        }
        for (double v : l) lmax = std::max(lmax, std::fabs(v));
        if (l[0] < -1e-6 * lmax) {
          wl_set_error("deformed Laplacian not positive definite on the Krylov space (alpha too large?)");
          return WL_ENOTSPD;
        }
      }
      const double cut = 1e-12 * lmax;
      if (coeffs_by_eig(Ke, b, hA, hB, hR0, [&](double x) { return x > cut ? scale / x : 0.0; }, F)) {
        wl_set_error("eigendecomposition of the projected matrix failed");
        return WL_ENOCONV;
      }
    }
  } else {
    if (coeffs_by_eig(Ke, b, hA, hB, hR0, [&](double x) { return std::exp(p * x); }, F)) {
      wl_set_error("eigendecomposition of the projected matrix failed");
      return WL_ENOCONV;
    }
  }
  return WL_OK;
}

namespace {

template <typename T>
wl_status phi_lanczos(wl_op* op, const T* X, T* Y, int b, const T* wv, const T* Xw) {
  wl_graph* g = op->g;
  const int64_t n = g->n;
  const int K = lanczos_steps(op, n, b);
  LanczosOp<T> L;
  lanczos_params(op, &L.a, &L.b0, &L.b1);
  WL_TRY(op->basis.ensure((size_t)(K + 1) * n * b * sizeof(T)));
  WL_TRY(op->wbuf.ensure((size_t)n * b * sizeof(T)));
  std::vector<double> hA, hB, hR0;
  int Ke = K;
  WL_TRY(block_lanczos<T>(g, L, X, b, K, op->d.reorth, op->basis.as<T>(), op->wbuf.as<T>(), op->small, hA, hB, hR0,
                          &Ke));
  std::vector<double> F;
  WL_TRY(lanczos_coefficients(op, Ke, b, hA, hB, hR0, F));
  return recombine<T>(g, op->basis.as<T>(), b, Ke, F, op->coef, wv, Xw, Y);
}

}  // namespace

template <typename T>
wl_status phi_apply_impl(wl_op* op, const T* X, T* Y, int b, const T* wv, const T* Xw) {
  if (op->g->n == 0) return WL_OK;
  if (op->d.method == WL_M_LANCZOS) return phi_lanczos<T>(op, X, Y, b, wv, Xw);
  if (op->d.method == WL_M_ARNOLDI) return phi_arnoldi<T>(op, X, Y, b, wv, Xw);
  if (op->d.method == WL_M_AMG_CG) return phi_amg<T>(op, X, Y, b, wv, Xw);
  return phi_recurrence<T>(op, X, Y, b, wv, Xw);
}

template wl_status phi_apply_impl<float>(wl_op*, const float*, float*, int, const float*, const float*);
template wl_status phi_apply_impl<double>(wl_op*, const double*, double*, int, const double*, const double*);

template <typename T>
wl_status expv_impl(wl_op* op, const T* U0, int b, const double* t, int nt, T* const* Y, int outer_dim,
                    double* err_est) {
  wl_graph* g = op->g;
  const int64_t n = g->n;
  const int K = expv_outer_steps(outer_dim, n);
  WL_TRY(op->outer_basis.ensure((size_t)(K + 1) * n * b * sizeof(T)));
  WL_TRY(op->outer_w.ensure((size_t)n * b * sizeof(T)));
  LanczosOp<T> L;
  L.kind = 1;
  L.inner = op;
  std::vector<double> hA, hB, hR0;
  int Ke = K;
  // The walk Laplacian of a graph with hubs has a few large, quickly converging Ritz
  // values; with local reorthogonalisation the basis then loses orthogonality and the
  // projected matrix gains spurious (even negative) eigenvalues, which exp(-t T)
  // amplifies.  The outer basis is therefore orthogonalised against every earlier
  // block (its cost is small next to the inner products with phi).
  WL_TRY(block_lanczos<T>(g, L, U0, b, K, std::max(op->d.reorth, 2), op->outer_basis.as<T>(), op->outer_w.as<T>(),
                          op->outer_small, hA, hB, hR0, &Ke));
  const int m = Ke * b;
  std::vector<double> Tm = assemble_T(Ke, b, hA, hB);
  // T = U diag(lam) U^T in factored form (U is applied to blocks, never formed)
  SymEig E;
  if (sym_eig_factor(m, Tm.data(), E)) {
    wl_set_error("eigendecomposition of the projected Laplacian failed");
    return WL_ENOCONV;
  }
  // W0 = U^T E_1 R0, then F_t = U exp(-t lam) W0 for all times at once (m x nt b)
  std::vector<double> W0((size_t)m * b, 0.0);
  for (int k = 0; k < b; ++k)
    for (int c = 0; c < b; ++c) W0[(size_t)k * b + c] = hR0[(size_t)k * b + c];
  sym_eig_apply_ut(E, b, W0.data());
  const int nb = nt * b;
  std::vector<double> Fall((size_t)m * nb);
  for (int i = 0; i < m; ++i)
    for (int it = 0; it < nt; ++it) {
      const double f = std::exp(-t[it] * E.lam[i]);
      for (int c = 0; c < b; ++c) Fall[(size_t)i * nb + it * b + c] = f * W0[(size_t)i * b + c];
    }
  sym_eig_apply_u(E, nb, Fall.data());
  for (int it = 0; it < nt; ++it) {
    std::vector<double> F((size_t)m * b);
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < b; ++c) F[(size_t)r * b + c] = Fall[(size_t)r * nb + it * b + c];
    if (err_est) {
      // || B_{K-1} F_last ||_F with F_last the last block row of F
      double e2 = 0.0;
      if (Ke == K) {
        const double* Bl = &hB[(size_t)(K - 1) * b * b];
        for (int r = 0; r < b; ++r)
          for (int c = 0; c < b; ++c) {
            double s = 0.0;
            for (int k = 0; k < b; ++k) s += Bl[(size_t)r * b + k] * F[(size_t)((K - 1) * b + k) * b + c];
            e2 += s * s;
          }
      }
      err_est[it] = std::sqrt(e2);
    }
    WL_TRY(recombine<T>(g, op->outer_basis.as<T>(), b, Ke, F, op->outer_coef, nullptr, nullptr, Y[it]));
    if (it + 1 < nt) WL_HIP(hipStreamSynchronize(g->ctx->stream));  // coefficient buffer is reused
  }
  return WL_OK;
}

template wl_status expv_impl<float>(wl_op*, const float*, int, const double*, int, float* const*, int, double*);
template wl_status expv_impl<double>(wl_op*, const double*, int, const double*, int, double* const*, int, double*);

// The chain P = diag(w)^{-1} phi (Sec. "Simulating discrete-time diffusion") is similar
// to the symmetric S = D^{-1/2} phi D^{-1/2}, whose top eigenvalue 1 has eigenvector
// sqrt(w).  Single-vector Lanczos, fully reorthogonalised, on S with that eigenvector
// deflated, from a seeded Gaussian start vector orthogonal to it: the extreme Ritz
// values of the projected tridiagonal matrix estimate lambda_2 and lambda_min of P, and
// the gap separates 1 from the next eigenvalue in modulus (the quantity compared
// across Laplacians in the tree experiment, Sec. 5).
template <typename T>
wl_status markov_gap_impl(wl_op* op, int outer_dim, uint64_t seed, double* lambda2, double* lambda_min,
                          double* gap) {
  wl_graph* g = op->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  WL_CHECK(n >= 3, WL_EINVAL, "wl_markov_gap: needs n >= 3");
  WL_TRY(ensure_w<T>(op));
  const int K = (int)std::max<int64_t>(2, std::min<int64_t>(outer_dim, n - 1));
  // outer basis: v = sqrt(w) / ||sqrt(w)|| in the block before slot 0, so that every
  // new Lanczos vector is orthogonalised against it with the earlier ones (a rounding-
  // level component along v would otherwise grow from step to step, by about
  // alpha / beta, until the eigenvalue 1 reappears among the Ritz values)
  WL_TRY(op->outer_basis.ensure((size_t)(K + 2) * n * sizeof(T)));
  WL_TRY(op->outer_w.ensure((size_t)n * sizeof(T)));
  T* vptr = op->outer_basis.as<T>();
  DevBuf& rw = op->mk_rw;
  DevBuf& x0 = op->mk_x0;
  DevBuf& t1 = op->mk_t1;
  DevBuf& t2 = op->mk_t2;
  DevBuf& dd = op->mk_dd;
  WL_TRY(rw.ensure((size_t)n * sizeof(T)));
  WL_TRY(x0.ensure((size_t)n * sizeof(T)));
  WL_TRY(t1.ensure((size_t)n * sizeof(T)));
  WL_TRY(t2.ensure((size_t)n * sizeof(T)));
  WL_TRY(dd.ensure(2 * sizeof(double)));
  WL_TRY(launch_wpow<T>(ctx, n, op->w.as<T>(), 1, rw.as<T>()));  // w^{-1/2}
  WL_TRY(launch_wpow<T>(ctx, n, op->w.as<T>(), 2, t1.as<T>()));  // sqrt(w)
  WL_TRY(launch_gram<T>(ctx, n, t1.as<T>(), 1, 0, 1, t1.as<T>(), 1, dd.as<double>()));
  double sw = 0.0;  // sum(w) = ||sqrt(w)||^2
  WL_HIP(hipMemcpyAsync(&sw, dd.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  WL_CHECK(sw > 0.0 && is_finite(sw), WL_ENUMERIC, "wl_markov_gap: walk degrees do not sum to a positive number");
  WL_TRY(launch_update<T>(ctx, n, t1.as<T>(), 1, 0, 0, nullptr, t1.as<T>(), 1.0 / std::sqrt(sw), nullptr, 0.0, vptr,
                          1, nullptr));
  // start vector: Gaussian, with its component along v removed
  WL_TRY(launch_probes<T>(ctx, WL_PROBE_GAUSS, seed, 0, n, 1, x0.as<T>()));
  WL_TRY(launch_gram<T>(ctx, n, vptr, 1, 0, 1, x0.as<T>(), 1, dd.as<double>()));
  WL_TRY(launch_update<T>(ctx, n, vptr, 1, 0, 1, dd.as<double>(), x0.as<T>(), 1.0, nullptr, -1.0, x0.as<T>(), 1,
                          nullptr));
  LanczosOp<T> L;
  L.kind = 2;
  L.inner = op;
  L.rw = rw.as<T>();
  L.tmp1 = t1.as<T>();
  L.tmp2 = t2.as<T>();
  std::vector<double> hA, hB, hR0;
  int Ke = K;
  WL_TRY(block_lanczos<T>(g, L, x0.as<T>(), 1, K, 3, vptr + n, op->outer_w.as<T>(), op->outer_small, hA, hB, hR0,
                          &Ke));
  std::vector<double> lam(Ke);
  if (tridiag_eigvals(Ke, hA.data(), hB.data(), lam.data())) {
    wl_set_error("wl_markov_gap: eigenvalues of the projected matrix failed");
    return WL_ENOCONV;
  }
  double lmax = lam[0], lmin = lam[0];
  for (double x : lam) {
    lmax = std::max(lmax, x);
    lmin = std::min(lmin, x);
  }
  if (lambda2) *lambda2 = lmax;
  if (lambda_min) *lambda_min = lmin;
  if (gap) *gap = 1.0 - std::max(std::fabs(lmax), std::fabs(lmin));
  return WL_OK;
}

template wl_status markov_gap_impl<float>(wl_op*, int, uint64_t, double*, double*, double*);
template wl_status markov_gap_impl<double>(wl_op*, int, uint64_t, double*, double*, double*);

// Spectral radius of the walk Laplacian: `steps` fully reorthogonalised single-vector
// Lanczos steps on L from a Gaussian vector (Philox stream `seed`); the largest Ritz
// value plus its residual norm (the Ritz value converges from below).
template <typename T>
wl_status laplacian_rho_impl(wl_op* op, int steps, uint64_t seed, double* rho) {
  wl_graph* g = op->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  WL_TRY(ensure_w<T>(op));
  const int K = (int)std::max<int64_t>(1, std::min<int64_t>(steps, n));
  DevBuf basis, wb, x0, small;
  WL_TRY(basis.ensure((size_t)(K + 1) * n * sizeof(T)));
  WL_TRY(wb.ensure((size_t)n * sizeof(T)));
  WL_TRY(x0.ensure((size_t)n * sizeof(T)));
  WL_TRY(launch_probes<T>(ctx, WL_PROBE_GAUSS, seed, 0, n, 1, x0.as<T>()));
  LanczosOp<T> L;
  L.kind = 1;
  L.inner = op;
  std::vector<double> hA, hB, hR0;
  int Ke = K;
  WL_TRY(block_lanczos<T>(g, L, x0.as<T>(), 1, K, 2, basis.as<T>(), wb.as<T>(), small, hA, hB, hR0, &Ke));
  // Ritz pair (theta, y) of the largest Ritz value; ||L V y - theta V y|| = |beta s_K|
  // with s_K the last component of y, which bounds the distance from theta to the
  // spectrum
  std::vector<double> Tm((size_t)Ke * Ke, 0.0), lam(Ke), S((size_t)Ke * Ke);
  for (int j = 0; j < Ke; ++j) {
    Tm[(size_t)j * Ke + j] = hA[j];
    if (j + 1 < Ke) Tm[(size_t)j * Ke + j + 1] = Tm[(size_t)(j + 1) * Ke + j] = hB[j];
  }
  if (dense_syev(Ke, Tm.data(), lam.data(), S.data())) {
    wl_set_error("spectral radius of the walk Laplacian: eigendecomposition of the projected matrix failed");
    return WL_ENOCONV;
  }
  int top = 0;
  for (int i = 1; i < Ke; ++i)
    if (lam[i] > lam[top]) top = i;
  *rho = lam[top] + std::fabs(hB[(size_t)(Ke - 1)] * S[(size_t)(Ke - 1) * Ke + top]);
  return WL_OK;
}

template wl_status laplacian_rho_impl<float>(wl_op*, int, uint64_t, double*);
template wl_status laplacian_rho_impl<double>(wl_op*, int, uint64_t, double*);

// ------------------------------------------------------------------ spectral scale
// kind 0: A; kind 1: A_mu(t).  Runs `steps` single-vector Lanczos steps from 1 and
// returns the extreme Ritz values.
wl_status lanczos_extreme(wl_graph* g, int kind, double mu, double t, int steps, double* lo, double* hi) {
  const int64_t n = g->n;
  const int K = (int)std::max<int64_t>(1, std::min<int64_t>(steps, n));
  LanczosOp<double> L;
  if (kind == 1) {
    L.a = -t;
    L.b0 = 1.0 - mu * mu * t * t;
    L.b1 = t * t * mu;
  }
  WL_TRY(g->tmp.ensure((size_t)4 * n * sizeof(double) + 256));
  double* basis = g->tmp.as<double>();
  double* W = basis + (size_t)3 * n;
  DevBuf ones, small;
  WL_TRY(ones.ensure((size_t)n * sizeof(double)));
  WL_TRY(launch_fill<double>(g->ctx, n, 1.0, ones.as<double>()));
  std::vector<double> hA, hB, hR0;
  int Ke = K;
  WL_TRY(block_lanczos<double>(g, L, ones.as<double>(), 1, K, 0, basis, W, small, hA, hB, hR0, &Ke, true));
  std::vector<double> a(Ke), bb(std::max(1, Ke - 1)), lam(Ke);
  for (int j = 0; j < Ke; ++j) a[j] = hA[j];
  for (int j = 0; j + 1 < Ke; ++j) bb[j] = hB[j];
  if (tridiag_eigvals(Ke, a.data(), bb.data(), lam.data())) {
    wl_set_error("tridiagonal eigenvalues did not converge");
    return WL_ENOCONV;
  }
  *lo = *std::min_element(lam.begin(), lam.end());
  *hi = *std::max_element(lam.begin(), lam.end());
  return WL_OK;
}

extern "C" {

wl_status wl_lambda_max(wl_graph* g, double tol, double* out) {
  WL_CHECK(g && out, WL_EINVAL, "wl_lambda_max: null argument");
  WL_CHECK(tol >= 0 && is_finite(tol), WL_EINVAL, "wl_lambda_max: bad tol");
  if (g->n == 0 || g->nnz == 0) {
    *out = 0.0;
    return WL_OK;
  }
  if (g->lam_max > 0) {
    *out = g->lam_max;
    return WL_OK;
  }
  DeviceGuard dg(g->ctx->device);
  if (tol == 0) tol = 1e-12;
  double prev = -1, lo, hi = 0;
  for (int steps = 60; steps <= 960; steps *= 2) {
    WL_TRY(lanczos_extreme(g, 0, 0.0, 0.0, steps, &lo, &hi));
    if (prev > 0 && std::fabs(hi - prev) <= tol * hi) break;
    if (steps >= g->n) break;
    prev = hi;
  }
  g->lam_max = hi;
  *out = hi;
  return WL_OK;
}

wl_status wl_spectral_radius(wl_graph* g, double mu, double tol, double* rho) {
  WL_CHECK(g && rho, WL_EINVAL, "wl_spectral_radius: null argument");
  WL_CHECK(mu >= 0.0 && mu <= 1.0, WL_EINVAL, "wl_spectral_radius: mu must lie in [0, 1]");
  WL_CHECK(tol >= 0 && is_finite(tol), WL_EINVAL, "wl_spectral_radius: bad tol");
  if (tol == 0) tol = 1e-10;
  double lam;
  WL_TRY(wl_lambda_max(g, 1e-12, &lam));
  if (mu == 0.0 || lam == 0.0) {
    *rho = lam;
    return WL_OK;
  }
  auto it = g->rho_cache.find(mu);
  if (it != g->rho_cache.end()) {
    *rho = it->second;
    return WL_OK;
  }
  DeviceGuard dg(g->ctx->device);
  const int steps = (int)std::min<int64_t>(g->n, 200);
  // f(t) = smallest Ritz value of A_mu(t); the first zero of f is 1 / rho(Z_mu)
  auto f = [&](double t, double* v) -> wl_status {
    double lo, hi, prev = 1e300;
    for (int s = steps; s <= 1600; s *= 2) {
      WL_TRY(lanczos_extreme(g, 1, mu, t, s, &lo, &hi));
      if (std::fabs(lo - prev) <= 1e-13 * std::max(1.0, std::fabs(hi)) || s >= g->n) break;
      prev = lo;
    }
    *v = lo;
    return WL_OK;
  };
  double tlo = 0.0, flo = 1.0, thi = 1.0 / lam, fhi;
  WL_TRY(f(thi, &fhi));
  int guard = 0;
  while (fhi > 0) {
    tlo = thi;
    flo = fhi;
    thi *= 1.05;
    WL_TRY(f(thi, &fhi));
    if (++guard > 400) {
      wl_set_error("wl_spectral_radius: no sign change of the deformed Laplacian's smallest eigenvalue");
      return WL_ENOCONV;
    }
  }
  // Illinois false position on [tlo, thi]
  int side = 0;
  for (int iter = 0; iter < 200 && (thi - tlo) > tol * thi * 0.25; ++iter) {
    double tm = (tlo * fhi - thi * flo) / (fhi - flo);
    if (!(tm > tlo && tm < thi)) tm = 0.5 * (tlo + thi);
    double fm;
    WL_TRY(f(tm, &fm));
    if (fm > 0) {
      tlo = tm;
      flo = fm;
      if (side == 1) fhi *= 0.5;
      side = 1;
    } else {
      thi = tm;
      fhi = fm;
      if (side == -1) flo *= 0.5;
      side = -1;
    }
  }
  const double r = 2.0 / (tlo + thi);
  g->rho_cache[mu] = r;
  *rho = r;
  return WL_OK;
}

// ------------------------------------------------------------------ operator
wl_status wl_op_create(wl_graph* g, const wl_op_desc* d, wl_op** out) {
  WL_CHECK(g && d && out, WL_EINVAL, "wl_op_create: null argument");
  *out = nullptr;
  WL_CHECK(d->mu >= 0.0 && d->mu <= 1.0, WL_EINVAL, "wl_op_create: mu must lie in [0, 1]");
  WL_CHECK(d->func == WL_F_RESOLVENT || d->func == WL_F_EXP || d->func == WL_F_LINEAR, WL_EINVAL,
           "wl_op_create: unknown func");
  WL_CHECK(d->func != WL_F_LINEAR || d->method == WL_M_AUTO || d->method == WL_M_RECURRENCE, WL_EUNSUPPORTED,
           "wl_op_create: the linear weights (standard Laplacian) are evaluated by their one-step series");
  WL_CHECK(is_finite(d->param) && d->param > 0.0, WL_EINVAL, "wl_op_create: param (alpha or beta) must be > 0");
  WL_CHECK(d->prec == WL_FP32 || d->prec == WL_FP64, WL_EINVAL, "wl_op_create: prec must be WL_FP32 or WL_FP64");
  WL_CHECK(d->krylov_dim >= 0 && d->krylov_dim <= 2000, WL_EINVAL, "wl_op_create: krylov_dim out of range");
  WL_CHECK(is_finite(d->tol) && d->tol >= 0.0, WL_EINVAL, "wl_op_create: bad tol");
  WL_CHECK(d->method >= WL_M_AUTO && d->method <= WL_M_AMG_CG, WL_EINVAL, "wl_op_create: unknown method");
  WL_CHECK(d->method != WL_M_AMG_CG || (d->func == WL_F_RESOLVENT && d->prec == WL_FP64), WL_EUNSUPPORTED,
           "wl_op_create: the multigrid-preconditioned CG solves resolvent systems in double precision");
  WL_CHECK(d->method != WL_M_ARNOLDI || d->func == WL_F_EXP, WL_EUNSUPPORTED,
           "wl_op_create: the Arnoldi method evaluates exponential weights only");
  WL_CHECK(d->method != WL_M_ARNOLDI || d->krylov_dim > 0, WL_EINVAL,
           "wl_op_create: the Arnoldi method needs an explicit krylov_dim");
  WL_CHECK(d->reorth >= 0 && d->reorth <= 2, WL_EINVAL, "wl_op_create: reorth must be 0, 1 or 2");
  int method = d->method;
  if (method == WL_M_AUTO) method = d->func == WL_F_RESOLVENT ? WL_M_LANCZOS : WL_M_RECURRENCE;
  WL_CHECK(!(method == WL_M_LANCZOS && d->func == WL_F_EXP && d->mu != 0.0), WL_EUNSUPPORTED,
           "wl_op_create: exponential weights with mu > 0 are not a function of one symmetric n x n matrix; "
           "use the recurrence");
  WL_CHECK(!(method == WL_M_RECURRENCE && d->func == WL_F_RESOLVENT && d->krylov_dim == 0), WL_EINVAL,
           "wl_op_create: the truncated resolvent series needs an explicit krylov_dim");
  DeviceGuard dg(g->ctx->device);
  double rho = 0.0;
  if (d->func == WL_F_RESOLVENT) {
    if (d->rho_hint > 0)
      rho = d->rho_hint;
    else
      WL_TRY(wl_spectral_radius(g, d->mu, 1e-10, &rho));
    WL_CHECK(d->param * rho < 1.0, WL_ERANGE,
             "wl_op_create: alpha * rho(Z_mu) = %.6g >= 1: the series does not converge", d->param * rho);
  }
  double lam_exp = 0.0;  // lambda_max(A) for exponential weights (series scaling, degree)
  if (d->func == WL_F_EXP) WL_TRY(wl_lambda_max(g, 1e-10, &lam_exp));
  int K = d->func == WL_F_LINEAR ? 1 : d->krylov_dim;
  if (method == WL_M_AMG_CG && K == 0) K = 1000;  // iteration limit
  if (K == 0) {
    const double tol = d->tol > 0 ? d->tol : 1e-12;
    if (d->func == WL_F_EXP) {
      const double lam = lam_exp;
      // smallest K with sum_{k>K} (beta lam)^k / k! <= tol * e^{beta lam}
      const double x = d->param * lam;
      double term = 1.0, tail = std::exp(x) - 1.0;
      K = 0;
      while (tail > tol * std::exp(x) && K < 2000) {
        ++K;
        term *= x / K;
        tail -= term;
      }
    } else {
      // conjugate-gradient style bound with a spectral-interval estimate of A_mu(alpha)
      double lam;
      WL_TRY(wl_lambda_max(g, 1e-10, &lam));
      const double a = d->param, mu = d->mu;
      const double top = 1.0 + a * lam + a * a * mu * g->max_deg;
      const double bot = std::max(1.0 - a * rho, 1e-6);
      const double kappa = top / bot;
      K = (int)std::ceil(0.5 * std::sqrt(kappa) * std::log(2.0 / tol)) + 2;
      K = std::min(K, 2000);
    }
  }
  auto* op = new wl_op;
  op->g = g;
  ++g->refs;
  op->d = *d;
  op->d.method = method;
  if (d->func == WL_F_LINEAR) op->d.param = 1.0;  // phi = I + A: one step of scale 1
  op->rho = rho;
  op->lam = lam_exp;
  op->K = K;
  if (method == WL_M_AMG_CG) {
    const wl_status s = amg_setup(op);
    if (s != WL_OK) {
      amg_destroy(op);
      delete op;
      graph_release(g);
      return s;
    }
  }
  *out = op;
  return WL_OK;
}

wl_status wl_op_info(const wl_op* op, int32_t* degree_or_steps, int32_t* method) {
  WL_CHECK(op, WL_EINVAL, "wl_op_info: op is null");
  if (degree_or_steps) *degree_or_steps = op->K;
  if (method) *method = op->d.method;
  return WL_OK;
}

wl_status wl_op_destroy(wl_op* op) {
  if (!op) return WL_OK;
  wl_graph* g = op->g;
  {
    DeviceGuard dg(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    amg_destroy(op);
    rk_cache_destroy(op);
    delete op;
  }
  graph_release(g);
  return WL_OK;
}

}  // extern "C"

template <typename T>
wl_status ensure_w(wl_op* op) {
  if (op->w_valid) return WL_OK;
  wl_graph* g = op->g;
  const int64_t n = g->n;
  WL_TRY(op->w.ensure(std::max<int64_t>(n, 1) * sizeof(T)));
  DevBuf& ones = op->inner_tmp;
  WL_TRY(ones.ensure(std::max<int64_t>(n, 1) * sizeof(T)));
  WL_TRY(launch_fill<T>(g->ctx, n, T(1), ones.as<T>()));
  WL_TRY(phi_apply_impl<T>(op, ones.as<T>(), op->w.as<T>(), 1, nullptr, nullptr));
  op->w_valid = true;
  return WL_OK;
}
template wl_status ensure_w<float>(wl_op*);
template wl_status ensure_w<double>(wl_op*);

extern "C" {

wl_status wl_fdeg(wl_op* op, void* d_w) {
  WL_CHECK(op, WL_EINVAL, "wl_fdeg: op is null");
  WL_CHECK(op->g->n == 0 || d_w, WL_EINVAL, "wl_fdeg: output is null");
  DeviceGuard dg(op->g->ctx->device);
  const size_t es = op->d.prec == WL_FP32 ? 4 : 8;
  if (op->d.prec == WL_FP32)
    WL_TRY(ensure_w<float>(op));
  else
    WL_TRY(ensure_w<double>(op));
  if (op->g->n > 0)
    WL_HIP(hipMemcpyAsync(d_w, op->w.p, (size_t)op->g->n * es, hipMemcpyDeviceToDevice, op->g->ctx->stream));
  return scan_output(op->g->ctx, op->d.prec, d_w, op->g->n, "wl_fdeg");
}

static wl_status check_block(wl_op* op, const void* X, const void* Y, int32_t b, const char* who) {
  WL_CHECK(op, WL_EINVAL, "%s: op is null", who);
  WL_CHECK(b >= 1 && b <= 64, WL_EINVAL, "%s: b must lie in [1, 64]", who);
  WL_CHECK(op->g->n == 0 || (X && Y), WL_EINVAL, "%s: null block", who);
  WL_CHECK(X != Y || op->g->n == 0, WL_EINVAL, "%s: X and Y must not alias", who);
  const size_t es = op->d.prec == WL_FP32 ? 4 : 8;
  WL_CHECK((reinterpret_cast<uintptr_t>(X) % es) == 0 && (reinterpret_cast<uintptr_t>(Y) % es) == 0, WL_EINVAL,
           "%s: misaligned block", who);
  return WL_OK;
}

wl_status wl_apply_phi(wl_op* op, const void* d_X, void* d_Y, int32_t b) {
  WL_TRY(check_block(op, d_X, d_Y, b, "wl_apply_phi"));
  DeviceGuard dg(op->g->ctx->device);
  if (op->d.prec == WL_FP32)
    WL_TRY(phi_apply_impl<float>(op, (const float*)d_X, (float*)d_Y, b, nullptr, nullptr));
  else
    WL_TRY(phi_apply_impl<double>(op, (const double*)d_X, (double*)d_Y, b, nullptr, nullptr));
  return scan_output(op->g->ctx, op->d.prec, d_Y, op->g->n * b, "wl_apply_phi");
}

wl_status wl_apply_L(wl_op* op, const void* d_X, void* d_Y, int32_t b) {
  WL_TRY(check_block(op, d_X, d_Y, b, "wl_apply_L"));
  DeviceGuard dg(op->g->ctx->device);
  if (op->d.prec == WL_FP32) {
    WL_TRY(ensure_w<float>(op));
    WL_TRY(phi_apply_impl<float>(op, (const float*)d_X, (float*)d_Y, b, op->w.as<float>(), (const float*)d_X));
  } else {
    WL_TRY(ensure_w<double>(op));
    WL_TRY(
        phi_apply_impl<double>(op, (const double*)d_X, (double*)d_Y, b, op->w.as<double>(), (const double*)d_X));
  }
  return scan_output(op->g->ctx, op->d.prec, d_Y, op->g->n * b, "wl_apply_L");
}

wl_status wl_markov_gap(wl_op* op, int32_t outer_dim, uint64_t seed, double* lambda2, double* lambda_min,
                        double* gap) {
  WL_CHECK(op, WL_EINVAL, "wl_markov_gap: op is null");
  WL_CHECK(outer_dim >= 2 && outer_dim <= 1000, WL_EINVAL, "wl_markov_gap: outer_dim must lie in [2, 1000]");
  DeviceGuard dg(op->g->ctx->device);
  if (op->d.prec == WL_FP32) return markov_gap_impl<float>(op, outer_dim, seed, lambda2, lambda_min, gap);
  return markov_gap_impl<double>(op, outer_dim, seed, lambda2, lambda_min, gap);
}

wl_status wl_expv(wl_op* op, const void* d_U0, int32_t b, const double* t, int32_t nt, void* const* d_Y,
                  int32_t outer_dim, double* err_est) {
  WL_CHECK(op, WL_EINVAL, "wl_expv: op is null");
  WL_CHECK(b >= 1 && b <= 64, WL_EINVAL, "wl_expv: b must lie in [1, 64]");
  WL_CHECK(nt >= 1 && t && d_Y, WL_EINVAL, "wl_expv: need nt >= 1 times and outputs");
  WL_CHECK(outer_dim >= 1 && outer_dim <= 1000, WL_EINVAL, "wl_expv: outer_dim out of range");
  WL_CHECK(op->g->n == 0 || d_U0, WL_EINVAL, "wl_expv: U0 is null");
  for (int i = 0; i < nt; ++i) {
    WL_CHECK(is_finite(t[i]) && t[i] >= 0, WL_EINVAL, "wl_expv: times must be finite and >= 0");
    WL_CHECK(op->g->n == 0 || (d_Y[i] && d_Y[i] != d_U0), WL_EINVAL, "wl_expv: bad output pointer %d", i);
  }
  if (op->g->n == 0) return WL_OK;
  DeviceGuard dg(op->g->ctx->device);
  if (op->d.prec == WL_FP32) {
    WL_TRY(ensure_w<float>(op));
    WL_TRY(expv_impl<float>(op, (const float*)d_U0, b, t, nt, (float* const*)d_Y, outer_dim, err_est));
  } else {
    WL_TRY(ensure_w<double>(op));
    WL_TRY(expv_impl<double>(op, (const double*)d_U0, b, t, nt, (double* const*)d_Y, outer_dim, err_est));
  }
  for (int i = 0; i < nt; ++i) WL_TRY(scan_output(op->g->ctx, op->d.prec, d_Y[i], op->g->n * b, "wl_expv"));
  return WL_OK;
}

wl_status wl_block_gram(wl_ctx* ctx, int32_t prec, int64_t n, int32_t nblk, int32_t bx, const void* d_X,
                        int32_t by, const void* d_Y, double* G) {
  WL_CHECK(ctx && G, WL_EINVAL, "wl_block_gram: null argument");
  WL_CHECK(prec == WL_FP32 || prec == WL_FP64, WL_EINVAL, "wl_block_gram: bad prec");
  WL_CHECK(n >= 1 && nblk >= 1 && nblk <= 4096, WL_EINVAL, "wl_block_gram: bad size");
  WL_CHECK(bx >= 1 && bx <= 64 && by >= 1 && by <= 64, WL_EINVAL, "wl_block_gram: widths must lie in [1, 64]");
  WL_CHECK(d_X && d_Y, WL_EINVAL, "wl_block_gram: null block");
  DeviceGuard dg(ctx->device);
  DevBuf d;
  const size_t cnt = (size_t)nblk * bx * by;
  WL_TRY(d.ensure(cnt * 8));
  if (prec == WL_FP32)
    WL_TRY(launch_gram<float>(ctx, n, (const float*)d_X, bx, n * bx, nblk, (const float*)d_Y, by, d.as<double>()));
  else
    WL_TRY(launch_gram<double>(ctx, n, (const double*)d_X, bx, n * bx, nblk, (const double*)d_Y, by,
                               d.as<double>()));
  WL_HIP(hipMemcpyAsync(G, d.p, cnt * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  return WL_OK;
}

wl_status wl_block_update(wl_ctx* ctx, int32_t prec, int64_t n, int32_t nblk, int32_t b, const void* d_X,
                          const double* C, const void* d_Yin, double alpha, double beta, void* d_Out, double* G) {
  WL_CHECK(ctx && C, WL_EINVAL, "wl_block_update: null argument");
  WL_CHECK(prec == WL_FP32 || prec == WL_FP64, WL_EINVAL, "wl_block_update: bad prec");
  WL_CHECK(n >= 1 && nblk >= 1 && nblk <= 4096, WL_EINVAL, "wl_block_update: bad size");
  WL_CHECK(b >= 1 && b <= 64, WL_EINVAL, "wl_block_update: b must lie in [1, 64]");
  WL_CHECK(d_X && d_Out, WL_EINVAL, "wl_block_update: null block");
  DeviceGuard dg(ctx->device);
  DevBuf dc, dg2;
  const size_t cnt = (size_t)nblk * b * b;
  WL_TRY(dc.ensure(cnt * 8));
  WL_TRY(dg2.ensure((size_t)b * b * 8));
  WL_HIP(hipMemcpyAsync(dc.p, C, cnt * 8, hipMemcpyHostToDevice, ctx->stream));
  if (prec == WL_FP32)
    WL_TRY(launch_update<float>(ctx, n, (const float*)d_X, b, n * b, nblk, dc.as<double>(), (const float*)d_Yin,
                                alpha, nullptr, beta, (float*)d_Out, b, G ? dg2.as<double>() : nullptr));
  else
    WL_TRY(launch_update<double>(ctx, n, (const double*)d_X, b, n * b, nblk, dc.as<double>(),
                                 (const double*)d_Yin, alpha, nullptr, beta, (double*)d_Out, b,
                                 G ? dg2.as<double>() : nullptr));
  if (G) WL_HIP(hipMemcpyAsync(G, dg2.p, (size_t)b * b * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  return WL_OK;
}

wl_status wl_probes(wl_ctx* ctx, int32_t prec, int32_t law, uint64_t seed, uint32_t stream, int64_t n, int32_t M,
                    void* d_out) {
  WL_CHECK(ctx, WL_EINVAL, "wl_probes: ctx is null");
  WL_CHECK(prec == WL_FP32 || prec == WL_FP64, WL_EINVAL, "wl_probes: bad prec");
  WL_CHECK(law == WL_PROBE_GAUSS || law == WL_PROBE_RADEMACHER, WL_EINVAL, "wl_probes: bad law");
  WL_CHECK(n >= 0 && M >= 1, WL_EINVAL, "wl_probes: bad size");
  WL_CHECK(n == 0 || d_out, WL_EINVAL, "wl_probes: output is null");
  DeviceGuard dg(ctx->device);
  if (prec == WL_FP32) return launch_probes<float>(ctx, law, seed, stream, n, M, (float*)d_out);
  return launch_probes<double>(ctx, law, seed, stream, n, M, (double*)d_out);
}

}  // extern "C"

// ------------------------------------------------------------------ caller workspace
// Every device buffer a call of wl_apply_phi / wl_apply_L / wl_expv touches, with its
// size, so that the call can run on one caller-provided region instead of library
// allocations: the plan lists the operator's (and context's) buffers; the scope points
// them into the region for the duration of the call and restores them afterwards.
namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct WsPlan {
  struct Item {
    DevBuf* buf;
    size_t bytes;
  };
  std::vector<Item> items;
  bool uses_w = false;
  void need(DevBuf& b, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    for (auto& it : items)
      if (it.buf == &b) {
        it.bytes = std::max(it.bytes, bytes);
        return;
      }
    items.push_back({&b, bytes});
  }
  size_t total() const {
    size_t s = 0;
    for (const auto& it : items) s += align256(it.bytes);
    return s;
  }
};

size_t elem_size(const wl_op* op) { return op->d.prec == WL_FP32 ? 4 : 8; }

// phi X on a block of width b (phi_apply_impl)
wl_status plan_phi(wl_op* op, int b, WsPlan& pl) {
  const int64_t n = op->g->n;
  if (n == 0) return WL_OK;
  const size_t s = elem_size(op), blk = (size_t)n * b * s;
  if (op->d.method == WL_M_ARNOLDI || op->d.method == WL_M_AMG_CG) {
    wl_set_error("caller workspace: Arnoldi and multigrid operators are not covered");
    return WL_EUNSUPPORTED;
  }
  if (op->d.method == WL_M_LANCZOS) {
    const int K = lanczos_steps(op, n, b);
    pl.need(op->basis, (size_t)(K + 1) * blk);
    pl.need(op->wbuf, blk);
    pl.need(op->small, SmallLayout{b, K, (size_t)b * b}.total() * sizeof(double));
    pl.need(op->coef, (size_t)K * b * b * sizeof(double));
    // fused steps take Grams of three blocks; full reorthogonalisation of up to K + 1
    const int nblk = (op->d.reorth > 1 || (int64_t)(K + 1) * b * 2 > n) ? K + 1 : 3;
    pl.need(op->g->ctx->partials, std::max(gram_partials_bound(n, op->d.prec, b, nblk),
                                           update_partials_bound(n, op->d.prec, b)));
    return WL_OK;
  }
  if (op->K >= 1) {
    pl.need(op->bufA, blk);
    pl.need(op->bufB, blk);
  }
  return WL_OK;
}

// the walk degrees, when the operator has not cached them
wl_status plan_w(wl_op* op, WsPlan& pl) {
  if (op->w_valid) return WL_OK;
  const size_t nb = (size_t)std::max<int64_t>(op->g->n, 1) * elem_size(op);
  pl.need(op->w, nb);
  pl.need(op->inner_tmp, nb);
  pl.uses_w = true;
  return plan_phi(op, 1, pl);
}

wl_status plan_call(wl_op* op, int call, int b, int outer_dim, WsPlan& pl) {
  const int64_t n = op->g->n;
  switch (call) {
    case WL_CALL_APPLY_PHI:
      return plan_phi(op, b, pl);
    case WL_CALL_APPLY_L:
      WL_TRY(plan_w(op, pl));
      return plan_phi(op, b, pl);
    case WL_CALL_EXPV: {
      WL_TRY(plan_w(op, pl));
      if (n == 0) return WL_OK;
      const int K = expv_outer_steps(outer_dim, n);
      const size_t blk = (size_t)n * b * elem_size(op);
      pl.need(op->outer_basis, (size_t)(K + 1) * blk);
      pl.need(op->outer_w, blk);
      pl.need(op->outer_small, SmallLayout{b, K, (size_t)b * b}.total() * sizeof(double));
      pl.need(op->outer_coef, (size_t)K * b * b * sizeof(double));
      pl.need(op->g->ctx->partials, std::max(gram_partials_bound(n, op->d.prec, b, K + 1),
                                             update_partials_bound(n, op->d.prec, b)));
      return plan_phi(op, b, pl);  // the inner phi products
    }
    default:
      wl_set_error("wl_workspace_size: unknown call %d", call);
      return WL_EINVAL;
  }
}

// Points the planned buffers into [base, base + total) for its lifetime; allocation is
// refused meanwhile (a missing plan entry becomes WL_EINTERNAL, never a hipMalloc) and
// kernel timing is off (it would create events).
class WsScope {
 public:
  WsScope(wl_op* op, const WsPlan& pl, void* base) : op_(op), uses_w_(pl.uses_w) {
    char* p = static_cast<char*>(base);
    for (const auto& it : pl.items) {
      saved_.push_back({it.buf, it.buf->p, it.buf->bytes, it.buf->borrowed});
      it.buf->p = p;
      it.buf->bytes = it.bytes;
      it.buf->borrowed = true;
      p += align256(it.bytes);
    }
    prof_ = op->g->ctx->profiling;
    op->g->ctx->profiling = false;
    ++wl_no_alloc;
  }
  ~WsScope() {
    for (auto it = saved_.rbegin(); it != saved_.rend(); ++it) {
      it->buf->p = it->p;
      it->buf->bytes = it->bytes;
      it->buf->borrowed = it->borrowed;
    }
    --wl_no_alloc;
    op_->g->ctx->profiling = prof_;
    if (uses_w_) op_->w_valid = false;  // the walk degrees lived in the caller's region
  }

 private:
  struct Saved {
    DevBuf* buf;
    void* p;
    size_t bytes;
    bool borrowed;
  };
  wl_op* op_;
  bool uses_w_;
  bool prof_ = false;
  std::vector<Saved> saved_;
};

wl_status ws_check(wl_op* op, int call, int b, int outer_dim, void* d_work, size_t work_bytes, WsPlan& pl,
                   const char* who) {
  WL_TRY(plan_call(op, call, b, outer_dim, pl));
  const size_t need = pl.total();
  WL_CHECK(need == 0 || d_work, WL_EINVAL, "%s: workspace is null", who);
  WL_CHECK((reinterpret_cast<uintptr_t>(d_work) & 255u) == 0, WL_EINVAL, "%s: workspace must be 256-byte aligned",
           who);
  WL_CHECK(work_bytes >= need, WL_EINVAL, "%s: workspace of %zu bytes is smaller than the %zu bytes needed", who,
           work_bytes, need);
  return WL_OK;
}

}  // namespace

// ------------------------------------------------------------------ fixed region
// wl_apply_L_noalloc runs on a region that is part of the library's code object: one
// static device array per GPU, held from module load until the process ends.  Host
// code never names the array in a kernel argument or copy (on the host its name is a
// stand-in, not a device address); the device address comes from hipGetSymbolAddress
// with the device current, once per device, at wl_ctx_create.
static __device__ __align__(256) unsigned char scratch[WL_NOALLOC_BYTES];

namespace {
std::mutex g_scratch_mu;
std::unordered_map<int, void*> g_scratch_ptr;  // device -> address of that device's copy
}  // namespace

static wl_status noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return WL_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    wl_set_error("fixed region: hipGetSymbolAddress failed on device %d: %s", device, hipGetErrorString(e));
    return WL_EDEVICE;
  }
  WL_CHECK((reinterpret_cast<uintptr_t>(ptr) & 255u) == 0, WL_EINTERNAL, "fixed region is not 256-byte aligned");
  g_scratch_ptr[device] = ptr;
  return WL_OK;
}

static void* noalloc_region(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

static wl_status phi_ws_call(wl_op* op, const void* d_X, void* d_Y, int32_t b, bool laplacian, void* d_work,
                             size_t work_bytes) {
  const char* who = laplacian ? "wl_apply_L_ws" : "wl_apply_phi_ws";
  WL_TRY(check_block(op, d_X, d_Y, b, who));
  DeviceGuard dg(op->g->ctx->device);
  WsPlan pl;
  WL_TRY(ws_check(op, laplacian ? WL_CALL_APPLY_L : WL_CALL_APPLY_PHI, b, 0, d_work, work_bytes, pl, who));
  WsScope scope(op, pl, d_work);
  return laplacian ? wl_apply_L(op, d_X, d_Y, b) : wl_apply_phi(op, d_X, d_Y, b);
}

extern "C" {

wl_status wl_workspace_size(const wl_op* op, int32_t call, int32_t b, int32_t outer_dim, size_t* bytes) {
  WL_CHECK(op && bytes, WL_EINVAL, "wl_workspace_size: null argument");
  WL_CHECK(b >= 1 && b <= 64, WL_EINVAL, "wl_workspace_size: b must lie in [1, 64]");
  WL_CHECK(call != WL_CALL_EXPV || (outer_dim >= 1 && outer_dim <= 1000), WL_EINVAL,
           "wl_workspace_size: outer_dim out of range");
  WsPlan pl;
  WL_TRY(plan_call(const_cast<wl_op*>(op), call, b, outer_dim, pl));
  *bytes = pl.total();
  return WL_OK;
}

wl_status wl_apply_phi_ws(wl_op* op, const void* d_X, void* d_Y, int32_t b, void* d_work, size_t work_bytes) {
  return phi_ws_call(op, d_X, d_Y, b, false, d_work, work_bytes);
}

wl_status wl_apply_L_ws(wl_op* op, const void* d_X, void* d_Y, int32_t b, void* d_work, size_t work_bytes) {
  return phi_ws_call(op, d_X, d_Y, b, true, d_work, work_bytes);
}

wl_status wl_apply_L_noalloc(wl_op* op, const void* d_X, void* d_Y, int32_t b) {
  WL_TRY(check_block(op, d_X, d_Y, b, "wl_apply_L_noalloc"));
  const int dev = op->g->ctx->device;
  DeviceGuard dg(dev);
  void* base = noalloc_region(dev);
  WL_CHECK(base, WL_EINTERNAL, "wl_apply_L_noalloc: fixed region of device %d not set up", dev);
  WsPlan pl;
  WL_TRY(plan_call(op, WL_CALL_APPLY_L, b, 0, pl));
  const size_t need = pl.total();
  WL_CHECK(need <= WL_NOALLOC_BYTES, WL_ERANGE,
           "wl_apply_L_noalloc: this call needs %zu bytes of workspace, above the fixed region's %zu bytes "
           "(use wl_apply_L_ws with a larger caller region)",
           need, (size_t)WL_NOALLOC_BYTES);
  WsScope scope(op, pl, base);
  return wl_apply_L(op, d_X, d_Y, b);
}

wl_status wl_expv_ws(wl_op* op, const void* d_U0, int32_t b, const double* t, int32_t nt, void* const* d_Y,
                     int32_t outer_dim, double* err_est, void* d_work, size_t work_bytes) {
  WL_CHECK(op, WL_EINVAL, "wl_expv_ws: op is null");
  WL_CHECK(b >= 1 && b <= 64, WL_EINVAL, "wl_expv_ws: b must lie in [1, 64]");
  WL_CHECK(outer_dim >= 1 && outer_dim <= 1000, WL_EINVAL, "wl_expv_ws: outer_dim out of range");
  DeviceGuard dg(op->g->ctx->device);
  WsPlan pl;
  WL_TRY(ws_check(op, WL_CALL_EXPV, b, outer_dim, d_work, work_bytes, pl, "wl_expv_ws"));
  WsScope scope(op, pl, d_work);
  return wl_expv(op, d_U0, b, t, nt, d_Y, outer_dim, err_est);
}

}  // extern "C"
