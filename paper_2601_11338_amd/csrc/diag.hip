// Machine ceilings the sparse products are measured against (diagnostics, not part of
// the method): the rate at which a GPU can gather whole rows of a table at random, the
// access pattern of every neighbour gather of a sparse product whose block does not
// fit in one XCD's L2.
#include "wl_internal.h"

namespace {

// Groups of LPN lanes gather row idx[e] (16 LPN bytes, one 16-byte vector per lane) of
// a table of `rows` rows for e < count, U rows per group in flight; each lane writes its
// running sum once (so the loads cannot be dropped).  Indices outside the table are
// skipped.
template <int LPN, int U>
__global__ __launch_bounds__(256) void k_gather_probe(const float4* __restrict__ table, int64_t rows,
                                                      const int32_t* __restrict__ idx, int64_t count,
                                                      float4* __restrict__ out) {
  const int64_t grp = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPN;
  const int v = threadIdx.x % LPN;
  const int64_t ngroups = (int64_t)gridDim.x * 256 / LPN;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t e0 = grp * U; e0 < count; e0 += ngroups * U) {
    int64_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      j[u] = e0 + u < count ? (int64_t)idx[e0 + u] : -1;
      if (j[u] >= rows) j[u] = -1;
    }
    float4 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = j[u] >= 0 ? table[j[u] * LPN + v] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc.x += x[u].x;
      acc.y += x[u].y;
      acc.z += x[u].z;
      acc.w += x[u].w;
    }
  }
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

template <int LPN>
void launch_probe(wl_ctx* ctx, int blocks, const float4* t, int64_t rows, const int32_t* idx, int64_t count,
                  float4* out) {
  hipLaunchKernelGGL((k_gather_probe<LPN, 8>), dim3(blocks), dim3(256), 0, ctx->stream, t, rows, idx, count, out);
}

}  // namespace

extern "C" wl_status wl_gather_probe(wl_ctx* ctx, const void* d_table, int64_t rows, int32_t row_bytes,
                                     const int32_t* d_idx, int64_t count, void* d_out, int32_t blocks, int32_t reps,
                                     double* ms) {
  WL_CHECK(ctx && d_table && d_idx && d_out && ms, WL_EINVAL, "wl_gather_probe: null argument");
  WL_CHECK(rows >= 1 && count >= 1 && blocks >= 1 && blocks <= 1 << 20 && reps >= 1, WL_EINVAL,
           "wl_gather_probe: sizes out of range");
  const int lpn = row_bytes / 16;
  WL_CHECK(row_bytes % 16 == 0 && (lpn == 1 || lpn == 2 || lpn == 4 || lpn == 8 || lpn == 16 || lpn == 32),
           WL_EINVAL, "wl_gather_probe: row_bytes must be 16 times 1, 2, 4, 8, 16 or 32");
  WL_CHECK(((reinterpret_cast<uintptr_t>(d_table) | reinterpret_cast<uintptr_t>(d_out)) & 15u) == 0, WL_EINVAL,
           "wl_gather_probe: table and out must be 16-byte aligned");
  DeviceGuard dg(ctx->device);
  const float4* t = static_cast<const float4*>(d_table);
  float4* out = static_cast<float4*>(d_out);
  auto run = [&]() {
    switch (lpn) {
      case 1: launch_probe<1>(ctx, blocks, t, rows, d_idx, count, out); break;
      case 2: launch_probe<2>(ctx, blocks, t, rows, d_idx, count, out); break;
      case 4: launch_probe<4>(ctx, blocks, t, rows, d_idx, count, out); break;
      case 8: launch_probe<8>(ctx, blocks, t, rows, d_idx, count, out); break;
      case 16: launch_probe<16>(ctx, blocks, t, rows, d_idx, count, out); break;
      default: launch_probe<32>(ctx, blocks, t, rows, d_idx, count, out); break;
    }
  };
  run();  // warm
  WL_HIP(hipGetLastError());
  hipEvent_t a, b;
  WL_HIP(hipEventCreate(&a));
  WL_HIP(hipEventCreate(&b));
  (void)hipEventRecord(a, ctx->stream);
  for (int r = 0; r < reps; ++r) run();
  (void)hipEventRecord(b, ctx->stream);
  hipError_t e = hipEventSynchronize(b);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  WL_CHECK(e == hipSuccess, WL_EDEVICE, "wl_gather_probe: %s", hipGetErrorString(e));
  *ms = (double)f / reps;
  return WL_OK;
}
