// Learned control variate for the stochastic diagonal estimator (no counterpart in
// the paper): cheap local features, exact diagonals for training, and a small MLP
// 8 -> 64 -> 64 -> 1 (tanh) trained with hand-written forward / backward / Adam kernels.
//
// Features of node i (structural quantities scaled by the operator parameter s, so one
// network serves graphs of different spectral radius):
//   x0 = log1p(s d_i)              degree
//   x1 = log1p(s^2 d_i)            = s^2 diag(A^2)_i
//   x2 = log1p(s^3 2 t_i)          = s^3 diag(A^3)_i, t_i triangles through i
//   x3 = log1p(s^2 S2_i)           S2_i = sum_{j in N(i)} d_j  (2-walk count (A^2 1)_i)
//   x4 = log1p(s mean_j d_j)       neighbour-degree moments
//   x5 = log1p(s sqrt(mean_j d_j^2))
//   x6 = log1p(s max_j d_j)
//   x7 = 2 t_i / (d_i (d_i - 1))   local clustering (0 if d_i < 2)
// Parameter vector layout: W1 (64x8 row-major), b1 (64), W2 (64x64), b2 (64), W3 (1x64), b3.
#include <cmath>
#include <cstdio>
#include <vector>

#include "wl_internal.h"

namespace {

constexpr int NIN = 8, NH = 64;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
constexpr int NPARAM = OB3 + 1;  // 4801

// triangles: for every stored edge (i, j) count |N(i) cap N(j)| by binary-searching the
// shorter list in the longer one; integer atomics keep the sum exact.
__global__ void k_triangles(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                            const int32_t* __restrict__ colidx, const int32_t* __restrict__ rowof,
                            unsigned long long* __restrict__ tri2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = rowof[e], j = colidx[e];
    int32_t a0 = rowptr[i], a1 = rowptr[i + 1], b0 = rowptr[j], b1 = rowptr[j + 1];
    if (a1 - a0 > b1 - b0) {
      int32_t t0 = a0, t1 = a1;
      a0 = b0;
      a1 = b1;
      b0 = t0;
      b1 = t1;
    }
    unsigned long long c = 0;
    for (int32_t p = a0; p < a1; ++p) {
      const int32_t v = colidx[p];
      int32_t lo = b0, hi = b1 - 1;
      while (lo <= hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t w = colidx[mid];
        if (w == v) {
          ++c;
          break;
        }
        if (w < v) lo = mid + 1; else hi = mid - 1;
      }
    }
    if (c) atomicAdd(&tri2[i], c);  // each triangle at i is seen from both of its edges at i
  }
}

__global__ void k_rowof(int64_t n, const int32_t* __restrict__ rowptr, int32_t* __restrict__ rowof) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) rowof[k] = (int32_t)i;
}

__global__ void k_features(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                           const unsigned long long* __restrict__ tri2, double s, float* __restrict__ feat) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = rowptr[i], b = rowptr[i + 1];
    const double d = b - a;
    double s1 = 0.0, s2 = 0.0, mx = 0.0;
    for (int32_t k = a; k < b; ++k) {
      const int32_t j = colidx[k];
      const double dj = rowptr[j + 1] - rowptr[j];
      s1 += dj;
      s2 += dj * dj;
      mx = dj > mx ? dj : mx;
    }
    const double t = tri2 ? 0.5 * (double)tri2[i] : 0.0;
    const double mean = d > 0 ? s1 / d : 0.0;
    const double rms = d > 0 ? sqrt(s2 / d) : 0.0;
    float* f = feat + i * NIN;
    f[0] = (float)log1p(s * d);
    f[1] = (float)log1p(s * s * d);
    f[2] = (float)log1p(s * s * s * 2.0 * t);
    f[3] = (float)log1p(s * s * s1);
    f[4] = (float)log1p(s * mean);
    f[5] = (float)log1p(s * rms);
    f[6] = (float)log1p(s * mx);
    f[7] = d >= 2 ? (float)(2.0 * t / (d * (d - 1.0))) : 0.f;
  }
}

// out[j] = Y[nodes[j0 + j], j] for the unit-vector block e_{nodes[j0 .. j0+b)}
template <typename T>
__global__ void k_unit_block(int64_t n, int b, const int32_t* __restrict__ nodes, int64_t j0, int64_t count,
                             T* __restrict__ E) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * b; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / b;
    const int c = (int)(e - r * b);
    const int64_t jj = j0 + c;
    E[e] = (jj < count && nodes[jj] == r) ? T(1) : T(0);
  }
}

template <typename T>
__global__ void k_extract_diag(int b, const int32_t* __restrict__ nodes, int64_t j0, int64_t count,
                               const T* __restrict__ Y, T* __restrict__ out) {
  const int c = threadIdx.x;
  const int64_t jj = j0 + c;
  if (c < b && jj < count) out[jj] = Y[(int64_t)nodes[jj] * b + c];
}

// ------------------------------------------------------------------ MLP
__global__ __launch_bounds__(256) void k_mlp_forward(int64_t n, const float* __restrict__ P,
                                                     const float* __restrict__ X, float* __restrict__ out) {
  __shared__ float sp[NPARAM];
  for (int e = threadIdx.x; e < NPARAM; e += blockDim.x) sp[e] = P[e];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float x[NIN], h1[NH];
#pragma unroll
    for (int c = 0; c < NIN; ++c) x[c] = X[i * NIN + c];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      float z = sp[OB1 + k];
#pragma unroll
      for (int c = 0; c < NIN; ++c) z += sp[OW1 + k * NIN + c] * x[c];
      h1[k] = tanhf(z);
    }
    float y = sp[OB3];
    for (int m = 0; m < NH; ++m) {
      float z = sp[OB2 + m];
#pragma unroll
      for (int k = 0; k < NH; ++k) z += sp[OW2 + m * NH + k] * h1[k];
      y += sp[OW3 + m] * tanhf(z);
    }
    out[i] = y;
  }
}

// Forward + backward for chunks of TB samples (one per thread); activations are staged
// in LDS (row = sample) so the cross-sample gradient sums read them back.  Per-workgroup
// partial gradients (double, fixed layout, the sum of squared residuals last) are
// reduced afterwards in a fixed order.
constexpr int TB = 128;
__global__ __launch_bounds__(TB) void k_mlp_grad(int64_t n, const float* __restrict__ P, const float* __restrict__ X,
                                                 const float* __restrict__ tgt, double inv_n,
                                                 double* __restrict__ partials) {
  __shared__ float sp[NPARAM];
  __shared__ float sA[TB][NH + 1];  // h1, later dz1
  __shared__ float sB[TB][NH + 1];  // h2, later dz2
  __shared__ float sx[TB][NIN];
  __shared__ float sdy[TB];
  __shared__ double sl[TB];
  const int t = threadIdx.x;
  for (int e = t; e < NPARAM; e += TB) sp[e] = P[e];
  double gW2[NH * NH / TB];
  double gW1[NH * NIN / TB];
  double gb1 = 0.0, gb2 = 0.0, gW3 = 0.0, gb3 = 0.0, loss = 0.0;
#pragma unroll
  for (int q = 0; q < NH * NH / TB; ++q) gW2[q] = 0.0;
#pragma unroll
  for (int q = 0; q < NH * NIN / TB; ++q) gW1[q] = 0.0;
  __syncthreads();
  const int64_t nchunks = (n + TB - 1) / TB;
  for (int64_t chk = blockIdx.x; chk < nchunks; chk += gridDim.x) {
    const int64_t i = chk * TB + t;
    const bool ok = i < n;
    // forward
    {
      float x[NIN], h1[NH];
#pragma unroll
      for (int c = 0; c < NIN; ++c) {
        x[c] = ok ? X[i * NIN + c] : 0.f;
        sx[t][c] = x[c];
      }
#pragma unroll
      for (int k = 0; k < NH; ++k) {
        float z = sp[OB1 + k];
#pragma unroll
        for (int c = 0; c < NIN; ++c) z += sp[OW1 + k * NIN + c] * x[c];
        h1[k] = tanhf(z);
        sA[t][k] = h1[k];
      }
      float y = sp[OB3];
      for (int m = 0; m < NH; ++m) {
        float z = sp[OB2 + m];
#pragma unroll
        for (int k = 0; k < NH; ++k) z += sp[OW2 + m * NH + k] * h1[k];
        const float h2 = tanhf(z);
        sB[t][m] = h2;
        y += sp[OW3 + m] * h2;
      }
      const float r = ok ? y - tgt[i] : 0.f;
      sdy[t] = (float)(2.0 * inv_n) * r;
      sl[t] = (double)r * (double)r;
    }
    __syncthreads();
    // output layer: dL/dW3[m] = sum_s dy_s h2_s[m]; dL/db3 = sum_s dy_s
    if (t < NH) {
      float a = 0.f;
      for (int s = 0; s < TB; ++s) a += sdy[s] * sB[s][t];
      gW3 += a;
    }
    if (t == 0) {
      double l = 0.0, d = 0.0;
      for (int s = 0; s < TB; ++s) {
        l += sl[s];
        d += sdy[s];
      }
      loss += l;
      gb3 += d;
    }
    __syncthreads();
    // dz2 = dy W3 (1 - h2^2), in place on the thread's own row
    {
      const float dy = sdy[t];
#pragma unroll
      for (int m = 0; m < NH; ++m) {
        const float h2 = sB[t][m];
        sB[t][m] = dy * sp[OW3 + m] * (1.f - h2 * h2);
      }
    }
    __syncthreads();
    // dL/dW2[m][k] = sum_s dz2_s[m] h1_s[k];  dL/db2[m] = sum_s dz2_s[m]
#pragma unroll
    for (int q = 0; q < NH * NH / TB; ++q) {
      const int e = t + TB * q;
      const int m = e / NH, k = e % NH;
      float acc = 0.f;
      for (int s = 0; s < TB; ++s) acc += sB[s][m] * sA[s][k];
      gW2[q] += acc;
    }
    if (t < NH) {
      float a = 0.f;
      for (int s = 0; s < TB; ++s) a += sB[s][t];
      gb2 += a;
    }
    // dh1 = W2^T dz2 for the thread's own sample
    float dz1[NH];
    {
#pragma unroll
      for (int k = 0; k < NH; ++k) dz1[k] = 0.f;
      for (int m = 0; m < NH; ++m) {
        const float d = sB[t][m];
#pragma unroll
        for (int k = 0; k < NH; ++k) dz1[k] += d * sp[OW2 + m * NH + k];
      }
#pragma unroll
      for (int k = 0; k < NH; ++k) {
        const float h1 = sA[t][k];
        dz1[k] *= 1.f - h1 * h1;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NH; ++k) sA[t][k] = dz1[k];
    __syncthreads();
    // dL/dW1[k][c] = sum_s dz1_s[k] x_s[c];  dL/db1[k] = sum_s dz1_s[k]
#pragma unroll
    for (int q = 0; q < NH * NIN / TB; ++q) {
      const int e = t + TB * q;
      const int k = e / NIN, c = e % NIN;
      float acc = 0.f;
      for (int s = 0; s < TB; ++s) acc += sA[s][k] * sx[s][c];
      gW1[q] += acc;
    }
    if (t < NH) {
      float a = 0.f;
      for (int s = 0; s < TB; ++s) a += sA[s][t];
      gb1 += a;
    }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * (NPARAM + 1);
#pragma unroll
  for (int q = 0; q < NH * NH / TB; ++q) out[OW2 + t + TB * q] = gW2[q];
#pragma unroll
  for (int q = 0; q < NH * NIN / TB; ++q) out[OW1 + t + TB * q] = gW1[q];
  if (t < NH) {
    out[OB1 + t] = gb1;
    out[OB2 + t] = gb2;
    out[OW3 + t] = gW3;
  }
  if (t == 0) {
    out[OB3] = gb3;
    out[NPARAM] = loss;
  }
}

__global__ void k_mlp_grad_finalize(int nparts, const double* __restrict__ partials, double* __restrict__ g) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= NPARAM; p += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < nparts; ++q) s += partials[(int64_t)q * (NPARAM + 1) + p];
    g[p] = s;
  }
}

__global__ void k_adam(float* __restrict__ P, const double* __restrict__ g, double* __restrict__ m,
                       double* __restrict__ v, double lr, double b1, double b2, double eps, double c1, double c2) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NPARAM; p += gridDim.x * blockDim.x) {
    const double gp = g[p];
    const double mp = b1 * m[p] + (1.0 - b1) * gp;
    const double vp = b2 * v[p] + (1.0 - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] = (float)((double)P[p] - lr * (mp / c1) / (sqrt(vp / c2) + eps));
  }
}

}  // namespace

struct wl_mlp {
  wl_ctx* ctx = nullptr;
  DevBuf params, m, v, grad, partials;
  int64_t step = 0;
};

namespace {
wl_status mlp_grad(wl_mlp* net, const float* feat, const float* tgt, int64_t n, double* loss) {
  wl_ctx* ctx = net->ctx;
  const int64_t nchunks = (n + TB - 1) / TB;
  const int grid = (int)(nchunks < 512 ? nchunks : 512);
  WL_TRY(net->partials.ensure((size_t)grid * (NPARAM + 1) * sizeof(double)));
  WL_TRY(net->grad.ensure((size_t)(NPARAM + 1) * sizeof(double)));
  hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(TB), 0, ctx->stream, n, net->params.as<float>(), feat, tgt,
                     1.0 / (double)n, net->partials.as<double>());
  WL_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_grad_finalize, dim3((NPARAM + 256) / 256), dim3(256), 0, ctx->stream, grid,
                     net->partials.as<double>(), net->grad.as<double>());
  WL_HIP(hipGetLastError());
  if (loss) {
    double l = 0.0;
    WL_HIP(hipMemcpyAsync(&l, net->grad.as<double>() + NPARAM, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    *loss = l / (double)n;
  }
  return WL_OK;
}
// Degree-3 series diagonal and the scale of the remainder at row r (the exact low-order
// part of diag phi and the size of what is left, which the network learns):
//   base  = 1 + c2m d + c3 tri2           (diag q_2 = (1 - mu) d, diag q_3 = (A^3)_rr)
//   scale = c4 max(1, d^2 + S2),  S2 = sum_{j in N(r)} d_j   (bounds the 4-walk count)
__device__ inline void surrogate_terms(int64_t r, const int32_t* __restrict__ rowptr,
                                       const int32_t* __restrict__ colidx, const unsigned long long* __restrict__ tri2,
                                       double c2m, double c3, double c4, double* base, double* scale) {
  const int32_t a = rowptr[r], e = rowptr[r + 1];
  const double d = e - a;
  double s2 = 0.0;
  for (int32_t k = a; k < e; ++k) {
    const int32_t j = colidx[k];
    s2 += (double)(rowptr[j + 1] - rowptr[j]);
  }
  *base = 1.0 + c2m * d + c3 * (double)tri2[r];
  *scale = c4 * fmax(1.0, d * d + s2);
}

template <typename T>
__global__ void k_surrogate_diag(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                 const unsigned long long* __restrict__ tri2, double c2m, double c3, double c4,
                                 T* __restrict__ base, T* __restrict__ scale) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double bs, sc;
    surrogate_terms(r, rowptr, colidx, tri2, c2m, c3, c4, &bs, &sc);
    if (base) base[r] = (T)bs;
    if (scale) scale[r] = (T)sc;
  }
}

// out[j] = (d[j] - base(nodes[j])) / scale(nodes[j]) in place (d: diag phi at the nodes)
template <typename T>
__global__ void k_surrogate_target(int64_t count, const int32_t* __restrict__ nodes,
                                   const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                   const unsigned long long* __restrict__ tri2, double c2m, double c3, double c4,
                                   T* __restrict__ d) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += (int64_t)gridDim.x * blockDim.x) {
    double bs, sc;
    surrogate_terms(nodes[j], rowptr, colidx, tri2, c2m, c3, c4, &bs, &sc);
    d[j] = (T)(((double)d[j] - bs) / sc);
  }
}

__global__ void k_affine(int64_t n, const float* __restrict__ base, const float* __restrict__ scale,
                         float* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (base ? base[i] : 0.f) + (scale ? scale[i] : 1.f) * y[i];
}

// c_2 (1 - mu), c_3, c_4 of the operator's weights
void surrogate_coeffs(const wl_op* op, double* c2m, double* c3, double* c4) {
  const double p = op->d.param;
  const bool ex = op->d.func == WL_F_EXP;
  if (op->d.func == WL_F_LINEAR) {  // c_k = 0 for k >= 2
    *c2m = *c3 = *c4 = 0.0;
    return;
  }
  *c2m = (ex ? p * p / 2.0 : p * p) * (1.0 - op->d.mu);
  *c3 = ex ? p * p * p / 6.0 : p * p * p;
  *c4 = ex ? p * p * p * p / 24.0 : p * p * p * p;
}

}  // namespace

wl_status graph_tri2(wl_graph* g, const unsigned long long** out) {
  hipStream_t st = g->ctx->stream;
  if (!g->tri2_valid) {
    WL_TRY(g->tri2.ensure((size_t)std::max<int64_t>(g->n, 1) * 8));
    if (g->n > 0) WL_HIP(hipMemsetAsync(g->tri2.p, 0, (size_t)g->n * 8, st));
    if (g->nnz > 0) {
      DevBuf rowof;
      WL_TRY(rowof.ensure((size_t)g->nnz * 4));
      const int gb = (int)std::min<int64_t>(8192, (g->n + 255) / 256);
      hipLaunchKernelGGL(k_rowof, dim3(gb), dim3(256), 0, st, g->n, g->rowptr, rowof.as<int32_t>());
      WL_HIP(hipGetLastError());
      const int ge = (int)std::min<int64_t>(65536, (g->nnz + 255) / 256);
      hipLaunchKernelGGL(k_triangles, dim3(ge), dim3(256), 0, st, g->n, g->nnz, g->rowptr, g->colidx,
                         rowof.as<int32_t>(), g->tri2.as<unsigned long long>());
      WL_HIP(hipGetLastError());
      // rowof is released (after a device synchronisation) when it leaves scope
    }
    g->tri2_valid = true;
  }
  *out = g->tri2.as<unsigned long long>();
  return WL_OK;
}

extern "C" {

wl_status wl_features(wl_graph* g, double scale, void* d_feat) {
  WL_CHECK(g, WL_EINVAL, "wl_features: graph is null");
  WL_CHECK(std::isfinite(scale) && scale > 0, WL_EINVAL, "wl_features: scale must be > 0");
  WL_CHECK(g->n == 0 || d_feat, WL_EINVAL, "wl_features: output is null");
  if (g->n == 0) return WL_OK;
  (void)hipSetDevice(g->ctx->device);
  hipStream_t st = g->ctx->stream;
  const unsigned long long* tri = nullptr;
  WL_TRY(graph_tri2(g, &tri));
  const int gb = (int)std::min<int64_t>(8192, (g->n + 255) / 256);
  hipLaunchKernelGGL(k_features, dim3(gb), dim3(256), 0, st, g->n, g->rowptr, g->colidx,
                     tri, scale, (float*)d_feat);
  WL_HIP(hipGetLastError());
  WL_HIP(hipStreamSynchronize(st));
  return WL_OK;
}

wl_status wl_diag_exact(wl_op* op, const int32_t* d_nodes, int64_t count, int32_t width, void* d_out) {
  WL_CHECK(op, WL_EINVAL, "wl_diag_exact: op is null");
  WL_CHECK(count >= 0 && (count == 0 || (d_nodes && d_out)), WL_EINVAL, "wl_diag_exact: bad node list");
  WL_CHECK(width >= 1 && width <= 64, WL_EINVAL, "wl_diag_exact: width must lie in [1, 64]");
  if (count == 0) return WL_OK;
  wl_graph* g = op->g;
  (void)hipSetDevice(g->ctx->device);
  const int64_t n = g->n;
  const size_t es = op->d.prec == WL_FP32 ? 4 : 8;
  DevBuf E, Y;
  WL_TRY(E.ensure((size_t)n * width * es));
  WL_TRY(Y.ensure((size_t)n * width * es));
  hipStream_t st = g->ctx->stream;
  const int gb = (int)std::min<int64_t>(8192, (n * width + 255) / 256);
  for (int64_t j0 = 0; j0 < count; j0 += width) {
    if (op->d.prec == WL_FP32) {
      hipLaunchKernelGGL((k_unit_block<float>), dim3(gb), dim3(256), 0, st, n, width, d_nodes, j0, count,
                         E.as<float>());
      WL_HIP(hipGetLastError());
      WL_TRY(wl_apply_phi(op, E.p, Y.p, width));
      hipLaunchKernelGGL((k_extract_diag<float>), dim3(1), dim3(64), 0, st, width, d_nodes, j0, count,
                         Y.as<float>(), (float*)d_out);
    } else {
      hipLaunchKernelGGL((k_unit_block<double>), dim3(gb), dim3(256), 0, st, n, width, d_nodes, j0, count,
                         E.as<double>());
      WL_HIP(hipGetLastError());
      WL_TRY(wl_apply_phi(op, E.p, Y.p, width));
      hipLaunchKernelGGL((k_extract_diag<double>), dim3(1), dim3(64), 0, st, width, d_nodes, j0, count,
                         Y.as<double>(), (double*)d_out);
    }
    WL_HIP(hipGetLastError());
  }
  WL_HIP(hipStreamSynchronize(st));
  return WL_OK;
}

wl_status wl_surrogate_diag(wl_op* op, void* d_base, void* d_scale) {
  WL_CHECK(op, WL_EINVAL, "wl_surrogate_diag: op is null");
  wl_graph* g = op->g;
  WL_CHECK(g->n == 0 || d_base || d_scale, WL_EINVAL, "wl_surrogate_diag: no output");
  if (g->n == 0) return WL_OK;
  (void)hipSetDevice(g->ctx->device);
  const unsigned long long* tri = nullptr;
  WL_TRY(graph_tri2(g, &tri));
  double c2m, c3, c4;
  surrogate_coeffs(op, &c2m, &c3, &c4);
  const int gb = (int)std::min<int64_t>(8192, (g->n + 255) / 256);
  if (op->d.prec == WL_FP32)
    hipLaunchKernelGGL(k_surrogate_diag<float>, dim3(gb), dim3(256), 0, g->ctx->stream, g->n, g->rowptr, g->colidx,
                       tri, c2m, c3, c4, (float*)d_base, (float*)d_scale);
  else
    hipLaunchKernelGGL(k_surrogate_diag<double>, dim3(gb), dim3(256), 0, g->ctx->stream, g->n, g->rowptr,
                       g->colidx, tri, c2m, c3, c4, (double*)d_base, (double*)d_scale);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status wl_surrogate_target(wl_op* op, const int32_t* d_nodes, int64_t count, int32_t width, void* d_out) {
  WL_TRY(wl_diag_exact(op, d_nodes, count, width, d_out));
  if (count == 0) return WL_OK;
  wl_graph* g = op->g;
  const unsigned long long* tri = nullptr;
  WL_TRY(graph_tri2(g, &tri));
  double c2m, c3, c4;
  surrogate_coeffs(op, &c2m, &c3, &c4);
  const int gb = (int)std::min<int64_t>(8192, (count + 255) / 256);
  if (op->d.prec == WL_FP32)
    hipLaunchKernelGGL(k_surrogate_target<float>, dim3(gb), dim3(256), 0, g->ctx->stream, count, d_nodes,
                       g->rowptr, g->colidx, tri, c2m, c3, c4, (float*)d_out);
  else
    hipLaunchKernelGGL(k_surrogate_target<double>, dim3(gb), dim3(256), 0, g->ctx->stream, count, d_nodes,
                       g->rowptr, g->colidx, tri, c2m, c3, c4, (double*)d_out);
  WL_HIP(hipGetLastError());
  WL_HIP(hipStreamSynchronize(g->ctx->stream));
  return WL_OK;
}

wl_status wl_mlp_predict(wl_mlp* net, const void* d_feat, int64_t n, const void* d_base, const void* d_scale,
                         void* d_out) {
  WL_TRY(wl_mlp_forward(net, d_feat, n, d_out));
  if (n == 0) return WL_OK;
  const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_affine, dim3(grid), dim3(256), 0, net->ctx->stream, n, (const float*)d_base,
                     (const float*)d_scale, (float*)d_out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status wl_mlp_create(wl_ctx* ctx, const float* h_params, wl_mlp** out) {
  WL_CHECK(ctx && out, WL_EINVAL, "wl_mlp_create: null argument");
  (void)hipSetDevice(ctx->device);
  auto* net = new wl_mlp;
  net->ctx = ctx;
  std::vector<float> init(NPARAM, 0.f);
  if (h_params) init.assign(h_params, h_params + NPARAM);
  std::vector<double> zeros(NPARAM, 0.0);
  wl_status s = net->params.ensure(NPARAM * sizeof(float));
  if (s == WL_OK) s = net->m.ensure(NPARAM * sizeof(double));
  if (s == WL_OK) s = net->v.ensure(NPARAM * sizeof(double));
  if (s != WL_OK) {
    delete net;
    return s;
  }
  if (hipMemcpy(net->params.p, init.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->m.p, zeros.data(), NPARAM * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->v.p, zeros.data(), NPARAM * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    delete net;
    wl_set_error("wl_mlp_create: upload failed");
    return WL_EDEVICE;
  }
  ++ctx->refs;
  *out = net;
  return WL_OK;
}

wl_status wl_mlp_destroy(wl_mlp* net) {
  if (!net) return WL_OK;
  wl_ctx* ctx = net->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete net;
  ctx_release(ctx);
  return WL_OK;
}

int32_t wl_mlp_num_params(void) { return NPARAM; }

wl_status wl_mlp_get_params(const wl_mlp* net, float* h_params) {
  WL_CHECK(net && h_params, WL_EINVAL, "wl_mlp_get_params: null argument");
  (void)hipSetDevice(net->ctx->device);
  WL_HIP(hipStreamSynchronize(net->ctx->stream));
  WL_HIP(hipMemcpy(h_params, net->params.p, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  return WL_OK;
}

wl_status wl_mlp_forward(wl_mlp* net, const void* d_feat, int64_t n, void* d_out) {
  WL_CHECK(net, WL_EINVAL, "wl_mlp_forward: net is null");
  WL_CHECK(n >= 0 && (n == 0 || (d_feat && d_out)), WL_EINVAL, "wl_mlp_forward: bad arguments");
  if (n == 0) return WL_OK;
  (void)hipSetDevice(net->ctx->device);
  const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, net->ctx->stream, n, net->params.as<float>(),
                     (const float*)d_feat, (float*)d_out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status wl_mlp_loss_grad(wl_mlp* net, const void* d_feat, const void* d_target, int64_t n, double* loss,
                           double* h_grad) {
  WL_CHECK(net && d_feat && d_target && n >= 1, WL_EINVAL, "wl_mlp_loss_grad: bad arguments");
  (void)hipSetDevice(net->ctx->device);
  WL_TRY(mlp_grad(net, (const float*)d_feat, (const float*)d_target, n, loss));
  if (h_grad) {
    WL_HIP(hipMemcpy(h_grad, net->grad.p, NPARAM * sizeof(double), hipMemcpyDeviceToHost));
  }
  return WL_OK;
}

wl_status wl_mlp_train_step(wl_mlp* net, const void* d_feat, const void* d_target, int64_t n, double lr,
                            double* loss) {
  WL_CHECK(net && d_feat && d_target && n >= 1, WL_EINVAL, "wl_mlp_train_step: bad arguments");
  WL_CHECK(std::isfinite(lr) && lr > 0, WL_EINVAL, "wl_mlp_train_step: lr must be > 0");
  (void)hipSetDevice(net->ctx->device);
  WL_TRY(mlp_grad(net, (const float*)d_feat, (const float*)d_target, n, loss));
  net->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 - std::pow(b1, (double)net->step), c2 = 1.0 - std::pow(b2, (double)net->step);
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, net->ctx->stream, net->params.as<float>(),
                     net->grad.as<double>(), net->m.as<double>(), net->v.as<double>(), lr, b1, b2, 1e-8, c1, c2);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status wl_mlp_save(const wl_mlp* net, const char* path) {
  WL_CHECK(net && path, WL_EINVAL, "wl_mlp_save: null argument");
  std::vector<float> p(NPARAM);
  WL_TRY(wl_mlp_get_params(net, p.data()));
  FILE* f = std::fopen(path, "wb");
  WL_CHECK(f, WL_EINVAL, "wl_mlp_save: cannot open %s", path);
  const char magic[8] = {'W', 'L', 'M', 'L', 'P', '0', '0', '1'};
  const int32_t np = NPARAM;
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 &&
            std::fwrite(p.data(), 4, NPARAM, f) == (size_t)NPARAM;
  std::fclose(f);
  WL_CHECK(ok, WL_EINVAL, "wl_mlp_save: write failed");
  return WL_OK;
}

wl_status wl_mlp_load(wl_ctx* ctx, const char* path, wl_mlp** out) {
  WL_CHECK(ctx && path && out, WL_EINVAL, "wl_mlp_load: null argument");
  FILE* f = std::fopen(path, "rb");
  WL_CHECK(f, WL_EINVAL, "wl_mlp_load: cannot open %s", path);
  char magic[8];
  int32_t np = 0;
  std::vector<float> p(NPARAM);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::fread(&np, 4, 1, f) == 1 && np == NPARAM &&
            std::fread(p.data(), 4, NPARAM, f) == (size_t)NPARAM;
  std::fclose(f);
  WL_CHECK(ok && std::string(magic, 8) == "WLMLP001", WL_EINVAL, "wl_mlp_load: %s is not a saved network", path);
  return wl_mlp_create(ctx, p.data(), out);
}

}  // extern "C"
