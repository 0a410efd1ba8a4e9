// Many graphs in one launch per Krylov step.
//
// The graphs of a batch are concatenated into one block-diagonal CSR whose per-graph
// row ranges are padded to multiples of 64 rows (padding rows have no edges), so
//  * every sparse product of the recurrence is one launch over all graphs, with the
//    per-graph coefficients of eq. qrec / the weights c_k read from a table indexed
//    by the row's graph id (graphs whose series is already converged skip their rows);
//  * every 16-row chunk belongs to one graph, so Gram products reduce per graph over
//    fixed "units" of rows (deterministic) and block updates read the coefficient
//    matrices of the row's graph;
//  * the small dense work (projection coefficients, Cholesky, exp(-t T) E_1 R_0) runs
//    one workgroup per graph.
// Diffusion per graph is exp(-t_g L_g) U0_g by block Lanczos on the walk Laplacian
// (inner phi products by the truncated series, eq. diffusion_on_G_with_downweighted_walk),
// and the average return probability p_hat(t_g) (eq. average_return_probabilities) is
// the leave-one-out Nystrom trace of Alg. 1 computed from the projected quantities alone:
// with Omega = V_0 R_0 and Y = V F, Omega^T Y = R_0^T F_0 and Y^T Y = F^T F.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "wl_internal.h"

namespace {

constexpr int UNIT_ROWS = 2048;  // rows per reduction unit (multiple of 16)
typedef double v4d __attribute__((ext_vector_type(4)));

// Segmented Gram: for every unit u (rows [us[u], us[u+1]) of one graph, a multiple of
// 16), partial[k][u] = X_k[rows]^T Y[rows] for b <= 16 columns, on the matrix cores
// (FP64 accumulation, the operand layout of the single-graph Gram).
template <int NB>
__global__ __launch_bounds__(256) void k_gram_seg(const int64_t* __restrict__ us, int nunits,
                                                  const float* __restrict__ X, int64_t sX, int nblk,
                                                  const float* __restrict__ Y, int b,
                                                  double* __restrict__ partials) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rsub = lane >> 4, c = lane & 15;
  const int kb0 = blockIdx.y * NB;
  const int nb = (nblk - kb0) < NB ? (nblk - kb0) : NB;
  const bool cok = c < b;
  for (int u = blockIdx.x * 4 + wave; u < nunits; u += gridDim.x * 4) {
    v4d acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
    const int64_t r0 = us[u], r1 = us[u + 1];
    const int cc = cok ? c : 0;  // lanes past the block width read column 0 and use zero
    for (int64_t r = r0; r < r1; r += 16) {
      // every operand of the 16 rows is requested before the first product (a branch
      // around each load would wait for it)
      float yv[4], xv[NB][4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int64_t row = r + 4 * m + rsub;
        yv[m] = Y[row * b + cc];
#pragma unroll
        for (int q = 0; q < NB; ++q) xv[q][m] = X[(int64_t)(kb0 + min(q, nb - 1)) * sX + row * b + cc];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double yb = cok ? (double)yv[m] : 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const double xa = (cok && q < nb) ? (double)xv[q][m] : 0.0;
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, yb, acc[q], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (q >= nb) break;
      double* out = partials + ((int64_t)(kb0 + q) * nunits + u) * 256;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(4 * v + rsub) * 16 + c] = acc[q][v];
    }
  }
}

// out_g[(k b + i) b + j] = sum_{u in graph g} partial[k][u][i 16 + j]  (fixed order);
// out_g = out + g * gs.
__global__ __launch_bounds__(256) void k_gram_seg_finalize(const double* __restrict__ partials, int nunits,
                                                           const int* __restrict__ gu0, int b,
                                                           double* __restrict__ out, int64_t gs) {
  const int g = blockIdx.z, k = blockIdx.y;
  const int t = threadIdx.x;
  const int el = t % 16, p = t / 16;  // 16 entries per block, 16 phases
  const int e = blockIdx.x * 16 + el;
  const int u0 = gu0[g], u1 = gu0[g + 1];
  __shared__ double s[256];
  double v = 0.0;
  if (e < 256) {
    const double* src = partials + (int64_t)k * nunits * 256 + e;
    for (int u = u0 + p; u < u1; u += 16) v += src[(int64_t)u * 256];
  }
  s[t] = v;
  __syncthreads();
  for (int h = 8; h > 0; h >>= 1) {
    if (p < h) s[t] += s[t + h * 16];
    __syncthreads();
  }
  if (p == 0 && e < 256) {
    const int i = e / 16, j = e % 16;
    if (i < b && j < b) out[(int64_t)g * gs + ((int64_t)k * b + i) * b + j] = s[t];
  }
}

// Out[r] = (wv ? wv[r] : alpha) Yin[r] + beta sum_k X_k[r] C_{g(r)}[k]   (b <= B <= 16),
// C_g = C + g * cgs, (nblk b) x b row-major double.  One row per thread; a workgroup's
// 256 consecutive rows nearly always belong to one graph (graphs span >= 64 aligned
// rows), whose coefficients are staged in LDS as float once per graph change (rows of
// another graph read theirs from memory).  Rows of exactly B floats load as float4.
template <int B>
__global__ __launch_bounds__(256) void k_update_seg(int64_t N, const float* X, int64_t sX, int nblk, int b,
                                                    const double* __restrict__ C, int64_t cgs,
                                                    const int32_t* __restrict__ gid, const float* Yin, double alpha,
                                                    const float* __restrict__ wv, double beta, float* Out) {
  extern __shared__ float sCg[];  // nblk * b * b
  const int cb = nblk * b * b;
  const bool vec = b == B;
  int staged = -1;
  for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x; r0 < N; r0 += (int64_t)gridDim.x * blockDim.x) {
    const int g0 = gid[r0];  // the same for the whole workgroup
    if (g0 != staged) {
      __syncthreads();
      const double* Cg = C + (int64_t)g0 * cgs;
      for (int e = threadIdx.x; e < cb; e += blockDim.x) sCg[e] = (float)Cg[e];
      __syncthreads();
      staged = g0;
    }
    const int64_t r = r0 + threadIdx.x;
    if (r >= N) continue;
    const int gr = gid[r];
    const double* Cglob = C + (int64_t)gr * cgs;
    float acc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = 0.f;
    for (int k = 0; k < nblk; ++k) {
      const float* xr = X + (int64_t)k * sX + r * b;
      float xv[B];
      if (vec) {
#pragma unroll
        for (int q = 0; q < B / 4; ++q) {
          const float4 v = reinterpret_cast<const float4*>(xr)[q];
          xv[4 * q] = v.x;
          xv[4 * q + 1] = v.y;
          xv[4 * q + 2] = v.z;
          xv[4 * q + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int i = 0; i < B; ++i) xv[i] = i < b ? xr[i] : 0.f;
      }
      if (gr == g0) {
        const float* Ck = sCg + k * b * b;
#pragma unroll
        for (int i = 0; i < B; ++i) {
          if (i >= b) break;
#pragma unroll
          for (int j = 0; j < B; ++j)
            if (j < b) acc[j] += xv[i] * Ck[i * b + j];
        }
      } else {
        const double* Ck = Cglob + (int64_t)k * b * b;
        for (int i = 0; i < b; ++i)
#pragma unroll
          for (int j = 0; j < B; ++j)
            if (j < b) acc[j] += xv[i] * (float)Ck[i * b + j];
      }
    }
    const float sc = wv ? wv[r] : (float)alpha;
    float* o = Out + r * b;
    const float* y = Yin ? Yin + r * b : nullptr;
    if (vec) {
#pragma unroll
      for (int q = 0; q < B / 4; ++q) {
        float4 v;
        const float4 yy = y ? reinterpret_cast<const float4*>(y)[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        v.x = (float)beta * acc[4 * q] + sc * yy.x;
        v.y = (float)beta * acc[4 * q + 1] + sc * yy.y;
        v.z = (float)beta * acc[4 * q + 2] + sc * yy.z;
        v.w = (float)beta * acc[4 * q + 3] + sc * yy.w;
        reinterpret_cast<float4*>(o)[q] = v;
      }
    } else {
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (j < b) o[j] = (float)beta * acc[j] + (y ? sc * y[j] : 0.f);
    }
  }
}

__global__ void k_dcopy_batched(int count, const double* __restrict__ x, double* __restrict__ y, int64_t gs) {
  const int64_t go = (int64_t)blockIdx.x * gs;
  for (int e = threadIdx.x; e < count; e += blockDim.x) y[go + e] = x[go + e];
}

// Graphs whose Krylov space is exhausted at step j (kcap[g] == j + 1 blocks span their
// whole space): zero the coupling B_j and the inverse Cholesky factor of the second
// pass, so V_{j+1} = 0 and every later block of that graph stays zero (its projected
// matrix decouples exactly instead of continuing on rounding noise).
__global__ void k_cap_blocks(int ng, const int32_t* __restrict__ kcap, int j, double* __restrict__ S, int64_t gs,
                             int64_t offRi, int64_t offB, int bb) {
  const int g = blockIdx.x;
  if (g >= ng || kcap[g] != j + 1) return;
  double* Sg = S + (int64_t)g * gs;
  for (int e = threadIdx.x; e < bb; e += blockDim.x) {
    Sg[offRi + e] = 0.0;
    Sg[offB + e] = 0.0;
  }
}

__global__ void k_dtranspose_batched(int b, const double* __restrict__ x, double* __restrict__ y, int64_t gs) {
  const int64_t go = (int64_t)blockIdx.x * gs;
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) y[go + (e % b) * b + e / b] = x[go + e];
}

// F_g = exp(-t_g T_g) E_1 R0_g for the block tridiagonal T_g (K blocks of b x b: A_j at
// S_g + offA + j bb, T_{j+1,j} = B_j at S_g + offB + j bb), one workgroup per graph, FP64.
// Sub-stepped Taylor series: s = ceil(t ||T||_inf) steps of length h = t / s, each
// sum_i (-h T)^i V / i! until the term is negligible (h ||T|| <= 1, so <= 30 terms).
constexpr int EXP_MAXM = 512;  // K b
__global__ __launch_bounds__(256) void k_expT_batched(int K, int b, const double* __restrict__ S, int64_t gs,
                                                      int64_t offA, int64_t offB, int64_t offR0,
                                                      const double* __restrict__ tvals, double* __restrict__ F,
                                                      int64_t fgs) {
  extern __shared__ double sh[];
  const int g = blockIdx.x;
  const int bb = b * b, m = K * b, mb = m * b;
  double* sA = sh;                 // K bb
  double* sB = sA + (size_t)K * bb;  // K bb
  double* sV = sB + (size_t)K * bb;  // m b   current vector
  double* sT = sV + mb;            // m b   current Taylor term
  double* sU = sT + mb;            // m b   scratch
  __shared__ double red[256];
  __shared__ double snorm;
  const double* Sg = S + (int64_t)g * gs;
  const int t = threadIdx.x;
  for (int e = t; e < K * bb; e += 256) {
    sA[e] = Sg[offA + e];
    sB[e] = Sg[offB + e];
  }
  for (int e = t; e < mb; e += 256) {
    const int r = e / b, c = e % b;
    sV[e] = r < b ? Sg[offR0 + r * b + c] : 0.0;
  }
  __syncthreads();
  // ||T||_inf
  double mx = 0.0;
  for (int r = t; r < m; r += 256) {
    const int j = r / b, i = r % b;
    double s = 0.0;
    for (int c = 0; c < b; ++c) {
      s += fabs(sA[j * bb + i * b + c]);
      if (j > 0) s += fabs(sB[(j - 1) * bb + i * b + c]);      // T_{j, j-1} = B_{j-1}
      if (j + 1 < K) s += fabs(sB[j * bb + c * b + i]);         // T_{j, j+1} = B_j^T
    }
    mx = fmax(mx, s);
  }
  red[t] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] = fmax(red[t], red[t + h]);
    __syncthreads();
  }
  if (t == 0) snorm = red[0];
  __syncthreads();
  const double tv = tvals[g];
  const int steps = (int)fmin(1e6, fmax(1.0, ceil(tv * snorm)));
  const double hstep = tv / steps;
  for (int st = 0; st < steps; ++st) {
    // term = V; sum into V itself: V_new = sum_i term_i
    for (int e = t; e < mb; e += 256) sT[e] = sV[e];
    __syncthreads();
    for (int i = 1; i <= 40; ++i) {
      // U = T * term
      for (int e = t; e < mb; e += 256) {
        const int r = e / b, c = e % b;
        const int j = r / b, ii = r % b;
        double s = 0.0;
        for (int k = 0; k < b; ++k) {
          s += sA[j * bb + ii * b + k] * sT[(j * b + k) * b + c];
          if (j > 0) s += sB[(j - 1) * bb + ii * b + k] * sT[((j - 1) * b + k) * b + c];
          if (j + 1 < K) s += sB[j * bb + k * b + ii] * sT[((j + 1) * b + k) * b + c];
        }
        sU[e] = s;
      }
      __syncthreads();
      double tn = 0.0, vn = 0.0;
      const double f = -hstep / i;
      for (int e = t; e < mb; e += 256) {
        const double v = f * sU[e];
        sT[e] = v;
        sV[e] += v;
        tn = fmax(tn, fabs(v));
        vn = fmax(vn, fabs(sV[e]));
      }
      red[t] = tn;
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] = fmax(red[t], red[t + h]);
        __syncthreads();
      }
      const double tmax = red[0];
      __syncthreads();
      red[t] = vn;
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] = fmax(red[t], red[t + h]);
        __syncthreads();
      }
      const double vmax = red[0];
      __syncthreads();
      if (tmax <= 1e-17 * vmax) break;
    }
  }
  double* Fg = F + (int64_t)g * fgs;
  for (int e = t; e < mb; e += 256) Fg[e] = sV[e];
}

struct Layout {  // small matrices of one graph (doubles), as in the single-graph driver
  int b, K;
  int64_t bb;
  int64_t A(int j) const { return (int64_t)j * bb; }
  int64_t B(int j) const { return (int64_t)(K + j) * bb; }
  int64_t R0() const { return (int64_t)(2 * K) * bb; }
  int64_t G() const { return (int64_t)(2 * K + 1) * bb; }
  int64_t R1() const { return (int64_t)(2 * K + 2) * bb; }
  int64_t Ri1() const { return (int64_t)(2 * K + 3) * bb; }
  int64_t R2() const { return (int64_t)(2 * K + 4) * bb; }
  int64_t Ri2() const { return (int64_t)(2 * K + 5) * bb; }
  int64_t Cc() const { return (int64_t)(2 * K + 6) * bb; }
  int64_t P() const { return (int64_t)(2 * K + 9) * bb; }   // 3 blocks
  int64_t Bt() const { return (int64_t)(2 * K + 12) * bb; }
  int64_t Ref() const { return (int64_t)(2 * K + 13) * bb; }  // one double: reference scale
  int64_t total() const { return (int64_t)(2 * K + 14) * bb; }
};

}  // namespace

// Scratch of one batched evaluation: recurrence buffers, Krylov basis, small matrices,
// Gram partials, times and per-graph step caps.  A captured graph owns its own.
struct BatchWork {
  DevBuf bufA, bufB, basis, S, F, partials, tvals, kcap;
  std::vector<char> cap_at;  // cap_at[j]: some graph's Krylov space ends at block j + 1
};

struct wl_batch {
  wl_ctx* ctx = nullptr;
  int ng = 0;
  std::vector<int64_t> n, roff, npad;
  int64_t N = 0;
  DevBuf rowptr, colidx, gid;
  wl_graph* G = nullptr;
  std::vector<wl_op_desc> d;
  std::vector<int> K;
  int Kmax = 0;
  DevBuf gtab;       // [Kmax][ng][5]
  DevBuf gtab_none;  // all-zero-finish copy used for phi 1 (no Laplacian finish)
  DevBuf w;          // walk degrees, N floats
  std::vector<int64_t> us;
  std::vector<int> gu0;
  DevBuf d_us, d_gu0;
  DevBuf ones;
  BatchWork work;  // scratch of the eager entry points
  XcdTileMap xmap;  // every graph's row tiles on one XCD
  bool use_xmap = false;  // chosen by wl_batch_autotune (timed against the plain order)
  int graphs = 0;  // live captured graphs (they hold pointers into the batch)
};

namespace {

wl_status batch_gram(wl_batch* bt, BatchWork& wk, const float* X, int64_t sX, int nblk, const float* Y, int b,
                     double* out, int64_t gs) {
  wl_ctx* ctx = bt->ctx;
  const int nunits = (int)bt->us.size() - 1;
  WL_TRY(wk.partials.ensure((size_t)nblk * nunits * 256 * sizeof(double)));
  const int blocks = std::max(1, std::min(1024, (nunits + 3) / 4));
  const int NB = nblk >= 3 ? 3 : nblk;
  dim3 grid(blocks, (nblk + NB - 1) / NB);
  if (NB == 1)
    hipLaunchKernelGGL(k_gram_seg<1>, grid, dim3(256), 0, ctx->stream, bt->d_us.as<int64_t>(), nunits, X, sX, nblk, Y,
                       b, wk.partials.as<double>());
  else if (NB == 2)
    hipLaunchKernelGGL(k_gram_seg<2>, grid, dim3(256), 0, ctx->stream, bt->d_us.as<int64_t>(), nunits, X, sX, nblk, Y,
                       b, wk.partials.as<double>());
  else
    hipLaunchKernelGGL(k_gram_seg<3>, grid, dim3(256), 0, ctx->stream, bt->d_us.as<int64_t>(), nunits, X, sX, nblk, Y,
                       b, wk.partials.as<double>());
  WL_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_gram_seg_finalize, dim3(16, nblk, bt->ng), dim3(256), 0, ctx->stream,
                     wk.partials.as<double>(), nunits, bt->d_gu0.as<int>(), b, out, gs);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status batch_update(wl_batch* bt, const float* X, int64_t sX, int nblk, int b, const double* C, int64_t cgs,
                       const float* Yin, double alpha, const float* wv, double beta, float* Out) {
  const int grid = (int)std::min<int64_t>(8192, (bt->N + 255) / 256);
  const size_t lds = (size_t)nblk * b * b * sizeof(float);
  WL_CHECK(lds <= 64 * 1024, WL_EINVAL, "batched update: %d coefficient blocks of %d x %d exceed 64 KiB", nblk, b, b);
  // float4 row loads need 16-byte aligned rows: b a multiple of 4 and aligned bases
  const bool al = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Out) |
                    reinterpret_cast<uintptr_t>(Yin)) & 15u) == 0 && (sX % 4) == 0;
  if (b <= 8 && (b == 8 ? al : true))
    hipLaunchKernelGGL((k_update_seg<8>), dim3(grid), dim3(256), lds, bt->ctx->stream, bt->N, X, sX, nblk, b, C,
                       cgs, bt->gid.as<int32_t>(), Yin, alpha, wv, beta, Out);
  else if (b <= 8)
    hipLaunchKernelGGL((k_update_seg<9>), dim3(grid), dim3(256), lds, bt->ctx->stream, bt->N, X, sX, nblk, b, C,
                       cgs, bt->gid.as<int32_t>(), Yin, alpha, wv, beta, Out);
  else if (b == 16 && al)
    hipLaunchKernelGGL((k_update_seg<16>), dim3(grid), dim3(256), lds, bt->ctx->stream, bt->N, X, sX, nblk, b, C,
                       cgs, bt->gid.as<int32_t>(), Yin, alpha, wv, beta, Out);
  else
    hipLaunchKernelGGL((k_update_seg<17>), dim3(grid), dim3(256), lds, bt->ctx->stream, bt->N, X, sX, nblk, b, C,
                       cgs, bt->gid.as<int32_t>(), Yin, alpha, wv, beta, Out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

// phi X for every graph by its truncated series (eq. qrec), optionally finished into
// the walk Laplacian (Y = w * X - phi X at each graph's last degree).
wl_status batch_phi(wl_batch* bt, BatchWork& wk, const float* X, float* Y, int b, bool laplacian) {
  wl_graph* g = bt->G;
  const int64_t N = bt->N;
  WL_TRY(wk.bufA.ensure((size_t)N * b * 4));
  WL_TRY(wk.bufB.ensure((size_t)N * b * 4));
  float* A = wk.bufA.as<float>();
  float* B = wk.bufB.as<float>();
  const SpmmShape sh = shape_for(g, WL_FP32, b);
  const double* tab = laplacian ? bt->gtab.as<double>() : bt->gtab_none.as<double>();
  const int64_t tstride = (int64_t)bt->ng * 5;
  {
    EpiArgs<float> ep;
    ep.xmap = bt->use_xmap ? &bt->xmap : nullptr;
    ep.gid = bt->gid.as<int32_t>();
    ep.gtab = tab;
    ep.Sin = X;
    ep.Sout = Y;
    ep.s0 = 1.0;
    if (laplacian) {
      ep.wv = bt->w.as<float>();
      ep.Xw = X;
    }
    ep.kclass = WL_KC_RECURRENCE;
    WL_TRY(launch_spmm<float>(g, X, A, b, ep, sh));
  }
  const float* Pm2 = X;
  float* Pm1 = A;
  for (int k = 2; k <= bt->Kmax; ++k) {
    EpiArgs<float> ep;
    ep.xmap = bt->use_xmap ? &bt->xmap : nullptr;
    ep.gid = bt->gid.as<int32_t>();
    ep.gtab = tab + (int64_t)(k - 1) * tstride;
    ep.Z = Pm2;
    ep.Sin = Y;
    ep.Sout = Y;
    ep.s0 = 1.0;
    if (laplacian) {
      ep.wv = bt->w.as<float>();
      ep.Xw = X;
    }
    ep.kclass = WL_KC_RECURRENCE;
    float* out = (k == 2) ? B : const_cast<float*>(Pm2);
    WL_TRY(launch_spmm<float>(g, Pm1, out, b, ep, sh));
    Pm2 = Pm1;
    Pm1 = out;
  }
  return WL_OK;
}

}  // namespace

struct wl_batch_graph {
  wl_batch* bt = nullptr;
  int b = 0, K = 0;
  BatchWork work;
  hipGraphExec_t exec = nullptr;
};

namespace {

wl_status expv_check(wl_batch* bt, int b, int outer_dim) {
  WL_CHECK(b >= 2 && b <= 16, WL_EINVAL, "batched diffusion: b must lie in [2, 16]");
  WL_CHECK(outer_dim >= 1 && outer_dim * b <= EXP_MAXM, WL_EINVAL, "batched diffusion: outer_dim * b must be <= %d",
           EXP_MAXM);
  // the projected matrix and its exponential's work vectors live in one workgroup's LDS
  WL_CHECK((size_t)5 * outer_dim * b * b * 8 <= 150 * 1024, WL_EINVAL,
           "batched diffusion: outer_dim * b^2 too large for the on-chip exponential (5 outer_dim b^2 doubles <= "
           "150 KiB)");
  return WL_OK;
}

// Every buffer the enqueued work touches, sized for (b, K), plus the per-graph caps.
wl_status expv_prepare(wl_batch* bt, BatchWork& wk, int b, int K) {
  wl_ctx* ctx = bt->ctx;
  const int ng = bt->ng;
  const int64_t blk = bt->N * b;
  Layout Ly{b, K, (int64_t)b * b};
  const int64_t gs = Ly.total();
  const int nunits = (int)bt->us.size() - 1;
  WL_TRY(wk.basis.ensure((size_t)(K + 1) * blk * 4));
  WL_TRY(wk.S.ensure((size_t)ng * gs * 8));
  WL_TRY(wk.F.ensure((size_t)ng * K * b * b * 8));
  WL_TRY(wk.tvals.ensure((size_t)ng * 8));
  WL_TRY(wk.kcap.ensure((size_t)ng * 4));
  WL_TRY(wk.partials.ensure((size_t)3 * nunits * 256 * sizeof(double)));
  WL_TRY(wk.bufA.ensure((size_t)blk * 4));
  WL_TRY(wk.bufB.ensure((size_t)blk * 4));
  // blocks after which a full-rank start block has exhausted each graph's Krylov space
  // (ceil(n_g / b)); later blocks would be rounding noise in FP32.  A graph whose space
  // grows more slowly (dependent columns, many small components) stops there with the
  // approximation reached by then; the tests on such graphs measure 1e-6 against the
  // dense exponential.
  std::vector<int32_t> kcap(ng);
  wk.cap_at.assign(K, 0);
  for (int g = 0; g < ng; ++g) {
    kcap[g] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(K, (bt->n[g] + b - 1) / b));
    wk.cap_at[kcap[g] - 1] = 1;
  }
  WL_HIP(hipMemcpyAsync(wk.kcap.p, kcap.data(), (size_t)ng * 4, hipMemcpyHostToDevice, ctx->stream));
  if (bt->use_xmap) {
    // the XCD tile map of the sparse products' shape is built (allocated, uploaded) now,
    // not on first use inside a captured sequence; every product of the diffusion runs
    // on library buffers of width b, so one shape covers them all
    EpiArgs<float> ep;
    ep.xmap = &bt->xmap;
    ep.prepare_only = 1;
    WL_TRY(launch_spmm<float>(bt->G, wk.bufA.as<float>(), wk.bufB.as<float>(), b, ep, shape_for(bt->G, WL_FP32, b)));
  }
  const size_t lds = (size_t)5 * K * b * b * sizeof(double);
  WL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_expT_batched),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  return WL_OK;
}

// The device part of the batched diffusion: kernels only (no allocation, no host
// synchronisation), so that it can be captured.  Times are read from wk.tvals.
wl_status expv_enqueue(wl_batch* bt, BatchWork& wk, const float* U0, int b, int K, float* Y) {
  wl_ctx* ctx = bt->ctx;
  const int ng = bt->ng;
  const int64_t blk = bt->N * b;
  Layout Ly{b, K, (int64_t)b * b};
  const int64_t gs = Ly.total();
  float* V = wk.basis.as<float>();
  double* S = wk.S.as<double>();
  const double tol = 1e-10, ptol = 1e-5;  // FP32 deflation thresholds (as the single-graph path)
  // V_0 R_0 = U0 by CholQR2, per graph
  WL_TRY(batch_gram(bt, wk, U0, 0, 1, U0, b, S + Ly.G(), gs));
  WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R1(), S + Ly.Ri1(), nullptr, nullptr, ng, gs,
                     S + Ly.Ref()));
  WL_TRY(batch_update(bt, U0, 0, 1, b, S + Ly.Ri1(), gs, nullptr, 0.0, nullptr, 1.0, V));
  WL_TRY(batch_gram(bt, wk, V, 0, 1, V, b, S + Ly.G(), gs));
  WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(), S + Ly.R0(),
                     ng, gs, nullptr, S + Ly.Ref(), ptol));
  WL_TRY(batch_update(bt, V, 0, 1, b, S + Ly.Ri2(), gs, nullptr, 0.0, nullptr, 1.0, V));
  for (int j = 0; j < K; ++j) {
    float* Vj = V + (int64_t)j * blk;
    float* Vn = V + (int64_t)(j + 1) * blk;
    WL_TRY(batch_phi(bt, wk, Vj, Vn, b, true));  // W' = L V_j
    if (j > 0) {
      hipLaunchKernelGGL(k_dtranspose_batched, dim3(ng), dim3(64), 0, ctx->stream, b, S + Ly.B(j - 1), S + Ly.Bt(),
                         gs);
      WL_HIP(hipGetLastError());
      WL_TRY(batch_update(bt, Vj - blk, 0, 1, b, S + Ly.Bt(), gs, Vn, 1.0, nullptr, -1.0, Vn));
    }
    const int nbv = j > 0 ? 2 : 1;
    float* Vlo = j > 0 ? Vj - blk : Vj;
    WL_TRY(batch_gram(bt, wk, Vlo, blk, nbv + 1, Vn, b, S + Ly.P(), gs));
    WL_TRY(launch_lanczos_proj(ctx, b, nbv, S + Ly.P(), S + Ly.A(j), S + Ly.Cc(), S + Ly.Ref(), ng, gs));
    // W = [V_{j-1} V_j W'] Cc in place, then CholQR2 on its true Gram
    WL_TRY(batch_update(bt, Vlo, blk, nbv + 1, b, S + Ly.Cc(), gs, nullptr, 0.0, nullptr, 1.0, Vn));
    WL_TRY(batch_gram(bt, wk, Vn, 0, 1, Vn, b, S + Ly.G(), gs));
    WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, nullptr, S + Ly.Ri1(), nullptr, S + Ly.R1(), ng, gs,
                       nullptr, S + Ly.Ref(), ptol));
    if (j + 1 == K) {  // residual coupling B_{K-1} = R1 of every graph
      hipLaunchKernelGGL(k_dcopy_batched, dim3(ng), dim3(64), 0, ctx->stream, b * b, S + Ly.R1(), S + Ly.B(j), gs);
      WL_HIP(hipGetLastError());
      break;
    }
    WL_TRY(batch_update(bt, Vn, 0, 1, b, S + Ly.Ri1(), gs, nullptr, 0.0, nullptr, 1.0, Vn));
    WL_TRY(batch_gram(bt, wk, Vn, 0, 1, Vn, b, S + Ly.G(), gs));
    WL_TRY(launch_chol(ctx, b, S + Ly.G(), tol, nullptr, nullptr, S + Ly.R2(), S + Ly.Ri2(), S + Ly.R1(),
                       S + Ly.B(j), ng, gs));
    if (wk.cap_at[j]) {
      hipLaunchKernelGGL(k_cap_blocks, dim3(ng), dim3(64), 0, ctx->stream, ng, wk.kcap.as<int32_t>(), j, S, gs,
                         Ly.Ri2(), Ly.B(j), b * b);
      WL_HIP(hipGetLastError());
    }
    WL_TRY(batch_update(bt, Vn, 0, 1, b, S + Ly.Ri2(), gs, nullptr, 0.0, nullptr, 1.0, Vn));
  }
  // F_g = exp(-t_g T_g) E_1 R0_g on the device, then Y = V F per graph
  const size_t lds = (size_t)5 * K * b * b * sizeof(double);
  hipLaunchKernelGGL(k_expT_batched, dim3(ng), dim3(256), lds, ctx->stream, K, b, S, gs, Ly.A(0), Ly.B(0), Ly.R0(),
                     wk.tvals.as<double>(), wk.F.as<double>(), (int64_t)K * b * b);
  WL_HIP(hipGetLastError());
  WL_TRY(batch_update(bt, V, blk, K, b, wk.F.as<double>(), (int64_t)K * b * b, nullptr, 0.0, nullptr, 1.0, Y));
  return WL_OK;
}

// p_hat / p_err per graph (leave-one-out Nystrom, Alg. 1) from F and R0 alone
// (Omega = V_0 R0, Y = V F: Omega^T Y = R0^T F_0, Y^T Y = F^T F).  Synchronises.
wl_status return_probabilities(wl_batch* bt, BatchWork& wk, int b, int K, double* p_hat, double* p_err) {
  wl_ctx* ctx = bt->ctx;
  const int ng = bt->ng;
  Layout Ly{b, K, (int64_t)b * b};
  const int64_t gs = Ly.total();
  if (p_hat || p_err) {
    // Nystrom trace per graph from F_g and R0_g alone (Omega = V_0 R0, Y = V F).
    std::vector<double> hF((size_t)ng * K * b * b), hS((size_t)ng * gs);
    WL_HIP(hipMemcpyAsync(hF.data(), wk.F.p, hF.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipMemcpyAsync(hS.data(), wk.S.p, hS.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    for (int g = 0; g < ng; ++g) {
      const double* Fg = &hF[(size_t)g * K * b * b];
      const double* R0 = &hS[(size_t)g * gs + Ly.R0()];
      const int M = b, m = K * b;
      std::vector<double> H((size_t)M * M, 0.0), Gm((size_t)M * M, 0.0);
      for (int i = 0; i < M; ++i)
        for (int jj = 0; jj < M; ++jj) {
          double s1 = 0.0, s2 = 0.0;
          for (int k = 0; k < M; ++k) s1 += R0[k * M + i] * Fg[k * M + jj];  // (R0^T F_0)
          for (int r = 0; r < m; ++r) s2 += Fg[(size_t)r * M + i] * Fg[(size_t)r * M + jj];
          H[(size_t)i * M + jj] = s1;
          Gm[(size_t)i * M + jj] = s2;
        }
      // leave-one-out Nystrom (same formulas as wl_estimate)
      std::vector<double> tj(M);
      for (int j = 0; j < M; ++j) {
        const int mm = M - 1;
        std::vector<double> Sm((size_t)mm * mm), lam(mm), U((size_t)mm * mm);
        std::vector<int> map;
        for (int a = 0; a < M; ++a)
          if (a != j) map.push_back(a);
        for (int a = 0; a < mm; ++a)
          for (int c = 0; c < mm; ++c)
            Sm[(size_t)a * mm + c] =
                0.5 * (H[(size_t)map[a] * M + map[c]] + H[(size_t)map[c] * M + map[a]]);
        double trPG = 0.0, hPh = 0.0;
        if (mm > 0 && dense_syev(mm, Sm.data(), lam.data(), U.data()) == 0) {
          double lmax = 0.0;
          for (double v : lam) lmax = std::max(lmax, v);
          std::vector<double> P((size_t)mm * mm, 0.0);
          for (int k = 0; k < mm; ++k) {
            if (!(lam[k] > 1e-10 * lmax)) continue;
            for (int a = 0; a < mm; ++a)
              for (int c = 0; c < mm; ++c) P[(size_t)a * mm + c] += U[(size_t)a * mm + k] * U[(size_t)c * mm + k] / lam[k];
          }
          for (int a = 0; a < mm; ++a)
            for (int c = 0; c < mm; ++c) {
              trPG += P[(size_t)a * mm + c] * Gm[(size_t)map[c] * M + map[a]];
              hPh += H[(size_t)j * M + map[a]] * P[(size_t)a * mm + c] * H[(size_t)j * M + map[c]];
            }
        }
        tj[j] = trPG + H[(size_t)j * M + j] - hPh;
      }
      double mean = 0.0;
      for (double v : tj) mean += v;
      mean /= M;
      double var = 0.0;
      for (double v : tj) var += (v - mean) * (v - mean);
      if (p_hat) p_hat[g] = mean / (double)bt->n[g];
      if (p_err) p_err[g] = std::sqrt(var / (M - 1)) / std::sqrt((double)M) / (double)bt->n[g];
    }
  }
  return WL_OK;
}

}  // namespace

extern "C" {

wl_status wl_batch_create(wl_ctx* ctx, int32_t ngraphs, wl_graph* const* graphs, const wl_op_desc* descs,
                          double tol, wl_batch** out) {
  WL_CHECK(ctx && graphs && descs && out, WL_EINVAL, "wl_batch_create: null argument");
  *out = nullptr;
  WL_CHECK(ngraphs >= 1 && ngraphs <= 65535, WL_EINVAL, "wl_batch_create: ngraphs must lie in [1, 65535]");
  WL_CHECK(std::isfinite(tol) && tol >= 0, WL_EINVAL, "wl_batch_create: bad tol");
  if (tol == 0) tol = 1e-10;
  (void)hipSetDevice(ctx->device);
  auto* bt = new wl_batch;
  bt->ctx = ctx;
  bt->ng = ngraphs;
  auto fail = [&](wl_status s) {
    if (bt->G) graph_release(bt->G);
    delete bt;
    return s;
  };
  // sizes, padded offsets, per-graph series degree
  int64_t nnz_tot = 0;
  bt->n.resize(ngraphs);
  bt->roff.resize(ngraphs);
  bt->npad.resize(ngraphs);
  bt->K.resize(ngraphs);
  bt->d.assign(descs, descs + ngraphs);
  for (int gi = 0; gi < ngraphs; ++gi) {
    wl_graph* g = graphs[gi];
    if (!g || g->ctx != ctx) {
      wl_set_error("wl_batch_create: graph %d is null or from another context", gi);
      return fail(WL_EINVAL);
    }
    const wl_op_desc& d = descs[gi];
    if (!(d.mu >= 0 && d.mu <= 1) || !(d.param > 0) || (d.func != WL_F_EXP && d.func != WL_F_RESOLVENT)) {
      wl_set_error("wl_batch_create: bad descriptor for graph %d", gi);
      return fail(WL_EINVAL);
    }
    bt->n[gi] = g->n;
    bt->npad[gi] = std::max<int64_t>(64, (g->n + 63) / 64 * 64);
    bt->roff[gi] = bt->N;
    bt->N += bt->npad[gi];
    nnz_tot += g->nnz;
    double lam;
    wl_status s = wl_lambda_max(g, 1e-10, &lam);
    if (s != WL_OK) return fail(s);
    int K = d.krylov_dim;
    if (K == 0) {
      if (d.func == WL_F_EXP) {
        const double x = d.param * lam;
        double term = 1.0, tail = std::exp(x) - 1.0;
        K = 0;
        while (tail > tol * std::exp(x) && K < 400) {
          ++K;
          term *= x / K;
          tail -= term;
        }
      } else {
        // ||q_k|| <= lambda_max^k: geometric tail of ratio r = alpha lambda_max
        double rho = d.rho_hint;
        if (!(rho > 0)) {
          s = wl_spectral_radius(g, d.mu, 1e-8, &rho);
          if (s != WL_OK) return fail(s);
        }
        if (d.param * rho >= 1.0) {
          wl_set_error("wl_batch_create: alpha * rho(Z_mu) >= 1 for graph %d", gi);
          return fail(WL_ERANGE);
        }
        // rigorous when alpha lambda_max < 1 (||q_k|| <= lambda_max^k); otherwise the
        // asymptotic ratio alpha rho(Z_mu) with a margin of 20 terms
        const double r = d.param * lam;
        if (r < 1.0)
          K = (int)std::ceil(std::log(tol * (1.0 - r)) / std::log(r));
        else
          K = (int)std::ceil(std::log(tol * (1.0 - d.param * rho)) / std::log(d.param * rho)) + 20;
        K = std::max(1, std::min(K, 400));
      }
    }
    bt->K[gi] = std::max(1, K);
    bt->Kmax = std::max(bt->Kmax, bt->K[gi]);
  }
  WL_TRY(wl_graph_check_size(bt->N, nnz_tot));
  // concatenated CSR on the host
  std::vector<int32_t> hrp(bt->N + 1), hgid(bt->N);
  std::vector<int32_t> hci((size_t)std::max<int64_t>(nnz_tot, 1));
  int64_t pos = 0;
  for (int gi = 0; gi < ngraphs; ++gi) {
    wl_graph* g = graphs[gi];
    std::vector<int32_t> rp(g->n + 1);
    if (hipMemcpy(rp.data(), g->rowptr, (g->n + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        (g->nnz > 0 && hipMemcpy(hci.data() + pos, g->colidx, g->nnz * 4, hipMemcpyDeviceToHost) != hipSuccess)) {
      wl_set_error("wl_batch_create: reading graph %d failed", gi);
      return fail(WL_EDEVICE);
    }
    const int64_t ro = bt->roff[gi];
    for (int64_t r = 0; r < bt->npad[gi]; ++r) {
      hrp[ro + r] = (int32_t)(pos + (r < g->n ? rp[r] : g->nnz));
      hgid[ro + r] = gi;
    }
    for (int64_t e = 0; e < g->nnz; ++e) hci[pos + e] += (int32_t)ro;
    pos += g->nnz;
  }
  hrp[bt->N] = (int32_t)pos;
  wl_status s = bt->rowptr.ensure((bt->N + 1) * 4);
  if (s == WL_OK) s = bt->colidx.ensure(hci.size() * 4);
  if (s == WL_OK) s = bt->gid.ensure(bt->N * 4);
  if (s != WL_OK) return fail(s);
  if (hipMemcpy(bt->rowptr.p, hrp.data(), (bt->N + 1) * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(bt->colidx.p, hci.data(), hci.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(bt->gid.p, hgid.data(), bt->N * 4, hipMemcpyHostToDevice) != hipSuccess) {
    wl_set_error("wl_batch_create: upload failed");
    return fail(WL_EDEVICE);
  }
  s = wl_graph_create(ctx, bt->N, pos, bt->rowptr.as<int32_t>(), bt->colidx.as<int32_t>(), 0, &bt->G);
  if (s != WL_OK) return fail(s);
  // XCD placement: graphs by decreasing nonzeros onto the least loaded XCD
  {
    std::vector<int> order(ngraphs);
    for (int gi = 0; gi < ngraphs; ++gi) order[gi] = gi;
    std::sort(order.begin(), order.end(), [&](int a, int c) { return graphs[a]->nnz > graphs[c]->nnz; });
    double load[XcdTileMap::NXCD] = {0};
    bt->xmap.start.assign(bt->roff.begin(), bt->roff.end());
    bt->xmap.end.resize(ngraphs);
    bt->xmap.xcd.resize(ngraphs);
    for (int gi = 0; gi < ngraphs; ++gi) bt->xmap.end[gi] = bt->roff[gi] + bt->npad[gi];
    for (int gi : order) {
      int best = 0;
      for (int x = 1; x < XcdTileMap::NXCD; ++x)
        if (load[x] < load[best]) best = x;
      bt->xmap.xcd[gi] = best;
      load[best] += (double)graphs[gi]->nnz + (double)bt->npad[gi];
    }
  }
  // reduction units
  bt->gu0.resize(ngraphs + 1);
  for (int gi = 0; gi < ngraphs; ++gi) {
    bt->gu0[gi] = (int)bt->us.size();
    for (int64_t r = 0; r < bt->npad[gi]; r += UNIT_ROWS) bt->us.push_back(bt->roff[gi] + r);
  }
  bt->gu0[ngraphs] = (int)bt->us.size();
  bt->us.push_back(bt->N);
  s = bt->d_us.ensure(bt->us.size() * 8);
  if (s == WL_OK) s = bt->d_gu0.ensure(bt->gu0.size() * 4);
  if (s != WL_OK) return fail(s);
  if (hipMemcpy(bt->d_us.p, bt->us.data(), bt->us.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(bt->d_gu0.p, bt->gu0.data(), bt->gu0.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(WL_EDEVICE);
  // coefficient tables: step k (1-based) of graph g: {a, b0, b1, sc, fin}
  std::vector<double> tab((size_t)bt->Kmax * ngraphs * 5, 0.0), tab0;
  for (int gi = 0; gi < ngraphs; ++gi) {
    const double sp = bt->d[gi].param, mu = bt->d[gi].mu;
    double omega = 1.0;
    for (int k = 1; k <= bt->K[gi]; ++k) {
      if (bt->d[gi].func == WL_F_EXP) omega /= k;  // c_k / s^k = 1 / k!
      double* c = &tab[((size_t)(k - 1) * ngraphs + gi) * 5];
      c[0] = sp;
      c[1] = k >= 3 ? sp * sp * mu * mu : 0.0;
      c[2] = k >= 2 ? -sp * sp * mu : 0.0;
      c[3] = omega;
      c[4] = k == bt->K[gi] ? 1.0 : 0.0;
    }
  }
  tab0 = tab;
  for (size_t i = 4; i < tab0.size(); i += 5) tab0[i] = 0.0;
  s = bt->gtab.ensure(tab.size() * 8);
  if (s == WL_OK) s = bt->gtab_none.ensure(tab.size() * 8);
  if (s != WL_OK) return fail(s);
  if (hipMemcpy(bt->gtab.p, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(bt->gtab_none.p, tab0.data(), tab0.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    return fail(WL_EDEVICE);
  // walk degrees w = phi 1 for every graph
  s = bt->w.ensure(bt->N * 4);
  if (s == WL_OK) s = bt->ones.ensure(bt->N * 4);
  if (s == WL_OK) s = launch_fill<float>(ctx, bt->N, 1.0f, bt->ones.as<float>());
  if (s == WL_OK) s = batch_phi(bt, bt->work, bt->ones.as<float>(), bt->w.as<float>(), 1, false);
  if (s == WL_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) s = WL_EDEVICE;
  if (s != WL_OK) return fail(s);
  ++ctx->refs;
  *out = bt;
  return WL_OK;
}

wl_status wl_batch_destroy(wl_batch* bt) {
  if (!bt) return WL_OK;
  WL_CHECK(bt->graphs == 0, WL_EINVAL, "wl_batch_destroy: %d captured graphs of this batch are still alive",
           bt->graphs);
  wl_ctx* ctx = bt->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  graph_release(bt->G);
  delete bt;
  ctx_release(ctx);
  return WL_OK;
}

wl_status wl_batch_info(const wl_batch* bt, int64_t* total_rows, int32_t* max_degree_series, int64_t* row_offsets,
                        int32_t* series_degrees) {
  WL_CHECK(bt, WL_EINVAL, "wl_batch_info: batch is null");
  if (total_rows) *total_rows = bt->N;
  if (max_degree_series) *max_degree_series = bt->Kmax;
  if (row_offsets)
    for (int g = 0; g < bt->ng; ++g) row_offsets[g] = bt->roff[g];
  if (series_degrees)
    for (int g = 0; g < bt->ng; ++g) series_degrees[g] = bt->K[g];
  return WL_OK;
}

wl_status wl_batch_autotune(wl_batch* bt, int32_t b) {
  WL_CHECK(bt, WL_EINVAL, "wl_batch_autotune: batch is null");
  WL_CHECK(b >= 1 && b <= 64, WL_EINVAL, "wl_batch_autotune: b must lie in [1, 64]");
  WL_TRY(wl_autotune(bt->G, WL_FP32, b));
  // then the tile order: XCD-grouped graphs against the plain order, timed on the
  // batch's own series products (walk degrees' coefficients, no finish)
  wl_ctx* ctx = bt->ctx;
  DeviceGuard dg(ctx->device);
  DevBuf X, Y;
  WL_TRY(X.ensure((size_t)bt->N * b * 4));
  WL_TRY(Y.ensure((size_t)bt->N * b * 4));
  WL_TRY(launch_fill<float>(ctx, bt->N * b, 1.0f, X.as<float>()));
  hipEvent_t e0, e1;
  WL_HIP(hipEventCreate(&e0));
  WL_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  bool best_map = false;
  wl_status s = WL_OK;
  for (int rep = 0; rep < 2 && s == WL_OK; ++rep)
    for (int m = 0; m < 2 && s == WL_OK; ++m) {
      bt->use_xmap = m == 1;
      s = batch_phi(bt, bt->work, X.as<float>(), Y.as<float>(), b, false);  // warm
      if (s != WL_OK) break;
      (void)hipEventRecord(e0, ctx->stream);
      s = batch_phi(bt, bt->work, X.as<float>(), Y.as<float>(), b, false);
      (void)hipEventRecord(e1, ctx->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep == 1 && ms < best) {
        best = ms;
        best_map = bt->use_xmap;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  bt->use_xmap = best_map;
  return s;
}

wl_status wl_batch_tile_order(const wl_batch* bt, int32_t* xcd_grouped) {
  WL_CHECK(bt && xcd_grouped, WL_EINVAL, "wl_batch_tile_order: null argument");
  *xcd_grouped = bt->use_xmap ? 1 : 0;
  return WL_OK;
}

wl_status wl_batch_set_tile_order(wl_batch* bt, int32_t xcd_grouped) {
  WL_CHECK(bt, WL_EINVAL, "wl_batch_set_tile_order: batch is null");
  bt->use_xmap = xcd_grouped != 0;
  return WL_OK;
}

wl_status wl_batch_apply_L(wl_batch* bt, const void* d_X, void* d_Y, int32_t b) {
  WL_CHECK(bt && d_X && d_Y && d_X != d_Y, WL_EINVAL, "wl_batch_apply_L: bad arguments");
  WL_CHECK(b >= 1 && b <= 64, WL_EINVAL, "wl_batch_apply_L: b must lie in [1, 64]");
  (void)hipSetDevice(bt->ctx->device);
  return batch_phi(bt, bt->work, (const float*)d_X, (float*)d_Y, b, true);
}

wl_status wl_batch_expv(wl_batch* bt, const void* d_U0, int32_t b, const double* t, int32_t outer_dim, void* d_Y,
                        double* p_hat, double* p_err) {
  WL_CHECK(bt && d_U0 && d_Y && t && d_U0 != d_Y, WL_EINVAL, "wl_batch_expv: bad arguments");
  WL_TRY(expv_check(bt, b, outer_dim));
  for (int g = 0; g < bt->ng; ++g) WL_CHECK(std::isfinite(t[g]) && t[g] >= 0, WL_EINVAL, "wl_batch_expv: bad t");
  wl_ctx* ctx = bt->ctx;
  (void)hipSetDevice(ctx->device);
  BatchWork& wk = bt->work;
  WL_TRY(expv_prepare(bt, wk, b, outer_dim));
  WL_HIP(hipMemcpyAsync(wk.tvals.p, t, (size_t)bt->ng * 8, hipMemcpyHostToDevice, ctx->stream));
  WL_TRY(expv_enqueue(bt, wk, (const float*)d_U0, b, outer_dim, (float*)d_Y));
  if (p_hat || p_err) WL_TRY(return_probabilities(bt, wk, b, outer_dim, p_hat, p_err));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  return WL_OK;
}

wl_status wl_batch_graph_create(wl_batch* bt, const void* d_U0, int32_t b, int32_t outer_dim, void* d_Y,
                                wl_batch_graph** out) {
  WL_CHECK(bt && d_U0 && d_Y && out && d_U0 != d_Y, WL_EINVAL, "wl_batch_graph_create: bad arguments");
  *out = nullptr;
  WL_TRY(expv_check(bt, b, outer_dim));
  wl_ctx* ctx = bt->ctx;
  (void)hipSetDevice(ctx->device);
  auto* gr = new wl_batch_graph;
  gr->bt = bt;
  gr->b = b;
  gr->K = outer_dim;
  wl_status s = expv_prepare(bt, gr->work, b, outer_dim);
  if (s != WL_OK) {
    delete gr;
    return s;
  }
  // capture on a private stream (the context's may be the legacy default stream, which
  // cannot be captured); no allocation, synchronisation or profiling event inside
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    delete gr;
    wl_set_error("wl_batch_graph_create: stream creation failed");
    return WL_EDEVICE;
  }
  (void)hipStreamSynchronize(ctx->stream);
  hipStream_t saved = ctx->stream;
  const int saved_prof = ctx->profiling;
  ctx->stream = cs;
  ctx->profiling = 0;
  hipGraph_t graph = nullptr;
  s = WL_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    wl_set_error("wl_batch_graph_create: stream capture could not start");
    s = WL_EDEVICE;
  } else {
    s = expv_enqueue(bt, gr->work, (const float*)d_U0, b, outer_dim, (float*)d_Y);
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (s == WL_OK && e != hipSuccess) {
      wl_set_error("wl_batch_graph_create: capture failed: %s", hipGetErrorString(e));
      s = WL_EDEVICE;
    }
  }
  ctx->stream = saved;
  ctx->profiling = saved_prof;
  if (s == WL_OK && hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    wl_set_error("wl_batch_graph_create: graph instantiation failed");
    s = WL_EDEVICE;
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  if (s != WL_OK) {
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    delete gr;
    return s;
  }
  ++bt->graphs;
  *out = gr;
  return WL_OK;
}

wl_status wl_batch_graph_launch(wl_batch_graph* gr, const double* t, double* p_hat, double* p_err) {
  WL_CHECK(gr && t, WL_EINVAL, "wl_batch_graph_launch: bad arguments");
  wl_batch* bt = gr->bt;
  for (int g = 0; g < bt->ng; ++g)
    WL_CHECK(std::isfinite(t[g]) && t[g] >= 0, WL_EINVAL, "wl_batch_graph_launch: bad t");
  wl_ctx* ctx = bt->ctx;
  (void)hipSetDevice(ctx->device);
  WL_HIP(hipMemcpyAsync(gr->work.tvals.p, t, (size_t)bt->ng * 8, hipMemcpyHostToDevice, ctx->stream));
  WL_HIP(hipGraphLaunch(gr->exec, ctx->stream));
  if (p_hat || p_err) {
    WL_TRY(return_probabilities(bt, gr->work, gr->b, gr->K, p_hat, p_err));
    WL_HIP(hipStreamSynchronize(ctx->stream));
  }
  return WL_OK;
}

wl_status wl_batch_graph_destroy(wl_batch_graph* gr) {
  if (!gr) return WL_OK;
  (void)hipSetDevice(gr->bt->ctx->device);
  (void)hipStreamSynchronize(gr->bt->ctx->stream);
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  --gr->bt->graphs;
  delete gr;
  return WL_OK;
}

}  // extern "C"
