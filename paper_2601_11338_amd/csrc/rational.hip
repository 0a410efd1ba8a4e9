// Rational Krylov estimate of the average return probability (Alg. 1, Sec. 4.4).
//
//   1. rho(L): the caller's value; else for a resolvent the bound max w - s / lambda(A_mu)
//      (phi positive definite, Gershgorin on A_mu), for other operators Lanczos on L;
//   2. poles: AAA on exp(-x) over [0, t* rho] (host), divided by pole_time;
//   3. basis: block rational Krylov space of L and Omega (eq. block-rational-Krylov),
//      built in real arithmetic: a real pole xi adds (L - xi)^{-1} U, a conjugate pair
//      (xi, conj xi) adds Re and Im of (L - xi)^{-1} U (together they span what the two
//      complex poles add), U the last basis block.  Every new block is orthogonalised
//      twice against the basis and orthonormalised by CholQR2 with deflation;
//   4. shifted solves: COCG (conjugate orthogonal CG for complex symmetric systems)
//      column by column, the M complex columns held as one n x 2M real block
//      [Re | Im]; for a resolvent operator on its symmetrised form, one sparse product
//      with A_mu(alpha) per iteration (see k_fl_sqrt; on graphs without long rows the
//      product, the shift and the p^T q sums are one kernel, k_fl_product), otherwise
//      one walk-Laplacian product on 2M columns per iteration;
//   5. projection: T = V^T L V (the Rayleigh quotient; with exact solves it equals the
//      reduced pencil Hhat Khat^{-1} of a pole sequence closed by infinity);
//   6. per time t, on the host from T's eigendecomposition T = S diag(lam) S^T and
//      Z = S^T E_1 R0 (Omega = V_0 R0): Omega^T Y(t) = Z^T e^{-t lam} Z / n and
//      Y(t)^T Y(t) = Z^T e^{-2 t lam} Z / n^2 with Y(t) = V e^{-tT} V^T Omega / n; the
//      leave-one-out Nystrom trace estimate needs only these two M x M matrices, so
//      Y(t) itself is never formed.
#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "wl_internal.h"

// Work buffers of wl_return_prob kept with the operator between calls: the basis and the
// solve blocks (freeing device memory waits for the whole device), the pinned summary
// slots, and the column-group runners with their Lanczos bases.
struct RkCache {
  DevBuf basis, wb, X, R, P, Q, V, dd, dsmall, part, sums, cg;
  double* hsum = nullptr;  // pinned host: two slots of the COCG summary (4 doubles each)
  hipEvent_t ev[2] = {nullptr, nullptr};
  wl_multi* groups_wide = nullptr;    // the operator on 2 Mp columns as 16-column groups
  wl_multi* groups_narrow = nullptr;  // ... on Mp columns
  int groups_mp = 0;                  // the padded width the groups were made for
  void drop_groups() {
    multi_groups_destroy(groups_wide);
    multi_groups_destroy(groups_narrow);
    groups_wide = groups_narrow = nullptr;
    groups_mp = 0;
  }
  ~RkCache() {
    drop_groups();
    if (hsum) (void)hipHostFree(hsum);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

void rk_cache_destroy(wl_op* op) {
  delete op->rk;
  op->rk = nullptr;
}

namespace {

constexpr int RK_MAXM = 32;       // columns of Omega (2M <= 64, the block-width limit)
constexpr int RK_THREADS = 256;   // 8 rows x 32 columns per pass
constexpr int RK_BLOCKS = 1024;   // grid of the row reductions (partials per block)


// Sum of per-block partials (nblk x K, row-major) into out[K], one workgroup per value,
// fixed summation order.
__global__ void k_rk_finish(int nblk, int K, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double s[RK_THREADS];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += part[(size_t)b * K + k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = s[0];
}

// Reduce nv values per column over the 8 row slots of a workgroup into part[block].
template <int NV>
__device__ void block_colsum(double (&v)[NV], int M, double* __restrict__ part) {
  __shared__ double s[NV][8][RK_MAXM];
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
#pragma unroll
  for (int q = 0; q < NV; ++q) s[q][ry][c] = v[q];
  __syncthreads();
  if (ry == 0 && c < M) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double a = 0.0;
      for (int y = 0; y < 8; ++y) a += s[q][y][c];
      part[(size_t)blockIdx.x * NV * M + q * M + c] = a;
    }
  }
}

// x = 0, r = p = [U | 0]; partial sums of ||u_c||^2
template <typename T>
__global__ void k_rk_init(int64_t n, int M, const T* __restrict__ U, T* __restrict__ X, T* __restrict__ R,
                          T* __restrict__ P, double* __restrict__ part) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  double v[1] = {0.0};
  if (c < M)
    for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
      const T u = U[r * M + c];
      const int64_t o = r * 2 * M + c;
      X[o] = T(0);
      X[o + M] = T(0);
      R[o] = u;
      R[o + M] = T(0);
      P[o] = u;
      P[o + M] = T(0);
      v[0] += (double)u * (double)u;
    }
  block_colsum<1>(v, M, part);
}

// Q <- Q - xi P (Q holds L P on entry); partials of p^T q (complex, unconjugated)
template <typename T>
__global__ void k_rk_shift_dot(int64_t n, int M, double a, double b, const T* __restrict__ P, T* __restrict__ Q,
                               double* __restrict__ part) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  double v[2] = {0.0, 0.0};
  if (c < M)
    for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
      const int64_t o = r * 2 * M + c;
      const double pr = P[o], pi = P[o + M];
      const double qr = (double)Q[o] - (a * pr - b * pi);
      const double qi = (double)Q[o + M] - (a * pi + b * pr);
      Q[o] = (T)qr;
      Q[o + M] = (T)qi;
      v[0] += pr * qr - pi * qi;
      v[1] += pr * qi + pi * qr;
    }
  block_colsum<2>(v, M, part);
}

// x += alpha p, r -= alpha q (complex alpha per column); partials of r^T r (complex)
// and ||r||^2
// With dre/dim given the third sum is ||d (.) r||^2 (the residual of the original system
// when r is that of the symmetrised one).
template <typename T>
__global__ void k_rk_xr(int64_t n, int M, const double* __restrict__ al, const T* __restrict__ P,
                        const T* __restrict__ Q,
                        T* __restrict__ X, T* __restrict__ R, const T* __restrict__ dre, const T* __restrict__ dim,
                        double* __restrict__ part) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  double v[3] = {0.0, 0.0, 0.0};
  if (c < M) {
    const double ar = al[c], ai = al[RK_MAXM + c];
    for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
      const int64_t o = r * 2 * M + c;
      const double pr = P[o], pi = P[o + M], qr = Q[o], qi = Q[o + M];
      X[o] = (T)((double)X[o] + ar * pr - ai * pi);
      X[o + M] = (T)((double)X[o + M] + ar * pi + ai * pr);
      const double rr = (double)R[o] - (ar * qr - ai * qi);
      const double ri = (double)R[o + M] - (ar * qi + ai * qr);
      R[o] = (T)rr;
      R[o + M] = (T)ri;
      v[0] += rr * rr - ri * ri;
      v[1] += 2.0 * rr * ri;
      const double w2 = dre ? (double)dre[r] * dre[r] + (double)dim[r] * dim[r] : 1.0;
      v[2] += w2 * (rr * rr + ri * ri);
    }
  }
  block_colsum<3>(v, M, part);
}

// ---- the resolvent's shifted systems without inner solves.  With phi = s A^{-1}
// (A = A_mu(alpha), s = 1 - mu^2 alpha^2) and D = diag(w) - xi I,
//   (L - xi I) x = u  <=>  (D A - s I) y = u, x = A y  <=>  (d A d - s I) z = u / d, y = d z
// for d = D^{1/2} elementwise: a complex symmetric system whose product is one sparse
// product with A.  Its residual r_z relates to the original one by r_x = d (.) r_z.

// d = sqrt(w - xi) (principal branch), as two real arrays
template <typename T>
__global__ void k_fl_sqrt(int64_t n, const T* __restrict__ w, double a, double b, T* __restrict__ dre,
                          T* __restrict__ dim) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = (double)w[i] - a, y = -b;
    const double r = sqrt(x * x + y * y);
    const double re = sqrt(0.5 * (r + x));
    const double im = (y >= 0 ? 1.0 : -1.0) * sqrt(fmax(0.0, 0.5 * (r - x)));
    dre[i] = (T)re;
    dim[i] = (T)im;
  }
}

// z = 0, r = p = u / d, V = d (.) p = u (the direction is kept as V alone: p = V / d);
// partials of r^T r (complex) and ||u||^2
template <typename T>
__global__ void k_fl_init(int64_t n, int M, const T* __restrict__ U, const T* __restrict__ dre,
                          const T* __restrict__ dim, T* __restrict__ X, T* __restrict__ R, T* __restrict__ V,
                          double* __restrict__ part) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  double v[3] = {0.0, 0.0, 0.0};
  if (c < M)
    for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
      const double u = U[r * M + c];
      const double dr = dre[r], di = dim[r], m2 = dr * dr + di * di;
      const double rr = u * dr / m2, ri = -u * di / m2;
      const int64_t o = r * 2 * M + c;
      X[o] = T(0);
      X[o + M] = T(0);
      R[o] = (T)rr;
      R[o + M] = (T)ri;
      V[o] = (T)u;  // d (.) (u / d)
      V[o + M] = T(0);
      v[0] += rr * rr - ri * ri;
      v[1] += 2.0 * rr * ri;
      v[2] += u * u;
    }
  block_colsum<3>(v, M, part);
}

// V = d (.) P (every complex column of a row scaled by that row's d)
template <typename T>
__global__ void k_fl_scale(int64_t n, int M, const T* __restrict__ dre, const T* __restrict__ dim,
                           const T* __restrict__ P, T* __restrict__ V) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  if (c >= M) return;
  for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
    const int64_t o = r * 2 * M + c;
    const double dr = dre[r], di = dim[r], pr = P[o], pi = P[o + M];
    V[o] = (T)(dr * pr - di * pi);
    V[o + M] = (T)(dr * pi + di * pr);
  }
}

// With V = d (.) p: x += alpha p (p = V / d) and the next direction
// V = d (.) (r + beta p) = d (.) r + beta V, in one pass
template <typename T>
__global__ void k_fl_dir(int64_t n, int M, const double* __restrict__ al, const double* __restrict__ be,
                         const T* __restrict__ dre, const T* __restrict__ dim, const T* __restrict__ R,
                         T* __restrict__ X, T* __restrict__ V) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  if (c >= M) return;
  const double ar = al[c], ai = al[RK_MAXM + c], br = be[c], bi = be[RK_MAXM + c];
  for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
    const int64_t o = r * 2 * M + c;
    const double dr = dre[r], di = dim[r], m2 = dr * dr + di * di;
    const double vr = V[o], vi = V[o + M];
    const double pr = (vr * dr + vi * di) / m2, pi = (vi * dr - vr * di) / m2;
    X[o] = (T)((double)X[o] + ar * pr - ai * pi);
    X[o + M] = (T)((double)X[o + M] + ar * pi + ai * pr);
    const double rr = R[o], ri = R[o + M];
    V[o] = (T)(dr * rr - di * ri + br * vr - bi * vi);
    V[o + M] = (T)(dr * ri + di * rr + br * vi + bi * vr);
  }
}

// r -= alpha q (complex alpha per column); partials of r^T r (complex) and ||d (.) r||^2
// (the residual of the original system)
template <typename T>
__global__ void k_fl_xr(int64_t n, int M, const double* __restrict__ al, const T* __restrict__ Q,
                        T* __restrict__ R, const T* __restrict__ dre, const T* __restrict__ dim,
                        double* __restrict__ part) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  double v[3] = {0.0, 0.0, 0.0};
  if (c < M) {
    const double ar = al[c], ai = al[RK_MAXM + c];
    for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
      const int64_t o = r * 2 * M + c;
      const double qr = Q[o], qi = Q[o + M];
      const double rr = (double)R[o] - (ar * qr - ai * qi);
      const double ri = (double)R[o + M] - (ar * qi + ai * qr);
      R[o] = (T)rr;
      R[o + M] = (T)ri;
      v[0] += rr * rr - ri * ri;
      v[1] += 2.0 * rr * ri;
      v[2] += ((double)dre[r] * dre[r] + (double)dim[r] * dim[r]) * (rr * rr + ri * ri);
    }
  }
  block_colsum<3>(v, M, part);
}

// Q <- d (.) Q - s p with p = V / d (Q holds A V on entry); partials of p^T q
template <typename T>
__global__ void k_fl_shift_dot(int64_t n, int M, const T* __restrict__ dre, const T* __restrict__ dim, double s,
                               const T* __restrict__ V, T* __restrict__ Q, double* __restrict__ part) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  double v[2] = {0.0, 0.0};
  if (c < M)
    for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
      const int64_t o = r * 2 * M + c;
      const double dr = dre[r], di = dim[r], m2 = dr * dr + di * di, vr = V[o], vi = V[o + M];
      const double pr = (vr * dr + vi * di) / m2, pi = (vi * dr - vr * di) / m2, ar = Q[o], ai = Q[o + M];
      const double qr = dr * ar - di * ai - s * pr;
      const double qi = dr * ai + di * ar - s * pi;
      Q[o] = (T)qr;
      Q[o + M] = (T)qi;
      v[0] += pr * qr - pi * qi;
      v[1] += pr * qi + pi * qr;
    }
  block_colsum<2>(v, M, part);
}

// Longest row the one-pass product below takes: each row is gathered by one lane group,
// so a graph with longer rows runs the sparse-product kernel (whose long rows get whole
// workgroups) followed by k_fl_shift_dot.
constexpr int FL_FUSED_MAXDEG = 256;
constexpr int FL_BLOCKS = 2048;  // workgroups of the one-pass product (a multiple of 8)

// One iteration's operator product of the symmetrised shifted system in one pass, the
// values of the sparse product (A_mu V = a A V + (b0 + b1 deg) V in FP32) followed by
// k_fl_shift_dot: Q = d (.) (A_mu V) - s p with p = V / d, and per-workgroup partials of
// p^T q (complex), laid out as block_colsum's.  M = 2 LPR complex columns: each row is
// LPR lanes of four values, the first half Re and the second Im, so lane l and its
// partner l ^ (LPR / 2) hold the two parts of the same four columns.  The rows are cut
// into 8 contiguous ranges, one per XCD (workgroup w runs on XCD w mod 8), so a row and
// the nearby rows its neighbours usually are go through one L2.
template <int LPR>
__global__ __launch_bounds__(256) void k_fl_product(const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ colidx, int64_t n,
                                                    const float* __restrict__ V, const float* __restrict__ dre,
                                                    const float* __restrict__ dim, float a, float b0, float b1,
                                                    double s, float* __restrict__ Q, double* __restrict__ part) {
  constexpr int M = 2 * LPR, W2 = 2 * M, H = LPR / 2, RG = 256 / LPR;
  const int l = threadIdx.x % LPR, rg = threadIdx.x / LPR;
  const bool re_half = l < H;
  const int col = 4 * l;
  const int64_t per = gridDim.x >> 3;                     // workgroups per XCD
  const int64_t span = ((n + 7) / 8 + RG - 1) / RG * RG;  // rows per XCD range
  const int64_t r0 = (int64_t)(blockIdx.x & 7) * span;
  const int64_t r1 = r0 + span < n ? r0 + span : n;
  double v0[4] = {0.0, 0.0, 0.0, 0.0}, v1[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0 + (int64_t)(blockIdx.x >> 3) * RG + rg; r < r1; r += per * RG) {
    const int beg = rowptr[r], end = rowptr[r + 1];
    const float4 z = *reinterpret_cast<const float4*>(V + r * W2 + col);
    const double dr = dre[r], di = dim[r];
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = beg; k < end; k += 4) {  // up to four neighbour rows in flight
      int j[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) j[u] = k + u < end ? colidx[k + u] : -1;
      float4 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        x[u] = j[u] >= 0 ? *reinterpret_cast<const float4*>(V + (int64_t)j[u] * W2 + col)
                         : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc.x += x[u].x;
        acc.y += x[u].y;
        acc.z += x[u].z;
        acc.w += x[u].w;
      }
    }
    const float cz = b0 + b1 * (float)(end - beg);
    const float y[4] = {a * acc.x + cz * z.x, a * acc.y + cz * z.y, a * acc.z + cz * z.z, a * acc.w + cz * z.w};
    const float zz[4] = {z.x, z.y, z.z, z.w};
    // each lane computes its own part of p and q: with sdi = -di on the Re lanes and +di
    // on the Im lanes, p_own = (z_own dr - sdi z_other) / |d|^2 and
    // q_own = dr y_own + sdi y_other - s p_own
    const double inv = 1.0 / (dr * dr + di * di);
    const double sdi = re_half ? -di : di;
    float out[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double yo = __shfl_xor(y[i], H, 64), zo = __shfl_xor(zz[i], H, 64);
      const double po = ((double)zz[i] * dr - sdi * zo) * inv;
      const double qo = dr * (double)y[i] + sdi * yo - s * po;
      const double qp = __shfl_xor(qo, H, 64);  // the partner's part of q
      out[i] = (float)qo;
      v0[i] += po * qo;  // Re: pr qr, Im: pi qi
      v1[i] += po * qp;  // Re: pr qi, Im: pi qr
    }
    *reinterpret_cast<float4*>(Q + r * W2 + col) = make_float4(out[0], out[1], out[2], out[3]);
  }
  // p^T q = sum (pr qr - pi qi) + i sum (pr qi + pi qr): the Re lane of each column pair
  // takes its partner's sums
  __shared__ double red[2][RG][M];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double o0 = __shfl_xor(v0[i], H, 64), o1 = __shfl_xor(v1[i], H, 64);
    if (re_half) {
      red[0][rg][col + i] = v0[i] - o0;
      red[1][rg][col + i] = v1[i] + o1;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * M; e += 256) {
    const int q = e / M, c = e - q * M;
    double t = 0.0;
    for (int y = 0; y < RG; ++y) t += red[q][y][c];
    part[(size_t)blockIdx.x * 2 * M + e] = t;
  }
}

// p = r + beta p (complex beta per column)
template <typename T>
__global__ void k_rk_dir(int64_t n, int M, const double* __restrict__ be, const T* __restrict__ R,
                         T* __restrict__ P) {
  const int c = threadIdx.x & 31, ry = threadIdx.x >> 5;
  if (c >= M) return;
  const double br = be[c], bi = be[RK_MAXM + c];
  for (int64_t r = (int64_t)blockIdx.x * 8 + ry; r < n; r += (int64_t)gridDim.x * 8) {
    const int64_t o = r * 2 * M + c;
    const double pr = P[o], pi = P[o + M];
    P[o] = (T)((double)R[o] + br * pr - bi * pi);
    P[o + M] = (T)((double)R[o + M] + br * pi + bi * pr);
  }
}

// part[block] = the largest value of v over the rows the block visits
template <typename T>
__global__ __launch_bounds__(256) void k_rk_vmax(int64_t n, const T* __restrict__ v, double* __restrict__ part) {
  __shared__ double s[4];
  double m = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, (double)v[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(s[0], s[1]), fmax(s[2], s[3]));
}

// out (n x M) = real (part 0) or imaginary (part 1) half of X (n x 2M)
template <typename T>
__global__ void k_rk_part(int64_t n, int M, const T* __restrict__ X, int part, T* __restrict__ out) {
  const int64_t total = n * M;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / M;
    const int c = (int)(e - r * M);
    out[e] = X[r * 2 * M + part * M + c];
  }
}

// dst (n x Mp) = src (n x M) followed by Mp - M zero columns
template <typename T>
__global__ void k_rk_pad(int64_t n, int M, int Mp, const T* __restrict__ src, T* __restrict__ dst) {
  const int64_t total = n * Mp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / Mp;
    const int c = (int)(e - r * Mp);
    dst[e] = c < M ? src[r * M + c] : T(0);
  }
}

// ---- COCG recurrence coefficients on the device.  Per column c < M (one thread each)
// the state holds rho (complex), the initial norm, the active flag and the step
// coefficients alpha, beta, so that no iteration waits for the host; the host reads
// the summary (columns still open, worst open residual, worst converged residual,
// breakdown flag) one iteration behind, while the next iteration runs.
struct CgState {
  double al[2 * RK_MAXM], be[2 * RK_MAXM];  // [re | im]
  double rho_re[RK_MAXM], rho_im[RK_MAXM], nrm0[RK_MAXM], active[RK_MAXM];
  double res_open, res_done, open, err;       // summary of the last update
};

__device__ double block_max64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// From the initial sums: flat (symmetrised systems) s = [r^T r (complex) | ||u||^2],
// else s = [||u||^2]; rho = r^T r, nrm0 = ||u||.
__global__ __launch_bounds__(64) void k_cg_setup(int M, int flat, const double* __restrict__ s, CgState* st) {
  const int c = threadIdx.x;
  double open = 0.0;
  if (c < M) {
    const double re = s[c], im = flat ? s[M + c] : 0.0, u2 = flat ? s[2 * M + c] : s[c];
    st->rho_re[c] = re;
    st->rho_im[c] = im;
    st->nrm0[c] = sqrt(u2);
    st->active[c] = u2 > 0.0 ? 1.0 : 0.0;
    st->al[c] = st->al[RK_MAXM + c] = st->be[c] = st->be[RK_MAXM + c] = 0.0;
    open = st->active[c];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) open += __shfl_xor(open, off, 64);
  if (c == 0) {
    st->open = open;
    st->res_open = st->res_done = st->err = 0.0;
  }
}

// alpha = rho / p^T (K - xi) p from s = [p^T q (complex)]; breakdown (p^T q = 0 in an
// open column) sets err = 1 and leaves that column's step at zero
__global__ __launch_bounds__(64) void k_cg_alpha(int M, const double* __restrict__ s, CgState* st) {
  const int c = threadIdx.x;
  if (c >= M) return;
  double ar = 0.0, ai = 0.0;
  if (st->active[c] != 0.0) {
    const double pr = s[c], pi = s[M + c], den = pr * pr + pi * pi;
    if (den == 0.0) {
      st->err = 1.0;
    } else {  // (rho_re + i rho_im) / (pr + i pi)
      ar = (st->rho_re[c] * pr + st->rho_im[c] * pi) / den;
      ai = (st->rho_im[c] * pr - st->rho_re[c] * pi) / den;
    }
  }
  st->al[c] = ar;
  st->al[RK_MAXM + c] = ai;
}

// From s = [r^T r (complex) | residual norm^2]: columns at or below tol close (their
// later steps are zero); open ones take beta = r^T r / rho and rho = r^T r.
__global__ __launch_bounds__(64) void k_cg_beta(int M, double tol, const double* __restrict__ s, CgState* st) {
  const int c = threadIdx.x;
  double worst = 0.0, done = 0.0, open = 0.0, bad = 0.0;
  if (c < M) {
    double br = 0.0, bi = 0.0;
    if (st->active[c] != 0.0) {
      const double res = sqrt(s[2 * M + c]) / st->nrm0[c];
      if (!isfinite(res)) {
        bad = 1.0;
      } else if (res <= tol) {
        st->active[c] = 0.0;
        done = res;
      } else {
        const double rr = s[c], ri = s[M + c];
        const double den = st->rho_re[c] * st->rho_re[c] + st->rho_im[c] * st->rho_im[c];
        br = (rr * st->rho_re[c] + ri * st->rho_im[c]) / den;
        bi = (ri * st->rho_re[c] - rr * st->rho_im[c]) / den;
        st->rho_re[c] = rr;
        st->rho_im[c] = ri;
        worst = res;
        open = 1.0;
      }
    }
    st->be[c] = br;
    st->be[RK_MAXM + c] = bi;
  }
  worst = block_max64(worst);
  done = block_max64(done);
  bad = block_max64(bad);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) open += __shfl_xor(open, off, 64);
  if (c == 0) {
    st->res_open = worst;
    st->res_done = fmax(st->res_done, done);
    st->open = open;
    if (bad != 0.0) st->err = 2.0;
  }
}

int grid_rows(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(RK_BLOCKS, (n + 7) / 8)); }

template <typename T>
struct RkWork {
  explicit RkWork(RkCache& c)
      : dsmall(c.dsmall), part(c.part), sums(c.sums), cg(c.cg), hsum(c.hsum), ev(c.ev),
        groups_wide(c.groups_wide), groups_narrow(c.groups_narrow) {}
  wl_op* op = nullptr;
  wl_ctx* ctx = nullptr;
  int64_t n = 0;
  int M = 0;
  T* basis = nullptr;  // nb_max blocks of n x M
  int nb = 0;          // blocks in the basis
  // the operator's cached buffers (RkCache)
  DevBuf& dsmall;      // device doubles: Grams, coefficients
  DevBuf &part, &sums;  // row-reduction partials and their sums
  DevBuf& cg;           // COCG state (CgState)
  double*& hsum;        // pinned host: two slots of the COCG summary (4 doubles each)
  hipEvent_t (&ev)[2];
  wl_multi*& groups_wide;    // the operator on 2M columns as 16-column groups
  wl_multi*& groups_narrow;  // ... on M columns
};

// Device sums of K values from the row-reduction partials (no host copy).
template <typename T>
void rk_finish(RkWork<T>& W, int K) {
  k_rk_finish<<<K, RK_THREADS, 0, W.ctx->stream>>>(grid_rows(W.n), K, W.part.template as<double>(),
                                                   W.sums.template as<double>());
}

// The COCG summary of the last coefficient update into pinned slot k (asynchronous,
// event recorded); rk_cg_read waits for slot k and returns {res_open, res_done, open, err}.
template <typename T>
wl_status rk_cg_post(RkWork<T>& W, int k) {
  if (!W.hsum) WL_HIP(hipHostMalloc(reinterpret_cast<void**>(&W.hsum), 8 * sizeof(double), hipHostMallocDefault));
  for (auto& e : W.ev)
    if (!e) WL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  const CgState* st = W.cg.template as<CgState>();
  WL_HIP(hipMemcpyAsync(W.hsum + 4 * k, &st->res_open, 4 * sizeof(double), hipMemcpyDeviceToHost, W.ctx->stream));
  WL_HIP(hipEventRecord(W.ev[k], W.ctx->stream));
  return WL_OK;
}

template <typename T>
wl_status rk_cg_read(RkWork<T>& W, int k, double* out) {
  WL_HIP(hipEventSynchronize(W.ev[k]));
  for (int i = 0; i < 4; ++i) out[i] = W.hsum[4 * k + i];
  return WL_OK;
}

// Y = L X on cols columns: the column-group runner when it covers the shape (16-column
// groups of a Lanczos operator), else the operator's own product on the whole block.
template <typename T>
wl_status rk_apply(RkWork<T>& W, const T* X, int cols, T* Y) {
  wl_multi* m = cols == 2 * W.M ? W.groups_wide : (cols == W.M ? W.groups_narrow : nullptr);
  if (m) {
    bool done = false;
    WL_TRY(multi_groups_apply<T>(m, X, 16, Y, true, &done));
    if (done) return WL_OK;
  }
  return phi_apply_impl<T>(W.op, X, Y, cols, W.op->w.template as<T>(), X);
}


// Host copy of the nb*bx x by Gram of the basis blocks [0, nblk) against Y.
template <typename T>
wl_status rk_gram(RkWork<T>& W, const T* X, int nblk, const T* Y, std::vector<double>& G) {
  const int M = W.M;
  WL_TRY(launch_gram<T>(W.ctx, W.n, X, M, W.n * M, nblk, Y, M, W.dsmall.template as<double>()));
  G.resize((size_t)nblk * M * M);
  WL_HIP(hipMemcpyAsync(G.data(), W.dsmall.p, G.size() * 8, hipMemcpyDeviceToHost, W.ctx->stream));
  WL_HIP(hipStreamSynchronize(W.ctx->stream));
  return WL_OK;
}

// Out = Yin - X C (X: nblk basis blocks, C host nblk*M x M), or Out = X_0 C when Yin null.
template <typename T>
wl_status rk_update(RkWork<T>& W, const T* X, int nblk, const std::vector<double>& C, const T* Yin, T* Out) {
  const int M = W.M;
  WL_HIP(hipMemcpyAsync(W.dsmall.p, C.data(), C.size() * 8, hipMemcpyHostToDevice, W.ctx->stream));
  if (Yin)
    WL_TRY(launch_update<T>(W.ctx, W.n, X, M, W.n * M, nblk, W.dsmall.template as<double>(), Yin, 1.0, nullptr,
                            -1.0, Out, M, nullptr));
  else
    WL_TRY(launch_update<T>(W.ctx, W.n, X, M, W.n * M, nblk, W.dsmall.template as<double>(), nullptr, 0.0, nullptr,
                            1.0, Out, M, nullptr));
  WL_HIP(hipStreamSynchronize(W.ctx->stream));  // C (host) may go out of scope on return
  return WL_OK;
}

// Orthonormalise block Wb (n x M) against the basis (two classical Gram-Schmidt passes)
// and append it by CholQR2 with deflation; R (host, M x M) receives the factor of the
// projected block (Wb_projected = V_new R).  Components whose true norm is below the
// deflation level relative to Wb's scale before projection are dropped (zero columns).
template <typename T>
wl_status rk_append(RkWork<T>& W, T* Wb, std::vector<double>* Rout) {
  const int M = W.M;
  const int64_t blk = W.n * M;
  std::vector<double> G, R1, R1i, R2, R2i;
  std::vector<char> k1, k2;
  WL_TRY(rk_gram<T>(W, Wb, 1, Wb, G));
  double ref = 0.0;
  for (int c = 0; c < M; ++c) ref = std::max(ref, G[(size_t)c * M + c]);
  if (W.nb > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<double> C;
      WL_TRY(rk_gram<T>(W, W.basis, W.nb, Wb, C));
      WL_TRY(rk_update<T>(W, W.basis, W.nb, C, Wb, Wb));
    }
    WL_TRY(rk_gram<T>(W, Wb, 1, Wb, G));
  }
  T* slot = W.basis + (size_t)W.nb * blk;
  const double tol = defl_tol<T>();
  host_chol_deflate(M, G, tol, ref, R1, R1i, k1);
  WL_TRY(rk_update<T>(W, Wb, 1, R1i, nullptr, slot));
  WL_TRY(rk_gram<T>(W, slot, 1, slot, G));
  host_chol_deflate(M, G, tol, 1.0, R2, R2i, k2);
  // true norms of the new components: diag(R2 R1); drop the negligible ones
  const double ptol = post_tol<T>();
  for (int c = 0; c < M; ++c) {
    const double d = std::fabs(R2[(size_t)c * M + c] * R1[(size_t)c * M + c]);
    if (!(d > ptol * std::sqrt(ref))) {
      for (int i = 0; i < M; ++i) R2i[(size_t)i * M + c] = 0.0;
      for (int j = 0; j < M; ++j) R2[(size_t)c * M + j] = 0.0;  // the dropped component has no coupling
    }
  }
  WL_TRY(rk_update<T>(W, slot, 1, R2i, nullptr, slot));
  if (Rout) {
    Rout->assign((size_t)M * M, 0.0);
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        double s = 0.0;
        for (int k = 0; k < M; ++k) s += R2[(size_t)i * M + k] * R1[(size_t)k * M + j];
        (*Rout)[(size_t)i * M + j] = s;
      }
  }
  ++W.nb;
  return WL_OK;
}

// COCG on (L - xi I) X = U, U real n x M, X complex as an n x 2M block [Re | Im].
// The recurrence coefficients live on the device (k_cg_*); the host learns that every
// column has converged one iteration late (the summary of iteration it - 1 is read while
// iteration it runs), so at most one extra iteration is made, a no-op for the closed
// columns (their steps are zero).
template <typename T>
wl_status rk_solve(RkWork<T>& W, std::complex<double> xi, const T* U, T* X, T* R, T* P, T* Q, double tol,
                   int max_iters, int* iters, double* res_out) {
  const int M = W.M;
  const int64_t n = W.n;
  wl_ctx* ctx = W.ctx;
  const int grid = grid_rows(n);
  CgState* st = W.cg.template as<CgState>();
  const double* sums = W.sums.template as<double>();
  k_rk_init<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, U, X, R, P, W.part.template as<double>());
  WL_HIP(hipGetLastError());
  rk_finish<T>(W, M);
  k_cg_setup<<<1, 64, 0, ctx->stream>>>(M, 0, sums, st);
  WL_HIP(hipGetLastError());
  WL_TRY(rk_cg_post<T>(W, 0));
  double sm[4];
  WL_TRY(rk_cg_read<T>(W, 0, sm));
  int it = 0, useful = 0;
  bool open = sm[2] > 0.0;
  for (; it < max_iters && open; ++it) {
    WL_TRY(rk_apply<T>(W, P, 2 * M, Q));  // Q = L P
    k_rk_shift_dot<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, xi.real(), xi.imag(), P, Q,
                                                            W.part.template as<double>());
    rk_finish<T>(W, 2 * M);
    k_cg_alpha<<<1, 64, 0, ctx->stream>>>(M, sums, st);
    k_rk_xr<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, st->al, P, Q, X, R, nullptr, nullptr,
                                                     W.part.template as<double>());
    rk_finish<T>(W, 3 * M);
    k_cg_beta<<<1, 64, 0, ctx->stream>>>(M, tol, sums, st);
    k_rk_dir<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, st->be, R, P);
    WL_HIP(hipGetLastError());
    WL_TRY(rk_cg_post<T>(W, it & 1));
    if (it > 0) {  // the previous iteration's summary, read while this one runs
      WL_TRY(rk_cg_read<T>(W, (it - 1) & 1, sm));
      WL_CHECK(sm[3] == 0.0, WL_ENUMERIC, sm[3] == 1.0 ? "rational Krylov: COCG broke down (p^T (L - xi) p = 0)"
                                                       : "rational Krylov: non-finite residual in the shifted solve");
      if (sm[2] == 0.0) {
        useful = it;
        open = false;
        break;
      }
    }
  }
  if (open && it > 0) {  // the last iteration's summary
    WL_TRY(rk_cg_read<T>(W, (it - 1) & 1, sm));
    WL_CHECK(sm[3] == 0.0, WL_ENUMERIC, sm[3] == 1.0 ? "rational Krylov: COCG broke down (p^T (L - xi) p = 0)"
                                                     : "rational Krylov: non-finite residual in the shifted solve");
    useful = it;
    open = sm[2] > 0.0;
  } else if (useful == 0) {
    useful = it;
  }
  *iters = useful;
  *res_out = open ? sm[0] : sm[1];
  if (open) {
    wl_set_error("rational Krylov: shifted solve did not reach %g in %d iterations (residual %g)", tol, max_iters,
                 sm[0]);
    return WL_ENOCONV;
  }
  return WL_OK;
}

// COCG on the symmetrised system of a resolvent operator (see k_fl_sqrt): the same
// solution x of (L - xi I) x = u as rk_solve, with one sparse product per iteration
// instead of a Lanczos run.  Convergence is judged on the original residual d (.) r_z.
// The direction is kept as V = d (.) p alone (p = V / d where needed); the solution
// lands in Q.
template <typename T>
wl_status rk_solve_flat(RkWork<T>& W, std::complex<double> xi, const T* U, T* X, T* R, T* Q, T* V, T* dre,
                        T* dim, double tol, int max_iters, int* iters, double* res_out) {
  const int M = W.M;
  const int64_t n = W.n;
  wl_ctx* ctx = W.ctx;
  wl_graph* g = W.op->g;
  const int grid = grid_rows(n);
  using cd = std::complex<double>;
  double a, b0, b1;
  lanczos_params(W.op, &a, &b0, &b1);  // A_mu(alpha) = a A + b0 I + b1 D, and phi = b0 A_mu^{-1}
  const double s = b0;
  EpiArgs<T> ep;
  ep.a = a;
  ep.b0 = b0;
  ep.b1 = b1;
  ep.kclass = WL_KC_LANCZOS_OP;
  const SpmmShape sh = shape_for(g, prec_of<T>(), 2 * M);
  const int eg = (int)std::min<int64_t>(4096, (n + 255) / 256);
  k_fl_sqrt<T><<<eg, 256, 0, ctx->stream>>>(n, W.op->w.template as<T>(), xi.real(), xi.imag(), dre, dim);
  WL_HIP(hipGetLastError());
  CgState* st = W.cg.template as<CgState>();
  const double* sums = W.sums.template as<double>();
  k_fl_init<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, U, dre, dim, X, R, V, W.part.template as<double>());
  WL_HIP(hipGetLastError());
  rk_finish<T>(W, 3 * M);
  k_cg_setup<<<1, 64, 0, ctx->stream>>>(M, 1, sums, st);
  WL_HIP(hipGetLastError());
  WL_TRY(rk_cg_post<T>(W, 0));
  double sm[4];
  WL_TRY(rk_cg_read<T>(W, 0, sm));
  // the operator product and the shift in one pass where every row fits a lane group
  const bool fused = sizeof(T) == 4 && (M == 16 || M == 32) && g->max_deg <= FL_FUSED_MAXDEG;
  const int fgrid = (int)std::min<int64_t>(FL_BLOCKS, std::max<int64_t>(8, ((n + 15) / 16 + 7) / 8 * 8));
  int it = 0, useful = 0;
  bool open = sm[2] > 0.0;
  for (; it < max_iters && open; ++it) {
    if (fused) {
      KernelStats* ks = nullptr;
      WL_TRY(kstats_begin(ctx, WL_KC_LANCZOS_OP, &ks));
      const float* Vf = reinterpret_cast<const float*>(V);
      const float* drf = reinterpret_cast<const float*>(dre);
      const float* dif = reinterpret_cast<const float*>(dim);
      float* Qf = reinterpret_cast<float*>(Q);
      if (M == 32)
        k_fl_product<16><<<fgrid, 256, 0, ctx->stream>>>(g->rowptr, g->colidx, n, Vf, drf, dif, (float)a,
                                                         (float)b0, (float)b1, s, Qf, W.part.template as<double>());
      else
        k_fl_product<8><<<fgrid, 256, 0, ctx->stream>>>(g->rowptr, g->colidx, n, Vf, drf, dif, (float)a,
                                                        (float)b0, (float)b1, s, Qf, W.part.template as<double>());
      WL_HIP(hipGetLastError());
      // CSR once, V gathered once and read once as its own rows, Q written, d
      WL_TRY(kstats_end(ctx, ks, 4.0 * g->nnz + 4.0 * (n + 1) + 3.0 * 4.0 * n * 2 * M + 8.0 * n));
      k_rk_finish<<<2 * M, RK_THREADS, 0, ctx->stream>>>(fgrid, 2 * M, W.part.template as<double>(),
                                                          W.sums.template as<double>());
    } else {
      ep.Z = V;
      WL_TRY(launch_spmm<T>(g, V, Q, 2 * M, ep, sh));  // Q = A_mu V, V = d (.) p
      k_fl_shift_dot<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, dre, dim, s, V, Q,
                                                              W.part.template as<double>());
      rk_finish<T>(W, 2 * M);
    }
    k_cg_alpha<<<1, 64, 0, ctx->stream>>>(M, sums, st);
    k_fl_xr<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, st->al, Q, R, dre, dim,
                                                     W.part.template as<double>());
    rk_finish<T>(W, 3 * M);
    k_cg_beta<<<1, 64, 0, ctx->stream>>>(M, tol, sums, st);
    k_fl_dir<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, st->al, st->be, dre, dim, R, X, V);
    WL_HIP(hipGetLastError());
    WL_TRY(rk_cg_post<T>(W, it & 1));
    if (it > 0) {  // the previous iteration's summary, read while this one runs
      WL_TRY(rk_cg_read<T>(W, (it - 1) & 1, sm));
      WL_CHECK(sm[3] == 0.0, WL_ENUMERIC, sm[3] == 1.0 ? "rational Krylov: COCG broke down (p^T K p = 0)"
                                                       : "rational Krylov: non-finite residual in the shifted solve");
      if (sm[2] == 0.0) {
        useful = it;
        open = false;
        break;
      }
    }
  }
  if (open && it > 0) {  // the last iteration's summary
    WL_TRY(rk_cg_read<T>(W, (it - 1) & 1, sm));
    WL_CHECK(sm[3] == 0.0, WL_ENUMERIC, sm[3] == 1.0 ? "rational Krylov: COCG broke down (p^T K p = 0)"
                                                     : "rational Krylov: non-finite residual in the shifted solve");
    useful = it;
    open = sm[2] > 0.0;
  } else if (useful == 0) {
    useful = it;
  }
  *iters = useful;
  *res_out = open ? sm[0] : sm[1];
  if (open) {
    wl_set_error("rational Krylov: shifted solve did not reach %g in %d iterations (residual %g)", tol, max_iters,
                 sm[0]);
    return WL_ENOCONV;
  }
  // x = A_mu (d (.) z)
  k_fl_scale<T><<<grid, RK_THREADS, 0, ctx->stream>>>(n, M, dre, dim, X, V);
  WL_HIP(hipGetLastError());
  ep.Z = V;
  WL_TRY(launch_spmm<T>(g, V, Q, 2 * M, ep, sh));
  return WL_OK;
}

template <typename T>
wl_status return_prob_impl(wl_op* op, const T* Om, int M, const double* ts, int nt, double t_max, double rho,
                           double pole_time, double aaa_tol, double solve_tol, int max_iters, double rcond,
                           double* p_hat, double* e_hat, double* poles_out, int poles_cap, wl_rk_info* info) {
  wl_graph* g = op->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  using cd = std::complex<double>;
  WL_TRY(ensure_w<T>(op));
  if (!op->rk) op->rk = new RkCache;
  RkCache& C = *op->rk;
  // work: sparse products times the probe columns they act on (a walk-Laplacian
  // product on b columns is op->K products: Lanczos steps or series degree)
  double products = 0.0;
  if (!(rho > 0.0) && op->d.func == WL_F_RESOLVENT) {
    // A resolvent's phi = s A_mu^{-1} is positive definite, so L = diag(w) - phi <= diag(w)
    // and rho(L) <= max w - s / lambda_max(A_mu), with lambda_max(A_mu) <= b0 + (b1 + |a|)
    // d_max (Gershgorin on A_mu = a A + b0 I + b1 D): an upper bound of the spectrum for
    // the AAA interval without a product
    double a, b0, b1;
    lanczos_params(op, &a, &b0, &b1);
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256));
    DevBuf& part = C.sums;
    WL_TRY(part.ensure((size_t)nb * sizeof(double)));
    k_rk_vmax<T><<<nb, 256, 0, ctx->stream>>>(n, op->w.template as<T>(), part.as<double>());
    WL_HIP(hipGetLastError());
    std::vector<double> hp(nb);
    WL_HIP(hipMemcpyAsync(hp.data(), part.p, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    const double wmax = *std::max_element(hp.begin(), hp.end());
    const double lam_a = b0 + (b1 + std::fabs(a)) * (double)g->max_deg;
    WL_CHECK(std::isfinite(wmax) && lam_a > 0.0, WL_ENUMERIC, "wl_return_prob: bad walk degrees for the bound of rho");
    rho = std::max(0.0, wmax - b0 / lam_a);
  } else if (!(rho > 0.0)) {
    WL_TRY(laplacian_rho_impl<T>(op, 40, 0x5eed, &rho));
    products += 40.0 * op->K;
  }
  std::vector<cd> poles;
  double aaa_err = 0.0;
  // with t_max rho <= aaa_tol, 1 - e^{-x} <= x keeps exp(-x) within the tolerance of the
  // constant 1 on the whole interval: no poles (L = 0, a graph without edges, included),
  // the space is Omega's alone
  if (t_max * rho > aaa_tol && exp_poles(t_max * rho, aaa_tol, 100, poles, &aaa_err)) {
    wl_set_error("wl_return_prob: AAA failed");
    return WL_ENOCONV;
  }
  for (auto& p : poles) p /= pole_time;
  // real poles and one representative (Im > 0) per conjugate pair
  const double itol = 1e-10;
  std::vector<cd> reps;
  int npos = 0, nneg = 0;
  for (const cd& p : poles) {
    if (std::fabs(p.imag()) <= itol * std::abs(p)) {
      reps.push_back(cd(p.real(), 0.0));
    } else if (p.imag() > 0) {
      reps.push_back(p);
      ++npos;
    } else {
      ++nneg;
    }
  }
  if (npos != nneg) {
    wl_set_error("wl_return_prob: AAA poles are not closed under conjugation");
    return WL_ENUMERIC;
  }
  int nb_max = 1;
  for (const cd& p : reps) nb_max += p.imag() == 0.0 ? 1 : 2;
  // Lanczos operators in FP32: the blocks are padded to a multiple of 16 columns (zero
  // columns, which deflate) so that every product runs as 16-column groups in lock
  // step instead of one wide block Lanczos process (whose small-matrix work grows
  // with the square of the width)
  const bool grouped = op->d.prec == WL_FP32 && op->d.method == WL_M_LANCZOS;
  const int Mp = grouped ? (M + 15) / 16 * 16 : M;
  RkWork<T> W(C);
  W.op = op;
  W.ctx = ctx;
  W.n = n;
  W.M = Mp;
  if (grouped && C.groups_mp != Mp) {  // made once per padded width, kept with the operator
    C.drop_groups();
    WL_TRY(multi_groups_create(op, 2 * Mp / 16, &C.groups_wide));
    WL_TRY(multi_groups_create(op, Mp / 16, &C.groups_narrow));
    C.groups_mp = Mp;
  }
  // resolvents: shifted solves on the symmetrised system (one sparse product per
  // iteration); other operators: COCG with the walk-Laplacian product itself
  const bool flat = op->d.func == WL_F_RESOLVENT;
  DevBuf &basis = C.basis, &wb = C.wb, &X = C.X, &R = C.R, &P = C.P, &Q = C.Q, &V = C.V, &dd = C.dd;
  const size_t blk = (size_t)n * Mp;
  WL_TRY(basis.ensure((size_t)nb_max * blk * sizeof(T)));
  WL_TRY(wb.ensure(blk * sizeof(T)));
  WL_TRY(X.ensure(2 * blk * sizeof(T)));
  WL_TRY(R.ensure(2 * blk * sizeof(T)));
  if (!flat) WL_TRY(P.ensure(2 * blk * sizeof(T)));
  WL_TRY(Q.ensure(2 * blk * sizeof(T)));
  if (flat) {
    WL_TRY(V.ensure(2 * blk * sizeof(T)));
    WL_TRY(dd.ensure(2 * (size_t)n * sizeof(T)));
  }
  WL_TRY(W.dsmall.ensure((size_t)nb_max * Mp * Mp * 8));
  WL_TRY(W.part.ensure((size_t)std::max(RK_BLOCKS * 3, FL_BLOCKS * 2) * Mp * 8));
  WL_TRY(W.sums.ensure((size_t)3 * Mp * 8));
  WL_TRY(W.cg.ensure(sizeof(CgState)));
  W.basis = basis.as<T>();
  const int eg = (int)std::min<int64_t>(4096, (2 * (int64_t)blk + 255) / 256);
  // V_0 R0 = Omega (padded)
  std::vector<double> R0;
  k_rk_pad<T><<<eg, 256, 0, ctx->stream>>>(n, M, Mp, Om, wb.as<T>());
  WL_HIP(hipGetLastError());
  WL_TRY(rk_append<T>(W, wb.as<T>(), &R0));
  int iters_total = 0, iters_max = 0, solves = 0;
  double worst = 0.0;
  for (const cd& xi : reps) {
    const T* U = W.basis + (size_t)(W.nb - 1) * blk;  // continuation: the last block
    int its = 0;
    double res = 0.0;
    if (flat)
      WL_TRY(rk_solve_flat<T>(W, xi, U, X.as<T>(), R.as<T>(), Q.as<T>(), V.as<T>(), dd.as<T>(),
                              dd.as<T>() + n, solve_tol, max_iters, &its, &res));
    else
      WL_TRY(rk_solve<T>(W, xi, U, X.as<T>(), R.as<T>(), P.as<T>(), Q.as<T>(), solve_tol, max_iters, &its, &res));
    const T* sol = flat ? Q.as<T>() : X.as<T>();
    products += flat ? 2.0 * M * (its + 1) : 2.0 * M * its * op->K;
    ++solves;
    iters_total += its;
    iters_max = std::max(iters_max, its);
    worst = std::max(worst, res);
    for (int part = 0; part < (xi.imag() != 0.0 ? 2 : 1); ++part) {
      k_rk_part<T><<<eg, 256, 0, ctx->stream>>>(n, Mp, sol, part, wb.as<T>());
      WL_HIP(hipGetLastError());
      WL_TRY(rk_append<T>(W, wb.as<T>(), nullptr));
    }
  }
  // T = V^T L V, one column block per basis block, symmetrised
  const int nb = W.nb, m = nb * Mp;
  std::vector<double> Tm((size_t)m * m), col;
  for (int j = 0; j < nb; ++j) {
    const T* Vj = W.basis + (size_t)j * blk;
    WL_TRY(rk_apply<T>(W, Vj, Mp, wb.as<T>()));
    WL_TRY(rk_gram<T>(W, W.basis, nb, wb.as<T>(), col));
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < Mp; ++c) Tm[(size_t)r * m + j * Mp + c] = col[(size_t)r * Mp + c];
  }
  for (int r = 0; r < m; ++r)
    for (int c = r + 1; c < m; ++c) {
      const double v = 0.5 * (Tm[(size_t)r * m + c] + Tm[(size_t)c * m + r]);
      Tm[(size_t)r * m + c] = Tm[(size_t)c * m + r] = v;
    }
  products += (double)nb * M * op->K;
  // T = S diag(lam) S^T in factored form; only Z = S^T E_1 R0 enters (m x M: the probe
  // columns, not the padding)
  SymEig E;
  if (sym_eig_factor(m, Tm.data(), E)) {
    wl_set_error("wl_return_prob: eigendecomposition of the projected matrix failed");
    return WL_ENOCONV;
  }
  const std::vector<double>& lam = E.lam;
  std::vector<double> Z((size_t)m * M, 0.0);
  for (int r = 0; r < Mp; ++r)
    for (int c = 0; c < M; ++c) Z[(size_t)r * M + c] = R0[(size_t)r * Mp + c];
  sym_eig_apply_ut(E, M, Z.data());
  // the times are independent (Alg. 1 runs them as a parallel loop): host threads
  const double inv_n = 1.0 / (double)n;
  const int nth = std::max(1, std::min({nt, 16, (int)std::max(1u, std::thread::hardware_concurrency())}));
  std::vector<char> failed(nth, 0);
  auto estimate_times = [&](int tid) {
    std::vector<double> H((size_t)M * M), G((size_t)M * M), e1(m), e2(m);
    for (int k = tid; k < nt; k += nth) {
      for (int e = 0; e < m; ++e) {
        e1[e] = std::exp(-ts[k] * lam[e]) * inv_n;
        e2[e] = e1[e] * e1[e];
      }
      for (int i = 0; i < M; ++i)
        for (int c = i; c < M; ++c) {
          double h = 0.0, gg = 0.0;
          for (int e = 0; e < m; ++e) {
            const double zz = Z[(size_t)e * M + i] * Z[(size_t)e * M + c];
            h += zz * e1[e];
            gg += zz * e2[e];
          }
          H[(size_t)i * M + c] = H[(size_t)c * M + i] = h;
          G[(size_t)i * M + c] = G[(size_t)c * M + i] = gg;
        }
      double tr = 0.0, te = 0.0;
      if (xnys_trace_host(M, H, G, rcond, &tr, &te)) {
        failed[tid] = 1;
        return;
      }
      if (p_hat) p_hat[k] = tr;
      if (e_hat) e_hat[k] = te;
    }
  };
  std::vector<std::thread> pool;
  int started = 1;
  try {
    for (; started < nth; ++started) pool.emplace_back(estimate_times, started);
  } catch (...) {  // no thread to be had: the caller's thread takes the rest
  }
  estimate_times(0);
  for (auto& th : pool) th.join();
  for (int tid = started; tid < nth; ++tid) estimate_times(tid);
  for (char f : failed)
    if (f) {
      wl_set_error("wl_return_prob: eigendecomposition of a Nystrom core failed");
      return WL_ENOCONV;
    }
  if (poles_out)
    for (int i = 0; i < (int)poles.size() && i < poles_cap; ++i) {
      poles_out[2 * i] = poles[i].real();
      poles_out[2 * i + 1] = poles[i].imag();
    }
  if (info) {
    info->npoles = (int32_t)poles.size();
    info->nblocks = nb;
    info->solves = solves;
    info->iters_total = iters_total;
    info->iters_max = iters_max;
    info->rho = rho;
    info->aaa_err = aaa_err;
    info->solve_res = worst;
    info->products = products;
  }
  return WL_OK;
}

wl_status copy_poles(const std::vector<std::complex<double>>& poles, double* out, int32_t cap, int32_t* npoles) {
  if (npoles) *npoles = (int32_t)poles.size();
  if (out)
    for (int i = 0; i < (int)poles.size() && i < cap; ++i) {
      out[2 * i] = poles[i].real();
      out[2 * i + 1] = poles[i].imag();
    }
  return WL_OK;
}

}  // namespace

extern "C" {

wl_status wl_aaa(int64_t N, const double* Z, const double* F, double tol, int32_t mmax, double* poles, int32_t cap,
                 int32_t* npoles, double* max_err) {
  WL_CHECK(N >= 2 && Z && F, WL_EINVAL, "wl_aaa: need N >= 2 points and values");
  WL_CHECK(mmax >= 1 && mmax <= 500, WL_EINVAL, "wl_aaa: mmax must lie in [1, 500]");
  WL_CHECK(tol >= 0.0, WL_EINVAL, "wl_aaa: tol must be >= 0");
  WL_CHECK(cap >= 0 && (cap == 0 || poles), WL_EINVAL, "wl_aaa: bad pole buffer");
  for (int64_t i = 0; i < N; ++i)
    WL_CHECK(std::isfinite(Z[i]) && std::isfinite(F[i]), WL_EINVAL, "wl_aaa: non-finite sample");
  std::vector<double> z, f, w;
  WL_CHECK(aaa_real(N, Z, F, tol, mmax, z, f, w, max_err) == 0, WL_ENOCONV, "wl_aaa: failed");
  std::vector<std::complex<double>> p;
  aaa_poles(z, w, p);
  return copy_poles(p, poles, cap, npoles);
}

wl_status wl_exp_poles(double xmax, double tol, int32_t mmax, double* poles, int32_t cap, int32_t* npoles,
                       double* max_err) {
  WL_CHECK(xmax > 0.0 && std::isfinite(xmax), WL_EINVAL, "wl_exp_poles: xmax must be positive");
  WL_CHECK(mmax >= 1 && mmax <= 500, WL_EINVAL, "wl_exp_poles: mmax must lie in [1, 500]");
  WL_CHECK(cap >= 0 && (cap == 0 || poles), WL_EINVAL, "wl_exp_poles: bad pole buffer");
  std::vector<std::complex<double>> p;
  WL_CHECK(exp_poles(xmax, tol, mmax, p, max_err) == 0, WL_ENOCONV, "wl_exp_poles: AAA failed");
  return copy_poles(p, poles, cap, npoles);
}

wl_status wl_return_prob(wl_op* op, const void* d_Omega, int32_t M, const double* t, int32_t nt, double t_max,
                         double rho, double pole_time, double aaa_tol, double solve_tol, int32_t max_iters,
                         double rcond, double* p_hat, double* e_hat, double* poles, int32_t poles_cap,
                         wl_rk_info* info) {
  WL_CHECK(op, WL_EINVAL, "wl_return_prob: op is null");
  WL_CHECK(M >= 2 && M <= RK_MAXM, WL_EINVAL, "wl_return_prob: M must lie in [2, %d]", RK_MAXM);
  WL_CHECK(d_Omega, WL_EINVAL, "wl_return_prob: Omega is null");
  WL_CHECK(nt >= 0 && (nt == 0 || t), WL_EINVAL, "wl_return_prob: bad time list");
  for (int k = 0; k < nt; ++k)
    WL_CHECK(std::isfinite(t[k]) && t[k] >= 0.0, WL_EINVAL, "wl_return_prob: times must be finite and >= 0");
  WL_CHECK(t_max > 0.0 && std::isfinite(t_max), WL_EINVAL, "wl_return_prob: t_max must be positive");
  WL_CHECK(pole_time > 0.0 && std::isfinite(pole_time), WL_EINVAL, "wl_return_prob: pole_time must be positive");
  WL_CHECK(std::isfinite(rho), WL_EINVAL, "wl_return_prob: rho must be finite (<= 0: estimate it)");
  WL_CHECK(aaa_tol > 0.0 && solve_tol > 0.0 && solve_tol < 1.0, WL_EINVAL, "wl_return_prob: bad tolerances");
  WL_CHECK(max_iters >= 1, WL_EINVAL, "wl_return_prob: max_iters must be >= 1");
  WL_CHECK(rcond >= 0.0 && rcond < 1.0, WL_EINVAL, "wl_return_prob: rcond must lie in [0, 1)");
  WL_CHECK(poles_cap >= 0 && (poles_cap == 0 || poles), WL_EINVAL, "wl_return_prob: bad pole buffer");
  WL_CHECK(op->g->n > M, WL_EINVAL, "wl_return_prob: needs n > M");
  DeviceGuard dg(op->g->ctx->device);
  if (op->d.prec == WL_FP32)
    return return_prob_impl<float>(op, (const float*)d_Omega, M, t, nt, t_max, rho, pole_time, aaa_tol, solve_tol,
                                   max_iters, rcond, p_hat, e_hat, poles, poles_cap, info);
  return return_prob_impl<double>(op, (const double*)d_Omega, M, t, nt, t_max, rho, pole_time, aaa_tol, solve_tol,
                                  max_iters, rcond, p_hat, e_hat, poles, poles_cap, info);
}

}  // extern "C"
