// Block kernels for several independent Lanczos processes run side by side.
//
// ng blocks of width gb are interleaved in one n x (ng gb) row-major block: row r holds
// group 0's gb values, then group 1's, ...  One sparse product then gathers every
// group's row segment of a neighbour from the same cache lines (two 16-wide FP32
// groups fill a 128-byte line that a single group would use half of).  The Gram and
// basis-update kernels below read and write that layout directly, so each group's
// Lanczos step (Sec. 4.1: projection, CholQR) costs one pass over the wide block
// instead of one per group, and the small matrices of all groups are factorised by
// one launch.
//
//   * gb = 16, FP32: matrix cores.  A wave takes 16-row chunks.  For the basis update
//     lane l loads row l % 16, columns 4 (l / 16) .. + 3 of the group (16 bytes) as
//     the A operand of v_mfma_f32_16x16x4f32 (step s uses the s-th float, i.e. the
//     columns {4 g + s}), with the matching rows of C from a lane-ordered LDS copy as
//     the B operand; the result rows 4 (l / 16) + v, column l % 16, are exactly the
//     operands of the FP64 Gram v_mfma_f64_16x16x4f64 (step v sums rows {4 g + v}).
//     The Gram kernel loads its operands in that same row-interleaved layout.
//   * gb = 1: scalar kernels, one row per lane, all groups of the row together.
// Partial sums are written per workgroup as [part][group][block][entry] and reduced
// by one finalize launch in a fixed order (deterministic).
#include <algorithm>

#include "wl_internal.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int G1_MAXG = 8;   // groups of single columns
constexpr int G1_MAXK = 64;  // blocks combined by one single-column update
constexpr int G16_MAXG = 4;  // 16-wide groups per workgroup (accumulator registers)
constexpr int G16_LDS_KB = 120;  // gfx950: up to 160 KiB of LDS per workgroup
constexpr int G16_SPLIT = 12;    // blocks per slice of a long combination (see launch_gupdate)

// ------------------------------------------------------------------ gb = 16 (FP32)

template <int NB, int NG>
__global__ __launch_bounds__(256) void k_ggram16(int64_t n, const float* __restrict__ X, int64_t sX,
                                                 const float* __restrict__ Y, int ld, int ngt,
                                                 double* __restrict__ partials, const double* __restrict__ skip,
                                                 int64_t gs) {
  const int qb = blockIdx.y * NG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  bool act[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) act[q] = qb + q < ngt && !(skip && skip[(int64_t)(qb + q) * gs] != 0.0);
  v4d acc[NG][NB];
#pragma unroll
  for (int q = 0; q < NG; ++q)
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[q][k] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t nchunks = (n + 15) / 16;
  for (int64_t ch = (int64_t)blockIdx.x * 4 + wave; ch < nchunks; ch += (int64_t)gridDim.x * 4) {
    const int64_t r0 = ch * 16;
    // every operand of the chunk is requested before the first product: addresses are
    // clamped into the block (rows past n, groups past the last) instead of branching
    // around the loads, and rows past n get a zero Y operand
    float y[NG][4], x[NG][NB][4];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const int64_t col = (int64_t)min(qb + q, ngt - 1) * 16 + c;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = min(r0 + 4 * g + v, n - 1);
        y[q][v] = Y[row * ld + col];
#pragma unroll
        for (int k = 0; k < NB; ++k) x[q][k][v] = X[(int64_t)k * sX + row * ld + col];
      }
    }
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      if (!act[q]) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double yd = r0 + 4 * g + v < n ? (double)y[q][v] : 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k)
          acc[q][k] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)x[q][k][v], yd, acc[q][k], 0, 0, 0);
      }
    }
  }
  __shared__ double red[NG * NB * 256];
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int q = 0; q < NG; ++q)
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int idx = (q * NB + k) * 256 + (4 * v + g) * 16 + c;  // FP64 16x16x4 output layout
            red[idx] = (w == 0 ? 0.0 : red[idx]) + acc[q][k][v];
          }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NG * NB * 256; e += 256) {
    const int q = e / (NB * 256);
    if (qb + q < ngt)
      partials[((int64_t)blockIdx.x * ngt + qb + q) * NB * 256 + (e - q * NB * 256)] = red[e];
  }
}

// NBF: the number of blocks when it is 1..4 (operands held in registers, no loads past
// the last block), 0 for any other count
template <bool GRAM, int NG, int NBF>
__global__ __launch_bounds__(256) void k_gupdate16(int64_t n, const float* X, int64_t sX, int nblk, int ld, int ngt,
                                                   const double* __restrict__ C, int64_t cs, const float* Yin,
                                                   double alpha, const float* __restrict__ wv, double beta,
                                                   float* Out, double* __restrict__ partials,
                                                   const double* __restrict__ skip,
                                                   const double* __restrict__ skip_gram, int64_t gs) {
  extern __shared__ float4 sCl[];  // [NG][nblk][64] lane-ordered B operands
  __shared__ double red[NG * 256];
  __shared__ __align__(16) float sT[4][16 * 20];  // per wave: a 16 x 16 result tile (row stride 20)
  const int qb = blockIdx.y * NG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  bool act[NG], gact[NG];
  bool any = false;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int64_t qq = qb + q;
    act[q] = qq < ngt && !(skip && skip[qq * gs] != 0.0);
    gact[q] = GRAM && act[q] && !(skip_gram && skip_gram[qq * gs] != 0.0);
    any = any || act[q];
  }
  if (!any) return;  // uniform over the workgroup
  for (int e = threadIdx.x; e < NG * nblk * 64; e += 256) {
    const int q = e / (nblk * 64), rem = e - q * nblk * 64;
    const int k = rem >> 6, l = rem & 63, gg = l >> 4, cc = l & 15;
    if (qb + q < ngt) {
      const double* Ck = C + (int64_t)(qb + q) * cs + (int64_t)k * 256 + (4 * gg) * 16 + cc;
      sCl[e] = make_float4((float)Ck[0], (float)Ck[16], (float)Ck[32], (float)Ck[48]);
    }
  }
  __syncthreads();
  const float tb = (float)beta, ta = (float)alpha;
  v4d gacc[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) gacc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t nchunks = (n + 15) / 16;
  constexpr bool few = NBF > 0;  // every operand of a chunk fits in registers
  for (int64_t ch = (int64_t)blockIdx.x * 4 + wave; ch < nchunks; ch += (int64_t)gridDim.x * 4) {
    const int64_t r0 = ch * 16;
    const bool okA = r0 + c < n;
    // with few blocks, all groups' operands of the chunk are requested before the first
    // product (addresses clamped into the block, rows past n zeroed)
    float4 xs[NG][NBF > 0 ? NBF : 1];
    if constexpr (few) {
      const int64_t rA = min(r0 + c, n - 1);
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        const float* xa = X + rA * ld + (int64_t)min(qb + q, ngt - 1) * 16 + 4 * g;
#pragma unroll
        for (int u = 0; u < NBF; ++u) {
          const float4 t = *reinterpret_cast<const float4*>(xa + (int64_t)u * sX);
          xs[q][u] = okA ? t : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      if (!act[q]) continue;
      const int64_t colq = (int64_t)(qb + q) * 16;
      const float* xa = X + (r0 + c) * ld + colq + 4 * g;
      const float4* cl = sCl + (int64_t)q * nblk * 64 + lane;
      v4f d = {0.f, 0.f, 0.f, 0.f};
      if constexpr (few) {
#pragma unroll
        for (int u = 0; u < NBF; ++u) {
          const float4 bq = cl[u * 64];
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[q][u].x, bq.x, d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[q][u].y, bq.y, d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[q][u].z, bq.z, d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[q][u].w, bq.w, d, 0, 0, 0);
        }
      }
      for (int k0 = 0; !few && k0 < nblk; k0 += 8) {  // eight blocks' loads in flight
        float4 x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          x[u] = (okA && k0 + u < nblk) ? *reinterpret_cast<const float4*>(xa + (int64_t)(k0 + u) * sX)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (k0 + u >= nblk) break;
          const float4 bq = cl[(k0 + u) * 64];
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u].x, bq.x, d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u].y, bq.y, d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u].z, bq.z, d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u].w, bq.w, d, 0, 0, 0);
        }
      }
      float o[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) o[v] = tb * d[v];
      if (Yin) {  // clamped loads, zero weight past n
        float yv[4], wq[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = min(r0 + 4 * g + v, n - 1);
          yv[v] = Yin[row * ld + colq + c];
          wq[v] = wv ? wv[row * ngt + qb + q] : ta;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (r0 + 4 * g + v < n) o[v] += wq[v] * yv[v];
      }
      if (gact[q]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double ov = (double)o[v];
          gacc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ov, ov, gacc[q], 0, 0, 0);
        }
      }
      // through the wave's LDS tile to row order: lane l stores row l / 4, columns
      // 4 (l % 4) .. + 3 as one 16-byte write
#pragma unroll
      for (int v = 0; v < 4; ++v) sT[wave][(4 * g + v) * 20 + c] = o[v];
      __builtin_amdgcn_wave_barrier();
      {
        const int rr = lane >> 2, cc = (lane & 3) * 4;
        const float4 t = *reinterpret_cast<const float4*>(&sT[wave][rr * 20 + cc]);
        if (r0 + rr < n) *reinterpret_cast<float4*>(Out + (r0 + rr) * ld + colq + cc) = t;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (!GRAM) return;
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int q = 0; q < NG; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int idx = q * 256 + (4 * v + g) * 16 + c;
          red[idx] = (w == 0 ? 0.0 : red[idx]) + gacc[q][v];
        }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NG * 256; e += 256) {
    const int q = e >> 8;
    if (qb + q < ngt) partials[((int64_t)blockIdx.x * ngt + qb + q) * 256 + (e & 255)] = red[e];
  }
}

// ------------------------------------------------------------------ gb = 1

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_ggram1(int64_t n, const T* __restrict__ X, int64_t sX,
                                                const T* __restrict__ Y, int ngt, double* __restrict__ partials,
                                                const double* __restrict__ skip, int64_t gs) {
  double acc[NB][G1_MAXG];
#pragma unroll
  for (int k = 0; k < NB; ++k)
#pragma unroll
    for (int q = 0; q < G1_MAXG; ++q) acc[k][q] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int q = 0; q < G1_MAXG; ++q) {
      if (q >= ngt) break;
      const double y = (double)Y[r * ngt + q];
#pragma unroll
      for (int k = 0; k < NB; ++k) acc[k][q] += (double)X[(int64_t)k * sX + r * ngt + q] * y;
    }
  }
  __shared__ double red[4][NB * G1_MAXG];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NB; ++k)
#pragma unroll
    for (int q = 0; q < G1_MAXG; ++q) {
      const double v = wave_sum_d(acc[k][q]);
      if (lane == 0) red[wave][k * G1_MAXG + q] = v;
    }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < NB * ngt) {
    const int q = t / NB, k = t - q * NB;
    double v = 0.0;
    if (!(skip && skip[(int64_t)q * gs] != 0.0)) {
      const int i = k * G1_MAXG + q;
      v = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
    }
    partials[((int64_t)blockIdx.x * ngt + q) * NB + k] = v;
  }
}

template <typename T, bool GRAM>
__global__ __launch_bounds__(256) void k_gupdate1(int64_t n, const T* X, int64_t sX, int nblk, int ngt,
                                                  const double* __restrict__ C, int64_t cs, const T* Yin,
                                                  double alpha, const T* __restrict__ wv, double beta, T* Out,
                                                  double* __restrict__ partials, const double* __restrict__ skip,
                                                  const double* __restrict__ skip_gram, int64_t gs) {
  __shared__ T sC[G1_MAXG * G1_MAXK];
  bool act[G1_MAXG], gact[G1_MAXG];
#pragma unroll
  for (int q = 0; q < G1_MAXG; ++q) {
    act[q] = q < ngt && !(skip && skip[(int64_t)q * gs] != 0.0);
    gact[q] = GRAM && act[q] && !(skip_gram && skip_gram[(int64_t)q * gs] != 0.0);
  }
  for (int e = threadIdx.x; e < ngt * nblk; e += 256) {
    const int q = e / nblk, k = e - q * nblk;
    sC[q * G1_MAXK + k] = (T)C[(int64_t)q * cs + k];
  }
  __syncthreads();
  const T tb = (T)beta, ta = (T)alpha;
  double dot[G1_MAXG];
#pragma unroll
  for (int q = 0; q < G1_MAXG; ++q) dot[q] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int q = 0; q < G1_MAXG; ++q) {
      if (q >= ngt) break;
      if (!act[q]) continue;
      T acc = T(0);
      for (int k = 0; k < nblk; ++k) acc += X[(int64_t)k * sX + r * ngt + q] * sC[q * G1_MAXK + k];
      T o = tb * acc;
      if (Yin) o += (wv ? wv[r * ngt + q] : ta) * Yin[r * ngt + q];
      Out[r * ngt + q] = o;
      if (gact[q]) dot[q] += (double)o * (double)o;
    }
  }
  if (!GRAM) return;
  __shared__ double red[4][G1_MAXG];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < G1_MAXG; ++q) {
    const double v = wave_sum_d(dot[q]);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < ngt) {
    const int q = threadIdx.x;
    partials[(int64_t)blockIdx.x * ngt + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
}

// ------------------------------------------------------------------ shared

// out[q gs + k E + e] = sum over parts of partials[part][q][k][e]; 16 entries x 16
// phases per workgroup, eight loads in flight per thread.  Groups with a set skip
// flag are left alone.
__global__ __launch_bounds__(256) void k_gfinalize(const double* __restrict__ partials, int nparts, int ngt,
                                                   int nblk, int E, double* __restrict__ out, int64_t gs,
                                                   const double* __restrict__ skip, int dg, int gb) {
  __shared__ double s[256];
  const int t = threadIdx.x, el = t & 15, p = t >> 4;
  const int64_t tot = (int64_t)ngt * nblk * E;
  const int64_t ent = (int64_t)blockIdx.x * 16 + el;
  bool live = ent < tot;
  int q = 0;
  if (live) {
    q = (int)(ent / ((int64_t)nblk * E));
    live = !(skip && skip[(int64_t)q * gs] != 0.0);
  }
  double v = 0.0;
  if (live) {
    double u[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int part = p;
    for (; part + 7 * 16 < nparts; part += 8 * 16) {
#pragma unroll
      for (int i = 0; i < 8; ++i) u[i] += partials[(int64_t)(part + i * 16) * tot + ent];
    }
    for (; part < nparts; part += 16) u[0] += partials[(int64_t)part * tot + ent];
    v = ((u[0] + u[1]) + (u[2] + u[3])) + ((u[4] + u[5]) + (u[6] + u[7]));
  }
  s[t] = v;
  __syncthreads();
  for (int h = 8; h > 0; h >>= 1) {
    if (p < h) s[t] += s[t + h * 16];
    __syncthreads();
  }
  if (p == 0 && live) {
    const int64_t rem = ent - (int64_t)q * nblk * E;
    double v0 = s[t];
    if (q == dg) {  // group of independent single columns: cross terms do not exist
      const int e = (int)(rem % E);
      if (e / gb != e % gb) v0 = 0.0;
    }
    out[(int64_t)q * gs + rem] = v0;
  }
}

__global__ void k_dcopy_groups(int ng, int count, const double* __restrict__ x, double* __restrict__ y,
                               int64_t gs) {
  for (int e = threadIdx.x; e < count; e += blockDim.x) y[(int64_t)blockIdx.x * gs + e] = x[(int64_t)blockIdx.x * gs + e];
}

template <typename T>
__global__ void k_group_copy(int64_t n, int b, int ng, int q, const T* __restrict__ X, T* __restrict__ Y,
                             int into_group) {
  const int64_t total = n * b;
  const int64_t wd = (int64_t)ng * b;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / b;
    const int c = (int)(i - r * b);
    if (into_group)
      Y[r * wd + (int64_t)q * b + c] = X[i];
    else
      Y[i] = X[r * wd + (int64_t)q * b + c];
  }
}

int gparts(int64_t work, int cap) {
  int64_t p = work;
  if (p > cap) p = cap;
  if (p < 1) p = 1;
  return (int)p;
}

template <int NB>
void launch_ggram16_nb(wl_ctx* ctx, dim3 grid, int ngchunk, int64_t n, const float* X, int64_t sX, const float* Y,
                       int ld, int ng, double* pp, const double* skip, int64_t gs) {
  if (ngchunk == 1)
    hipLaunchKernelGGL((k_ggram16<NB, 1>), grid, dim3(256), 0, ctx->stream, n, X, sX, Y, ld, ng, pp, skip, gs);
  else if (ngchunk == 2)
    hipLaunchKernelGGL((k_ggram16<NB, 2>), grid, dim3(256), 0, ctx->stream, n, X, sX, Y, ld, ng, pp, skip, gs);
  else
    hipLaunchKernelGGL((k_ggram16<NB, 4>), grid, dim3(256), 0, ctx->stream, n, X, sX, Y, ld, ng, pp, skip, gs);
}

template <bool GRAM, int NG, int NBF>
void launch_gupdate16_k(wl_ctx* ctx, dim3 grid, size_t lds, int64_t n, const float* X, int64_t sX, int nblk, int ld,
                        int ng, const double* C, int64_t cs, const float* Yin, double alpha, const float* wv,
                        double beta, float* Out, double* pp, const double* skip, const double* skip_gram,
                        int64_t gs) {
  static bool lds_set = false;  // once per instantiation and process (the attribute is per function)
  if (!lds_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_gupdate16<GRAM, NG, NBF>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, G16_LDS_KB * 1024);
    lds_set = true;
  }
  hipLaunchKernelGGL((k_gupdate16<GRAM, NG, NBF>), grid, dim3(256), lds, ctx->stream, n, X, sX, nblk, ld, ng, C,
                     cs, Yin, alpha, wv, beta, Out, pp, skip, skip_gram, gs);
}

template <bool GRAM, int NG>
void launch_gupdate16_nb(wl_ctx* ctx, dim3 grid, size_t lds, int64_t n, const float* X, int64_t sX, int nblk, int ld,
                         int ng, const double* C, int64_t cs, const float* Yin, double alpha, const float* wv,
                         double beta, float* Out, double* pp, const double* skip, const double* skip_gram,
                         int64_t gs) {
  switch (nblk) {
    case 1: return launch_gupdate16_k<GRAM, NG, 1>(ctx, grid, lds, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv,
                                                   beta, Out, pp, skip, skip_gram, gs);
    case 2: return launch_gupdate16_k<GRAM, NG, 2>(ctx, grid, lds, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv,
                                                   beta, Out, pp, skip, skip_gram, gs);
    case 3: return launch_gupdate16_k<GRAM, NG, 3>(ctx, grid, lds, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv,
                                                   beta, Out, pp, skip, skip_gram, gs);
    case 4: return launch_gupdate16_k<GRAM, NG, 4>(ctx, grid, lds, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv,
                                                   beta, Out, pp, skip, skip_gram, gs);
    default: return launch_gupdate16_k<GRAM, NG, 0>(ctx, grid, lds, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv,
                                                    beta, Out, pp, skip, skip_gram, gs);
  }
}

template <bool GRAM>
void launch_gupdate16_ng(wl_ctx* ctx, dim3 grid, size_t lds, int ngchunk, int64_t n, const float* X, int64_t sX,
                         int nblk, int ld, int ng, const double* C, int64_t cs, const float* Yin, double alpha,
                         const float* wv, double beta, float* Out, double* pp, const double* skip,
                         const double* skip_gram, int64_t gs) {
  if (ngchunk == 1)
    launch_gupdate16_nb<GRAM, 1>(ctx, grid, lds, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv, beta, Out, pp, skip,
                                 skip_gram, gs);
  else if (ngchunk == 2)
    launch_gupdate16_nb<GRAM, 2>(ctx, grid, lds, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv, beta, Out, pp, skip,
                                 skip_gram, gs);
  else
    launch_gupdate16_nb<GRAM, 4>(ctx, grid, lds, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv, beta, Out, pp, skip,
                                 skip_gram, gs);
}

// groups per workgroup for the 16-wide kernels: a power of two <= 4 whose operands fit
int group_chunk(int ng, int nblk) {
  int c = G16_MAXG;
  while (c > 1 && (c > ng || c * nblk > G16_LDS_KB)) c >>= 1;
  return c;
}

}  // namespace

bool grouped_supported(int prec, int gb, int ng) {
  if (ng < 1) return false;
  if (gb == 16) return prec == WL_FP32;
  if (gb == 1) return ng <= G1_MAXG;
  return false;
}

template <typename T>
wl_status launch_ggram(wl_ctx* ctx, int64_t n, int gb, int ng, const T* X, int64_t sX, int nblk, const T* Y,
                       double* out, int64_t gs, const double* skip, int dg) {
  WL_CHECK(grouped_supported(prec_of<T>(), gb, ng), WL_EUNSUPPORTED, "grouped Gram: unsupported group shape");
  WL_CHECK(nblk >= 1 && nblk <= 3, WL_EINVAL, "grouped Gram: 1..3 blocks");
  if (n == 0) return WL_OK;
  const int E = gb * gb;
  int nparts = 1;
  if constexpr (sizeof(T) == 4) {
    if (gb == 16) {
      const int ngc = group_chunk(ng, 1);
      nparts = gparts(((n + 15) / 16 + 15) / 16, 1024);
      WL_TRY(ctx->partials.ensure((size_t)nparts * ng * nblk * E * sizeof(double)));
      const dim3 grid((unsigned)nparts, (unsigned)((ng + ngc - 1) / ngc));
      double* pp = ctx->partials.as<double>();
      const int ld = ng * 16;
      if (nblk == 1)
        launch_ggram16_nb<1>(ctx, grid, ngc, n, X, sX, Y, ld, ng, pp, skip, gs);
      else if (nblk == 2)
        launch_ggram16_nb<2>(ctx, grid, ngc, n, X, sX, Y, ld, ng, pp, skip, gs);
      else
        launch_ggram16_nb<3>(ctx, grid, ngc, n, X, sX, Y, ld, ng, pp, skip, gs);
      WL_HIP(hipGetLastError());
    }
  }
  if (gb == 1) {
    nparts = gparts((n + 2047) / 2048, 512);
    WL_TRY(ctx->partials.ensure((size_t)nparts * ng * nblk * sizeof(double)));
    double* pp = ctx->partials.as<double>();
    if (nblk == 1)
      hipLaunchKernelGGL((k_ggram1<T, 1>), dim3(nparts), dim3(256), 0, ctx->stream, n, X, sX, Y, ng, pp, skip, gs);
    else if (nblk == 2)
      hipLaunchKernelGGL((k_ggram1<T, 2>), dim3(nparts), dim3(256), 0, ctx->stream, n, X, sX, Y, ng, pp, skip, gs);
    else
      hipLaunchKernelGGL((k_ggram1<T, 3>), dim3(nparts), dim3(256), 0, ctx->stream, n, X, sX, Y, ng, pp, skip, gs);
    WL_HIP(hipGetLastError());
  }
  const int64_t tot = (int64_t)ng * nblk * E;
  hipLaunchKernelGGL(k_gfinalize, dim3((unsigned)((tot + 15) / 16)), dim3(256), 0, ctx->stream,
                     ctx->partials.as<double>(), nparts, ng, nblk, E, out, gs, skip, dg, gb);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_gupdate(wl_ctx* ctx, int64_t n, int gb, int ng, const T* X, int64_t sX, int nblk,
                         const double* C, int64_t cs, const T* Yin, double alpha, const T* wv, double beta, T* Out,
                         double* gram_out, int64_t gs, const double* skip, const double* skip_gram, int dg) {
  WL_CHECK(grouped_supported(prec_of<T>(), gb, ng), WL_EUNSUPPORTED, "grouped update: unsupported group shape");
  WL_CHECK(nblk >= 0 && nblk <= (gb == 1 ? G1_MAXK : G16_LDS_KB), WL_EINVAL, "grouped update: too many blocks");
  WL_CHECK(!(skip && gram_out && skip_gram != skip), WL_EINVAL,
           "grouped update: a skippable update yields a Gram only where it runs (skip_gram = skip)");
  if (n == 0) return WL_OK;
  const int E = gb * gb;
  int nparts = 1;
  if constexpr (sizeof(T) == 4) {
    const bool out_apart = Out + (int64_t)n * ng * 16 <= X || Out >= X + (int64_t)(nblk - 1) * sX + n * ng * 16;
    if (gb == 16 && nblk > G16_SPLIT && !gram_out && !skip && out_apart) {
      // a long combination (a recombination over the whole basis): in slices of
      // G16_SPLIT blocks, each slice adding onto Out, so that a workgroup's staged
      // coefficients stay small enough for several workgroups per CU
      for (int k0 = 0; k0 < nblk; k0 += G16_SPLIT) {
        const int kb = std::min(G16_SPLIT, nblk - k0);
        const bool first = k0 == 0;
        WL_TRY(launch_gupdate<T>(ctx, n, gb, ng, X + (int64_t)k0 * sX, sX, kb, C + (int64_t)k0 * E, cs,
                                 first ? Yin : Out, first ? alpha : 1.0, first ? wv : nullptr, beta, Out, nullptr,
                                 gs, nullptr, nullptr, dg));
      }
      return WL_OK;
    }
    if (gb == 16) {
      const int ngc = group_chunk(ng, std::max(nblk, 1));
      nparts = gparts(((n + 15) / 16 + 15) / 16, 1024);
      const dim3 grid((unsigned)nparts, (unsigned)((ng + ngc - 1) / ngc));
      const size_t lds = (size_t)ngc * nblk * 64 * sizeof(float4);
      const int ld = ng * 16;
      if (gram_out) {
        WL_TRY(ctx->partials.ensure((size_t)nparts * ng * E * sizeof(double)));
        launch_gupdate16_ng<true>(ctx, grid, lds, ngc, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv, beta, Out,
                                  ctx->partials.as<double>(), skip, skip_gram, gs);
      } else {
        launch_gupdate16_ng<false>(ctx, grid, lds, ngc, n, X, sX, nblk, ld, ng, C, cs, Yin, alpha, wv, beta, Out,
                                   nullptr, skip, nullptr, gs);
      }
      WL_HIP(hipGetLastError());
    }
  }
  if (gb == 1) {
    nparts = gparts((n + 1023) / 1024, gram_out ? 512 : 2048);
    if (gram_out) {
      WL_TRY(ctx->partials.ensure((size_t)nparts * ng * sizeof(double)));
      hipLaunchKernelGGL((k_gupdate1<T, true>), dim3(nparts), dim3(256), 0, ctx->stream, n, X, sX, nblk, ng, C, cs,
                         Yin, alpha, wv, beta, Out, ctx->partials.as<double>(), skip, skip_gram, gs);
    } else {
      hipLaunchKernelGGL((k_gupdate1<T, false>), dim3(nparts), dim3(256), 0, ctx->stream, n, X, sX, nblk, ng, C,
                         cs, Yin, alpha, wv, beta, Out, nullptr, skip, nullptr, gs);
    }
    WL_HIP(hipGetLastError());
  }
  if (gram_out) {
    const int64_t tot = (int64_t)ng * E;
    hipLaunchKernelGGL(k_gfinalize, dim3((unsigned)((tot + 15) / 16)), dim3(256), 0, ctx->stream,
                       ctx->partials.as<double>(), nparts, ng, 1, E, gram_out, gs, skip_gram, dg, gb);
    WL_HIP(hipGetLastError());
  }
  return WL_OK;
}

// ------------------------------------------------------------------ deferred normalisation
namespace {

// The basis blocks of the lock-step Lanczos are kept as stored blocks W_j with a factor
// N_j (16 x 16 per group) such that V_j = W_j N_j is orthonormal: the CholQR
// normalisation is folded into the products that read the block instead of a pass over
// it.  All small matrices of a group sit gs doubles apart; N_j at Nb + j 256.

// Identity in every group's N_0.
__global__ void k_eye_groups(double* __restrict__ N0, int64_t gs) {
  const int64_t o = (int64_t)blockIdx.x * gs;
  for (int e = threadIdx.x; e < 256; e += blockDim.x) N0[o + e] = (e >> 4) == (e & 15) ? 1.0 : 0.0;
}

// From the Gram Pt = [W_{j-1} W_j W']^T W' (nbv + 1 blocks of 16 x 16) of the stored blocks:
// P1 = N_{j-1}^T Pt_1, A = sym(N_j^T Pt_2) (the true projections), and the update
// coefficients for the stored blocks Cc = [-N_{j-1} P1; -N_j A; I]; ref = max diag of
// W'^T W' (the block's scale before projection).  One workgroup of 256 per group.
__global__ __launch_bounds__(256) void k_lanczos_proj_deferred(int nbv, const double* __restrict__ P,
                                                               const double* __restrict__ Nprev,
                                                               const double* __restrict__ Ncur,
                                                               double* __restrict__ Aout, double* __restrict__ Cc,
                                                               int64_t gs, double* __restrict__ ref_out) {
  const int64_t go = (int64_t)blockIdx.x * gs;
  P += go;
  Aout += go;
  Cc += go;
  const double* Np = nbv == 2 ? Nprev + go : nullptr;
  const double* Nc = Ncur + go;
  __shared__ double sP1[256], sA[256];
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  const double* Pt1 = P;                       // [W_{j-1}]^T W' (nbv = 2)
  const double* Pt2 = P + (nbv - 1) * 256;     // W_j^T W'
  // true projections: rows of N^T Pt
  double a = 0.0, p1 = 0.0;
  for (int k = 0; k < 16; ++k) {
    a += Nc[k * 16 + i] * Pt2[k * 16 + j];
    if (Np) p1 += Np[k * 16 + i] * Pt1[k * 16 + j];
  }
  sA[t] = a;
  sP1[t] = p1;
  __syncthreads();
  const double as = 0.5 * (sA[i * 16 + j] + sA[j * 16 + i]);
  __syncthreads();
  sA[t] = as;
  Aout[t] = as;
  __syncthreads();
  // Cc blocks for the stored blocks
  double c1 = 0.0, c2 = 0.0;
  for (int k = 0; k < 16; ++k) {
    if (Np) c1 += Np[i * 16 + k] * sP1[k * 16 + j];
    c2 += Nc[i * 16 + k] * sA[k * 16 + j];
  }
  if (nbv == 2) Cc[t] = -c1;
  Cc[(nbv - 1) * 256 + t] = -c2;
  Cc[nbv * 256 + t] = i == j ? 1.0 : 0.0;
  if (t == 0 && ref_out) {
    const double* Gp = P + nbv * 256;
    double m = 0.0;
    for (int d = 0; d < 16; ++d) m = fmax(m, Gp[d * 16 + d]);
    ref_out[go] = m;
  }
}

// After the step's CholQR: N_{j+1} = skip ? Ri1 : Ri2 (the block was normalised
// explicitly by Ri1 only where a second pass was needed), and the three-term
// coefficient of the next product for the stored W_j: Ct = N_j B_j^T (16 x 16).
__global__ __launch_bounds__(256) void k_lanczos_next(const double* __restrict__ skip, const double* __restrict__ Ri1,
                                                      const double* __restrict__ Ri2, const double* __restrict__ Ncur,
                                                      const double* __restrict__ B, double* __restrict__ Nnext,
                                                      double* __restrict__ Ct, int64_t gs) {
  const int64_t go = (int64_t)blockIdx.x * gs;
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  const bool sk = skip[go] != 0.0;
  Nnext[go + t] = sk ? Ri1[go + t] : Ri2[go + t];
  double c = 0.0;
  for (int k = 0; k < 16; ++k) c += Ncur[go + i * 16 + k] * B[go + j * 16 + k];
  Ct[go + t] = c;
}

}  // namespace

wl_status launch_eye_groups(wl_ctx* ctx, int ng, double* N0, int64_t gs) {
  hipLaunchKernelGGL(k_eye_groups, dim3(ng), dim3(256), 0, ctx->stream, N0, gs);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status launch_lanczos_proj_deferred(wl_ctx* ctx, int ng, int nbv, const double* P, const double* Nprev,
                                       const double* Ncur, double* Aout, double* Cc, int64_t gs, double* ref_out) {
  WL_CHECK(nbv == 1 || nbv == 2, WL_EINVAL, "lanczos projection: bad sizes");
  hipLaunchKernelGGL(k_lanczos_proj_deferred, dim3(ng), dim3(256), 0, ctx->stream, nbv, P, Nprev, Ncur, Aout, Cc, gs,
                     ref_out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status launch_lanczos_next(wl_ctx* ctx, int ng, const double* skip, const double* Ri1, const double* Ri2,
                              const double* Ncur, const double* B, double* Nnext, double* Ct, int64_t gs) {
  hipLaunchKernelGGL(k_lanczos_next, dim3(ng), dim3(256), 0, ctx->stream, skip, Ri1, Ri2, Ncur, B, Nnext, Ct, gs);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status launch_dcopy_groups(wl_ctx* ctx, int ng, int count, const double* x, double* y, int64_t gs) {
  if (ng < 1 || count < 1) return WL_OK;
  hipLaunchKernelGGL(k_dcopy_groups, dim3(ng), dim3(256), 0, ctx->stream, ng, count, x, y, gs);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_group_copy(wl_ctx* ctx, int64_t n, int b, int ng, int q, const T* X, T* Y, bool into_group) {
  if (n == 0) return WL_OK;
  const int grid = (int)std::min<int64_t>(8192, (n * b + 255) / 256);
  hipLaunchKernelGGL(k_group_copy<T>, dim3(grid), dim3(256), 0, ctx->stream, n, b, ng, q, X, Y, into_group ? 1 : 0);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

#define WL_INST_GROUPED(T)                                                                                        \
  template wl_status launch_ggram<T>(wl_ctx*, int64_t, int, int, const T*, int64_t, int, const T*, double*,        \
                                     int64_t, const double*, int);                                                 \
  template wl_status launch_gupdate<T>(wl_ctx*, int64_t, int, int, const T*, int64_t, int, const double*, int64_t, \
                                       const T*, double, const T*, double, T*, double*, int64_t, const double*,    \
                                       const double*, int);                                                        \
  template wl_status launch_group_copy<T>(wl_ctx*, int64_t, int, int, int, const T*, T*, bool);
WL_INST_GROUPED(float)
WL_INST_GROUPED(double)
