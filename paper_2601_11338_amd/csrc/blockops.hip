// Tall-skinny block kernels for the Krylov drivers and estimators (gfx950).
//
//  * gram:    X^T Y for n x B blocks (B <= 64), double accumulation.  FP32 blocks of
//             16, 32 or 64 columns use the FP64 matrix cores on 16-row chunks;
//             other shapes stage 32-row tiles in LDS with every thread owning
//             entries (i, j); single columns are plain 16-byte dot products.
//             Per-workgroup partials are reduced by a second kernel in a fixed
//             order, so results are bitwise reproducible.
//  * update:  Out = w (.) Yin + beta * sum_k X_k C_k.  16-wide FP32 blocks run as a
//             tall-skinny product on the FP32 matrix cores with the FP64 Gram of the
//             result fused (block CholQR needs W^T W right after W is formed); other
//             widths hold rows in registers with C_k (B x B) broadcast from LDS;
//             single columns are 16-byte vector updates.
//  * chol:    Cholesky with deflation of a B x B Gram and the inverse of its
//             factor, one single-wave workgroup per matrix (batched over graphs or
//             operator groups).
//  * probes:  Philox4x32-10 (Salmon et al., SC'11) Rademacher / Gaussian blocks.
//  * small helpers: fills, scaled row sums, degree vector, CSR validation.
#include "wl_internal.h"

namespace {

constexpr int GRAM_TR = 32;  // rows per LDS tile in the Gram kernel

template <int B>
__global__ __launch_bounds__(256) void k_gram_partial(int64_t n, const float* __restrict__ Xf,
                                                      const double* __restrict__ Xd, int ldx, int64_t sX,
                                                      const float* __restrict__ Yf, const double* __restrict__ Yd,
                                                      int ldy, int bx, int by, double* __restrict__ partials) {
  constexpr int E = B * B;
  constexpr int QE = E >= 256 ? E / 256 : 1;
  __shared__ double sx[GRAM_TR * B];
  __shared__ double sy[GRAM_TR * B];
  __shared__ double sred[256];
  const int tid = threadIdx.x;
  const int64_t xoff = (int64_t)blockIdx.y * sX;
  double acc[QE];
#pragma unroll
  for (int q = 0; q < QE; ++q) acc[q] = 0.0;
  // entries-per-thread layout for E < 256: P row phases
  constexpr int P = E >= 256 ? 1 : 256 / E;
  const int e_small = tid % E;
  const int p_small = tid / E;
  const int64_t ntiles = (n + GRAM_TR - 1) / GRAM_TR;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * GRAM_TR;
    for (int idx = tid; idx < GRAM_TR * B; idx += 256) {
      const int r = idx / B, c = idx % B;
      const int64_t row = row0 + r;
      double xv = 0.0, yv = 0.0;
      if (row < n) {
        if (c < bx) xv = Xf ? (double)Xf[xoff + row * ldx + c] : Xd[xoff + row * ldx + c];
        if (c < by) yv = Yf ? (double)Yf[row * ldy + c] : Yd[row * ldy + c];
      }
      sx[idx] = xv;
      sy[idx] = yv;
    }
    __syncthreads();
    if constexpr (E >= 256) {
#pragma unroll
      for (int q = 0; q < QE; ++q) {
        const int e = tid + q * 256;
        const int i = e / B, j = e % B;
        double s = acc[q];
#pragma unroll 8
        for (int r = 0; r < GRAM_TR; ++r) s += sx[r * B + i] * sy[r * B + j];
        acc[q] = s;
      }
    } else {
      if (p_small < P) {
        const int i = e_small / B, j = e_small % B;
        double s = acc[0];
        for (int r = p_small; r < GRAM_TR; r += P) s += sx[r * B + i] * sy[r * B + j];
        acc[0] = s;
      }
    }
    __syncthreads();
  }
  double* out = partials + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * E;
  if constexpr (E >= 256) {
#pragma unroll
    for (int q = 0; q < QE; ++q) out[tid + q * 256] = acc[q];
  } else {
    sred[tid] = (p_small < P) ? acc[0] : 0.0;
    __syncthreads();
    if (tid < E) {
      double s = 0.0;
      for (int p = 0; p < P; ++p) s += sred[tid + p * E];
      out[tid] = s;
    }
  }
}

// out[(k*bx + i)*by + j] = sum_q partials[k][q][i*B + j].  Fixed-order reduction:
// a block owns EB = min(E, 16) entries; thread (entry, phase p) sums q = p, p + P, ...
// (P = 256 / EB), then the P phase sums are combined by a tree in LDS.
__global__ __launch_bounds__(256) void k_gram_finalize(const double* __restrict__ partials, int nparts, int B,
                                                       int bx, int by, double* __restrict__ out,
                                                       const double* __restrict__ skip) {
  if (skip && *skip != 0.0) return;  // the caller does not need this Gram
  __shared__ double s[256];
  const int E = B * B;
  const int EB = E < 16 ? E : 16;
  const int P = 256 / EB;
  const int k = blockIdx.y;
  const int t = threadIdx.x;
  const int el = t % EB, p = t / EB;
  const int e = blockIdx.x * EB + el;
  double v = 0.0;
  if (e < E) {
    // eight independent sums so that eight loads are in flight per thread
    const double* src = partials + (int64_t)k * nparts * E + e;
    double u[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int q = p;
    for (; q + 7 * P < nparts; q += 8 * P) {
#pragma unroll
      for (int i = 0; i < 8; ++i) u[i] += src[(int64_t)(q + i * P) * E];
    }
    for (; q < nparts; q += P) u[0] += src[(int64_t)q * E];
    v = ((u[0] + u[1]) + (u[2] + u[3])) + ((u[4] + u[5]) + (u[6] + u[7]));
  }
  s[t] = v;
  __syncthreads();
  for (int h = P / 2; h > 0; h >>= 1) {
    if (p < h) s[t] += s[t + h * EB];
    __syncthreads();
  }
  if (p == 0 && e < E) {
    const int i = e / B, j = e % B;
    if (i < bx && j < by) out[((int64_t)k * bx + i) * by + j] = s[t];
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// X^T Y for FP32 blocks with B = 16 NT columns on the matrix cores, accumulated in
// FP64 (v_mfma_f64_16x16x4f64: D += A B with A 16x4, B 4x16).  For four consecutive
// rows r..r+3 lane l supplies A[i][kk] = X[r + kk][i] and B[kk][j] = Y[r + kk][j] with
// kk = l / 16 and i = j = l % 16.  D[i][j] sits in lane l, element v with
// i = 4 v + l / 16, j = l % 16 (layout measured on gfx950 with a probe whose inputs
// make every output entry identify its (i, j)).
// NB X blocks (block k at X + k sX) share one pass over Y; the ny groups of NB blocks
// are separate workgroups over the same rows of Y.  Workgroups are dispatched to the 8
// XCDs round-robin, so the 1-D grid of gx ny workgroups (gx row sets, a multiple of 8)
// gives the ny workgroups of one row set ids 8 apart: they run on one XCD at about the
// same time and Y's rows come from HBM once into its L2.  Every wave walks 16-row
// chunks.  When every operand row is exactly B = 16 NT floats (aligned), a chunk is loaded with 16-byte coalesced loads into
// registers one chunk ahead (the loads of chunk i + 1 are in flight while chunk i,
// staged in the wave's own LDS slice, feeds the matrix cores); otherwise one element
// per lane comes straight from memory.  The four waves' accumulators are summed in
// LDS in a fixed order and each workgroup writes one partial (deterministic).
template <int NT, int NB>
__global__ __launch_bounds__(256) void k_gram_mfma(int64_t n, const float* __restrict__ X, int ldx, int64_t sX,
                                                   int nblk, const float* __restrict__ Y, int ldy, int bx, int by,
                                                   double* __restrict__ partials, const double* __restrict__ skip,
                                                   int gx, int ny) {
  if (skip && *skip != 0.0) return;  // the caller does not need this Gram
  const int wg_id = blockIdx.x;
  const int grp = (wg_id >> 3) % ny;                     // group of NB X blocks
  const int rset = ((wg_id >> 3) / ny) * 8 + (wg_id & 7);  // row set, < gx
  constexpr int B = 16 * NT;
  constexpr int TILE = 16 * B;  // floats per 16-row tile of one operand
  constexpr size_t TILE_BYTES = (size_t)4 * (NB + 1) * TILE * sizeof(float);
  constexpr size_t RED_BYTES = (size_t)NB * B * B * sizeof(double);
  __shared__ __align__(16) unsigned char smem[TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES];
  float(*sm)[NB + 1][TILE] = reinterpret_cast<float(*)[NB + 1][TILE]>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kb0 = grp * NB;
  const int nb = (nblk - kb0) < NB ? (nblk - kb0) : NB;
  v4d acc[NB][NT][NT];
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int J = 0; J < NT; ++J) acc[q][I][J] = v4d{0.0, 0.0, 0.0, 0.0};
  const int rsub = lane >> 4, c = lane & 15;
  const bool packed = ldx == B && ldy == B && bx == B && by == B && (sX % 4) == 0 &&
                      ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15u) == 0;
  const int64_t nchunks = (n + 15) / 16;
  const int64_t cstride = (int64_t)gx * 4;
  if (packed) {
    // 16 rows x B floats = 4 B float4 per operand, NT per lane
    float4 ry[NT], rx[NB][NT];
    auto fetch = [&](int64_t ch) {
      const int64_t r0 = ch * 16;
#pragma unroll
      for (int s = 0; s < NT; ++s) {
        const int f = s * 64 + lane;  // float4 index inside the tile
        const int64_t row = r0 + (f * 4) / B;
        const bool rok = row < n;
        const int64_t off = r0 * B + (int64_t)f * 4;
        ry[s] = rok ? *reinterpret_cast<const float4*>(Y + off) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int q = 0; q < NB; ++q)
          rx[q][s] = (rok && q < nb) ? *reinterpret_cast<const float4*>(X + (int64_t)(kb0 + q) * sX + off)
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    int64_t ch = (int64_t)rset * 4 + wave;
    if (ch < nchunks) fetch(ch);
    for (; ch < nchunks; ch += cstride) {
#pragma unroll
      for (int s = 0; s < NT; ++s) {
        const int f = s * 64 + lane;
        *reinterpret_cast<float4*>(&sm[wave][NB][f * 4]) = ry[s];
#pragma unroll
        for (int q = 0; q < NB; ++q) *reinterpret_cast<float4*>(&sm[wave][q][f * 4]) = rx[q][s];
      }
      __builtin_amdgcn_wave_barrier();
      if (ch + cstride < nchunks) fetch(ch + cstride);  // next chunk in flight during the products
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int rl = 4 * m + rsub;
        double yb[NT];
#pragma unroll
        for (int J = 0; J < NT; ++J) yb[J] = (double)sm[wave][NB][rl * B + 16 * J + c];
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int I = 0; I < NT; ++I) {
            const double xa = (double)sm[wave][q][rl * B + 16 * I + c];
#pragma unroll
            for (int J = 0; J < NT; ++J)
              acc[q][I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, yb[J], acc[q][I][J], 0, 0, 0);
          }
      }
      __builtin_amdgcn_wave_barrier();
    }
  } else {
    for (int64_t ch = (int64_t)rset * 4 + wave; ch < nchunks; ch += cstride) {
      const int64_t r0 = ch * 16;
      // every operand element of the chunk is requested before the first product, at
      // addresses clamped into the blocks (a branch around each load would wait for it);
      // out-of-range entries are zeroed afterwards
      float ys[4][NT], xs[4][NB][NT];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int64_t row = min(r0 + 4 * m + rsub, n - 1);
#pragma unroll
        for (int J = 0; J < NT; ++J) ys[m][J] = Y[row * ldy + min(16 * J + c, by - 1)];
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int I = 0; I < NT; ++I)
            xs[m][q][I] = X[(int64_t)(kb0 + min(q, nb - 1)) * sX + row * ldx + min(16 * I + c, bx - 1)];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const bool rok = r0 + 4 * m + rsub < n;
        double yb[NT];
#pragma unroll
        for (int J = 0; J < NT; ++J) yb[J] = (rok && 16 * J + c < by) ? (double)ys[m][J] : 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int I = 0; I < NT; ++I) {
            const double xa = (rok && q < nb && 16 * I + c < bx) ? (double)xs[m][q][I] : 0.0;
#pragma unroll
            for (int J = 0; J < NT; ++J)
              acc[q][I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, yb[J], acc[q][I][J], 0, 0, 0);
          }
      }
    }
  }
  // waves 0..3 add their accumulators into LDS in turn (the tiles are no longer needed)
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
          for (int J = 0; J < NT; ++J)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int idx = q * B * B + (16 * I + 4 * v + rsub) * B + 16 * J + c;
              red[idx] = (w == 0 ? 0.0 : red[idx]) + acc[q][I][J][v];
            }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nb * B * B; e += 256) {
    const int q = e / (B * B);
    partials[((int64_t)(kb0 + q) * gx + rset) * (B * B) + (e - q * B * B)] = red[e];
  }
}

// Out = (wv ? wv[r] : alpha) Yin + beta sum_k X_k C_k for FP32 blocks whose rows are
// exactly B floats (B = 4 LPR): LPR lanes hold one row as float4 fragments (coalesced
// 16-byte accesses across the wave); the row is shared inside its lane group with
// shuffles.  The C_k are staged in LDS (converted to float) once per workgroup when
// they fit (kc blocks at a time otherwise), and the X_k fragments of up to four
// blocks are loaded together so their latencies overlap.
template <int B>
__global__ __launch_bounds__(256) void k_update_f4(int64_t n, const float* X, int64_t sX, int nblk, int kc,
                                                   const double* __restrict__ C, const float* Yin, double alpha,
                                                   const float* __restrict__ wv, double beta, float* Out,
                                                   const double* __restrict__ skip) {
  if (skip && *skip != 0.0) return;  // identity update the caller elides
  constexpr int LPR = B / 4;
  constexpr int RPT = 256 / LPR;  // rows per tile
  extern __shared__ float sC[];   // kc blocks of B x B
  const int sub = threadIdx.x % LPR;
  const int rloc = threadIdx.x / LPR;
  const float tb = (float)beta;
  const bool once = kc >= nblk;
  if (once) {
    for (int e = threadIdx.x; e < nblk * B * B; e += 256) sC[e] = (float)C[e];
    __syncthreads();
  }
  const int64_t ntiles = (n + RPT - 1) / RPT;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row = t * RPT + rloc;
    const bool ok = row < n;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < nblk; c0 += kc) {
      const int c1 = c0 + kc < nblk ? c0 + kc : nblk;
      if (!once) {
        __syncthreads();
        for (int e = threadIdx.x; e < (c1 - c0) * B * B; e += 256) sC[e] = (float)C[(int64_t)c0 * B * B + e];
        __syncthreads();
      }
      for (int k0 = c0; k0 < c1; k0 += 4) {
        float4 xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          xv[u] = (ok && k0 + u < c1) ? *reinterpret_cast<const float4*>(X + (int64_t)(k0 + u) * sX + row * B + 4 * sub)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (k0 + u >= c1) break;
          const float* Ck = sC + (int64_t)(k0 + u - c0) * B * B;
#pragma unroll
          for (int src = 0; src < LPR; ++src) {
            float v[4];
            v[0] = __shfl(xv[u].x, src, LPR);
            v[1] = __shfl(xv[u].y, src, LPR);
            v[2] = __shfl(xv[u].z, src, LPR);
            v[3] = __shfl(xv[u].w, src, LPR);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float* crow = Ck + (4 * src + q) * B + 4 * sub;
#pragma unroll
              for (int cc = 0; cc < 4; ++cc) acc[cc] += v[q] * crow[cc];
            }
          }
        }
      }
    }
    if (ok) {
      float4 o = make_float4(tb * acc[0], tb * acc[1], tb * acc[2], tb * acc[3]);
      if (Yin) {
        const float sc = wv ? wv[row] : (float)alpha;
        const float4 y = *reinterpret_cast<const float4*>(Yin + row * B + 4 * sub);
        o.x += sc * y.x;
        o.y += sc * y.y;
        o.z += sc * y.z;
        o.w += sc * y.w;
      }
      *reinterpret_cast<float4*>(Out + row * B + 4 * sub) = o;
    }
  }
}

// Out = beta sum_k X_k C_k + (wv ? wv : alpha) .* Yin for n x 16 FP32 blocks, as a
// tall-skinny product on the matrix cores (v_mfma_f32_16x16x4f32), optionally with the
// Gram Out^T Out accumulated in FP64 on the same registers (v_mfma_f64_16x16x4f64).
// A wave takes 16-row chunks.  Lane l loads 16 bytes of the chunk, row l % 16, columns
// 4 (l / 16) .. + 3; product step s uses the s-th of them as the A operand, i.e. the
// step runs over the columns {4 g + s : g = 0..3} of every X_k, and lane l supplies the
// matching B operand C_k[4 (l / 16) + s][l % 16] from a lane-ordered copy of C in LDS.
// Lane l then holds result rows 4 (l / 16) + v, column l % 16 (v = 0..3), which are
// also exactly its operands for the Gram: step v sums over rows {4 g + v}.  Rows past
// n load zeros and are not stored.  Out may alias X_k or Yin (a chunk is read whole
// before it is written).  The four waves' Grams are summed in LDS in a fixed order;
// each workgroup writes one 16 x 16 partial.
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int UPD_MFMA_MAXK = 48;

template <bool GRAM>
__global__ __launch_bounds__(256) void k_update_mfma16(int64_t n, const float* X, int64_t sX, int nblk,
                                                       const double* __restrict__ C, const float* Yin, double alpha,
                                                       const float* __restrict__ wv, double beta, float* Out,
                                                       double* __restrict__ partials,
                                                       const double* __restrict__ skip,
                                                       const double* __restrict__ skip_gram) {
  if (skip && *skip != 0.0) return;  // identity update the caller elides
  extern __shared__ float4 sCl[];  // nblk x 64 lane-ordered operands (nblk KiB)
  __shared__ double red[256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  for (int e = threadIdx.x; e < nblk * 64; e += 256) {
    const int k = e >> 6, l = e & 63, gg = l >> 4, cc = l & 15;
    const double* Ck = C + (int64_t)k * 256 + (4 * gg) * 16 + cc;
    sCl[e] = make_float4((float)Ck[0], (float)Ck[16], (float)Ck[32], (float)Ck[48]);
  }
  __syncthreads();
  const bool gram = GRAM && !(skip_gram && *skip_gram != 0.0);
  const float tb = (float)beta, ta = (float)alpha;
  v4d gacc = {0.0, 0.0, 0.0, 0.0};
  const int64_t nchunks = (n + 15) / 16;
  const int64_t cstride = (int64_t)gridDim.x * 4;
  for (int64_t ch = (int64_t)blockIdx.x * 4 + wave; ch < nchunks; ch += cstride) {
    const int64_t r0 = ch * 16;
    const bool okA = r0 + c < n;
    const float* xa = X + (r0 + c) * 16 + 4 * g;
    v4f d = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < nblk; k0 += 4) {
      float4 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        x[u] = (okA && k0 + u < nblk) ? *reinterpret_cast<const float4*>(xa + (int64_t)(k0 + u) * sX)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (k0 + u >= nblk) break;
        const float4 bq = sCl[(k0 + u) * 64 + lane];
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
        yv[v] = Yin[row * 16 + c];
        wq[v] = wv ? wv[row] : ta;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (r0 + 4 * g + v < n) o[v] += wq[v] * yv[v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * g + v;
      if (row < n) Out[row * 16 + c] = o[v];
    }
    if (gram) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double ov = (double)o[v];
        gacc = __builtin_amdgcn_mfma_f64_16x16x4f64(ov, ov, gacc, 0, 0, 0);
      }
    }
  }
  if (!gram) return;  // uniform over the workgroup
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int idx = (4 * v + g) * 16 + c;  // FP64 16x16x4 output layout
        red[idx] = (w == 0 ? 0.0 : red[idx]) + gacc[v];
      }
    }
    __syncthreads();
  }
  partials[(int64_t)blockIdx.x * 256 + threadIdx.x] = red[threadIdx.x];
}

// The same for n x 32 FP32 blocks: the 32 x 32 product as 2 x 2 tiles of 16 on
// v_mfma_f32_16x16x4f32.  Lane l loads the 16 bytes at columns 16 h + 4 (l / 16)
// (h = 0, 1) of chunk row l % 16; product step (h, s) takes component s of half h as
// the A operand (the columns {16 h + 4 g + s : g = 0..3}) against the B operand
// C_k[16 h + 4 (l / 16) + s][16 t + l % 16] of output tile t, lane-ordered in LDS
// (4 KiB per block, at most UPD32_MAXK blocks per launch: longer combinations are
// chained launches that accumulate into Out).  Lane l holds result rows
// 4 (l / 16) + v of the columns l % 16 and 16 + l % 16; the optional Gram Out^T Out
// (FP64 matrix cores) takes its three distinct 16 x 16 tiles from the same registers.
// Each workgroup writes one full 32 x 32 partial.
constexpr int UPD32_MAXK = 12;

template <bool GRAM>
__global__ __launch_bounds__(256) void k_update_mfma32(int64_t n, const float* X, int64_t sX, int nblk,
                                                       const double* __restrict__ C, const float* Yin, double alpha,
                                                       const float* __restrict__ wv, double beta, float* Out,
                                                       double* __restrict__ partials,
                                                       const double* __restrict__ skip,
                                                       const double* __restrict__ skip_gram) {
  if (skip && *skip != 0.0) return;  // identity update the caller elides
  extern __shared__ float4 sCl[];     // [block][tile t][half h][lane], nblk x 4 KiB
  __shared__ double red[3][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  for (int e = threadIdx.x; e < nblk * 256; e += 256) {
    const int k = e >> 8, th = (e >> 6) & 3, l = e & 63;
    const int t = th >> 1, h = th & 1, gg = l >> 4, cc = l & 15;
    const double* Ck = C + (int64_t)k * 1024 + (16 * h + 4 * gg) * 32 + 16 * t + cc;
    sCl[e] = make_float4((float)Ck[0], (float)Ck[32], (float)Ck[64], (float)Ck[96]);
  }
  __syncthreads();
  const bool gram = GRAM && !(skip_gram && *skip_gram != 0.0);
  const float tb = (float)beta, ta = (float)alpha;
  v4d g00 = {0.0, 0.0, 0.0, 0.0}, g01 = g00, g11 = g00;
  const int64_t nchunks = (n + 15) / 16;
  const int64_t cstride = (int64_t)gridDim.x * 4;
  for (int64_t ch = (int64_t)blockIdx.x * 4 + wave; ch < nchunks; ch += cstride) {
    const int64_t r0 = ch * 16;
    const bool okA = r0 + c < n;
    const float* xa = X + (r0 + c) * 32 + 4 * g;
    v4f d0 = {0.f, 0.f, 0.f, 0.f}, d1 = d0;
    for (int k0 = 0; k0 < nblk; k0 += 4) {
      float4 x[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          x[u][h] = (okA && k0 + u < nblk) ? *reinterpret_cast<const float4*>(xa + (int64_t)(k0 + u) * sX + 16 * h)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (k0 + u >= nblk) break;
        const float4* bk = sCl + (k0 + u) * 256 + lane;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float4 b0 = bk[h * 64], b1 = bk[128 + h * 64];
          d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u][h].x, b0.x, d0, 0, 0, 0);
          d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u][h].x, b1.x, d1, 0, 0, 0);
          d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u][h].y, b0.y, d0, 0, 0, 0);
          d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u][h].y, b1.y, d1, 0, 0, 0);
          d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u][h].z, b0.z, d0, 0, 0, 0);
          d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u][h].z, b1.z, d1, 0, 0, 0);
          d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u][h].w, b0.w, d0, 0, 0, 0);
          d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u][h].w, b1.w, d1, 0, 0, 0);
        }
      }
    }
    float o0[4], o1[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      o0[v] = tb * d0[v];
      o1[v] = tb * d1[v];
    }
    if (Yin) {  // clamped loads, zero weight past n
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = min(r0 + 4 * g + v, n - 1);
        const float y0 = Yin[row * 32 + c], y1 = Yin[row * 32 + 16 + c];
        const float wq = wv ? wv[row] : ta;
        if (r0 + 4 * g + v < n) {
          o0[v] += wq * y0;
          o1[v] += wq * y1;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * g + v;
      if (row < n) {
        Out[row * 32 + c] = o0[v];
        Out[row * 32 + 16 + c] = o1[v];
      }
    }
    if (gram) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double a = (double)o0[v], b = (double)o1[v];
        g00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, g00, 0, 0, 0);
        g01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, g01, 0, 0, 0);
        g11 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, g11, 0, 0, 0);
      }
    }
  }
  if (!gram) return;  // uniform over the workgroup
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int idx = (4 * v + g) * 16 + c;  // FP64 16x16x4 output layout
        red[0][idx] = (w == 0 ? 0.0 : red[0][idx]) + g00[v];
        red[1][idx] = (w == 0 ? 0.0 : red[1][idx]) + g01[v];
        red[2][idx] = (w == 0 ? 0.0 : red[2][idx]) + g11[v];
      }
    }
    __syncthreads();
  }
  // the 32 x 32 partial: [[G00, G01], [G01^T, G11]]
  const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
  double* P = partials + (int64_t)blockIdx.x * 1024;
  P[i * 32 + j] = red[0][threadIdx.x];
  P[i * 32 + 16 + j] = red[1][threadIdx.x];
  P[(16 + j) * 32 + i] = red[1][threadIdx.x];
  P[(16 + i) * 32 + 16 + j] = red[2][threadIdx.x];
}

template <typename T, int B>
struct RowVec {
  T v[B];
};

// Single-column blocks are plain vectors: rows are consecutive, so each lane moves 16
// contiguous bytes per load.  Dot products accumulate in FP64.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float4 type;
  static constexpr int W = 4;
};
template <>
struct Vec16<double> {
  typedef double2 type;
  static constexpr int W = 2;
};

template <typename T>
__device__ __forceinline__ double vdot(const typename Vec16<T>::type& x, const typename Vec16<T>::type& y) {
  if constexpr (Vec16<T>::W == 4)
    return (double)x.x * (double)y.x + (double)x.y * (double)y.y + (double)x.z * (double)y.z +
           (double)x.w * (double)y.w;
  else
    return (double)x.x * (double)y.x + (double)x.y * (double)y.y;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int VDOT_KB = 4;  // vectors X_k dotted with Y per workgroup

// partials[k * gridDim.x + blockIdx.x] = X_k . Y over this workgroup's rows, for
// k in [blockIdx.y * VDOT_KB, +VDOT_KB) and k < nblk.
template <typename T>
__global__ __launch_bounds__(256) void k_vdot(int64_t n, const T* __restrict__ X, int64_t sX, int nblk,
                                              const T* __restrict__ Y, double* __restrict__ partials,
                                              const double* __restrict__ skip) {
  if (skip && *skip != 0.0) return;
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  const int k0 = blockIdx.y * VDOT_KB;
  const int kn = min(VDOT_KB, nblk - k0);
  double acc[VDOT_KB] = {0.0, 0.0, 0.0, 0.0};
  const int64_t nv = n / W;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += (int64_t)gridDim.x * 256) {
    const V y = reinterpret_cast<const V*>(Y)[i];
#pragma unroll
    for (int kk = 0; kk < VDOT_KB; ++kk)
      if (kk < kn) acc[kk] += vdot<T>(reinterpret_cast<const V*>(X + (int64_t)(k0 + kk) * sX)[i], y);
  }
  if (blockIdx.x == 0) {  // rows past the last whole vector
    const int64_t r = nv * W + threadIdx.x;
    if (r < n) {
#pragma unroll
      for (int kk = 0; kk < VDOT_KB; ++kk)
        if (kk < kn) acc[kk] += (double)X[(int64_t)(k0 + kk) * sX + r] * (double)Y[r];
    }
  }
  __shared__ double red[4][VDOT_KB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int kk = 0; kk < VDOT_KB; ++kk) {
    const double v = wave_sum(acc[kk]);
    if (lane == 0) red[wave][kk] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < kn)
    partials[(int64_t)(k0 + threadIdx.x) * gridDim.x + blockIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

constexpr int VUPD_MAXK = 64;  // vectors combined by one update

// Out = (wv ? wv : alpha) .* Yin + beta * sum_k C[k] X_k on vectors (Out may alias X_k
// or Yin: every element is read and written by the same lane); with partials, the
// workgroup's part of Out . Out goes to partials[blockIdx.x].
template <typename T>
__global__ __launch_bounds__(256) void k_vupdate(int64_t n, const T* X, int64_t sX, int nblk,
                                                 const double* __restrict__ C, const T* Yin, double alpha,
                                                 const T* __restrict__ wv, double beta, T* Out,
                                                 double* __restrict__ partials, const double* __restrict__ skip) {
  if (skip && *skip != 0.0) return;
  typedef typename Vec16<T>::type V;
  constexpr int W = Vec16<T>::W;
  __shared__ T sC[VUPD_MAXK];
  if ((int)threadIdx.x < nblk) sC[threadIdx.x] = (T)C[threadIdx.x];
  __syncthreads();
  const T tb = (T)beta, ta = (T)alpha;
  double dot = 0.0;
  const int64_t nv = n / W;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += (int64_t)gridDim.x * 256) {
    T acc[W];
#pragma unroll
    for (int l = 0; l < W; ++l) acc[l] = T(0);
    for (int k = 0; k < nblk; ++k) {
      const V x = reinterpret_cast<const V*>(X + (int64_t)k * sX)[i];
      const T c = sC[k];
      const T* xs = reinterpret_cast<const T*>(&x);
#pragma unroll
      for (int l = 0; l < W; ++l) acc[l] += xs[l] * c;
    }
    T o[W];
#pragma unroll
    for (int l = 0; l < W; ++l) o[l] = tb * acc[l];
    if (Yin) {
      const V y = reinterpret_cast<const V*>(Yin)[i];
      const T* ys = reinterpret_cast<const T*>(&y);
      if (wv) {
        const V w = reinterpret_cast<const V*>(wv)[i];
        const T* ws = reinterpret_cast<const T*>(&w);
#pragma unroll
        for (int l = 0; l < W; ++l) o[l] += ws[l] * ys[l];
      } else {
#pragma unroll
        for (int l = 0; l < W; ++l) o[l] += ta * ys[l];
      }
    }
    V ov;
    __builtin_memcpy(&ov, o, sizeof(V));
    reinterpret_cast<V*>(Out)[i] = ov;
    if (partials) {
#pragma unroll
      for (int l = 0; l < W; ++l) dot += (double)o[l] * (double)o[l];
    }
  }
  if (blockIdx.x == 0) {  // rows past the last whole vector
    const int64_t r = nv * W + threadIdx.x;
    if (r < n) {
      T acc = T(0);
      for (int k = 0; k < nblk; ++k) acc += X[(int64_t)k * sX + r] * sC[k];
      T o = tb * acc;
      if (Yin) o += (wv ? wv[r] : ta) * Yin[r];
      Out[r] = o;
      if (partials) dot += (double)o * (double)o;
    }
  }
  if (partials) {
    __shared__ double red[4];
    const double v = wave_sum(dot);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Out[r,:] = (wv ? wv[r] : alpha) * Yin[r,:] + beta * sum_k X_k[r,0:bx] C_k,  C_k = C[k*bx:(k+1)*bx, 0:by]
template <typename T, int B>
__global__ __launch_bounds__(256) void k_update(int64_t n, const T* X, int ldx, int64_t sX, int nblk,
                                                int bx, const double* __restrict__ C, const T* Yin, int ldy,
                                                double alpha, const T* __restrict__ wv, double beta, T* Out,
                                                int by, double* __restrict__ gram_partials) {
  // rows of the result staged per chunk for the fused Gram (keeps LDS <= 64 KiB)
  constexpr int CHR = (256 * (B + 1) * (int)sizeof(T) <= 65536) ? 256 : 65536 / ((B + 1) * (int)sizeof(T)) / 64 * 64;
  __shared__ T sC[B * B];
  __shared__ T sO[CHR * (B + 1)];
  const int tid = threadIdx.x;
  const T tb = (T)beta;
  constexpr int E = B * B;
  constexpr int QE = E >= 256 ? E / 256 : 1;
  double gacc[QE];
#pragma unroll
  for (int q = 0; q < QE; ++q) gacc[q] = 0.0;
  constexpr int P = E >= 256 ? 1 : 256 / E;
  const int64_t ntiles = (n + 255) / 256;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row = t * 256 + tid;
    const bool ok = row < n;
    T acc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = T(0);
    for (int k = 0; k < nblk; ++k) {
      __syncthreads();
      for (int e = tid; e < B * B; e += 256) {
        const int i = e / B, j = e % B;
        sC[e] = (i < bx && j < by) ? (T)C[((int64_t)k * bx + i) * by + j] : T(0);
      }
      __syncthreads();
      if (ok) {
        const T* xr = X + (int64_t)k * sX + row * ldx;
        T xv[B];
#pragma unroll
        for (int i = 0; i < B; ++i) xv[i] = (i < bx) ? xr[i] : T(0);
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
          for (int j = 0; j < B; ++j) acc[j] += xv[i] * sC[i * B + j];
      }
    }
    if (ok) {
      const T sc = wv ? wv[row] : (T)alpha;
      T* orow = Out + row * ldy;
      const T* yrow = Yin ? Yin + row * ldy : nullptr;
#pragma unroll
      for (int j = 0; j < B; ++j) {
        if (j < by) {
          T o = tb * acc[j];
          if (yrow) o += sc * yrow[j];
          orow[j] = o;
          acc[j] = o;
        }
      }
    }
    if (gram_partials) {
      for (int c0 = 0; c0 < 256; c0 += CHR) {
        const int rows = (256 - c0) < CHR ? (256 - c0) : CHR;
        __syncthreads();
        if (tid >= c0 && tid < c0 + CHR) {
#pragma unroll
          for (int j = 0; j < B; ++j) sO[(tid - c0) * (B + 1) + j] = (ok && j < by) ? acc[j] : T(0);
        }
        __syncthreads();
        if constexpr (E >= 256) {
#pragma unroll
          for (int q = 0; q < QE; ++q) {
            const int e = tid + q * 256;
            const int i = e / B, j = e % B;
            double s = gacc[q];
            for (int r = 0; r < rows; ++r) s += (double)sO[r * (B + 1) + i] * (double)sO[r * (B + 1) + j];
            gacc[q] = s;
          }
        } else {
          const int e = tid % E, p = tid / E;
          if (p < P) {
            const int i = e / B, j = e % B;
            double s = gacc[0];
            for (int r = p; r < rows; r += P) s += (double)sO[r * (B + 1) + i] * (double)sO[r * (B + 1) + j];
            gacc[0] = s;
          }
        }
      }
    }
  }
  if (gram_partials) {
    double* out = gram_partials + (int64_t)blockIdx.x * E;
    if constexpr (E >= 256) {
#pragma unroll
      for (int q = 0; q < QE; ++q) out[tid + q * 256] = gacc[q];
    } else {
      __shared__ double sred[256];
      const int p = tid / E;
      __syncthreads();
      sred[tid] = (p < P) ? gacc[0] : 0.0;
      __syncthreads();
      if (tid < E) {
        double s = 0.0;
        for (int q = 0; q < P; ++q) s += sred[tid + q * E];
        out[tid] = s;
      }
    }
  }
}

// Right-looking Cholesky with deflation of the b x b matrix in sG (LDS, row stride 65),
// 64 threads: a pivot <= thr zeroes its row of R and marks the column deflated.  Then
// the inverse of R on the non-deflated columns (zero elsewhere) overwrites sG and, if
// Rinv is given, is copied to global memory.
__device__ void chol_deflate(int b, double* sG, double* sR, int* defl, double thr, double* __restrict__ Rinv) {
  // Right-looking Cholesky of the upper triangle of sG (stride 65) with deflation: a
  // pivot at or below thr gives a zero row of R.  Every lane derives the pivot's root
  // and reciprocals itself, and the trailing update is spread over all 64 lanes with
  // the operands of four entries loaded before any is written (the workgroup is one
  // wave, so LDS accesses stay in program order).
  __shared__ double sdi[64];  // 1 / R_kk (0 for a deflated k)
  const int t = threadIdx.x;
  const int bb = b * b;
  for (int e = t; e < bb; e += 64) sR[(e / b) * 65 + e % b] = 0.0;
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    const double p = sG[k * 65 + k];
    const bool dk = !(p > thr) || !(p > 0.0);
    const double rkk = dk ? 0.0 : sqrt(p);
    const double irkk = dk ? 0.0 : 1.0 / rkk;
    const double ip = irkk * irkk;
    if (t == 0) {
      defl[k] = dk ? 1 : 0;
      sdi[k] = irkk;
    }
    if (t >= k && t < b) sR[k * 65 + t] = (t == k) ? rkk : sG[k * 65 + t] * irkk;
    for (int e0 = 0; e0 < bb; e0 += 256) {
      double gi[4], gj[4], gij[4];
      int at[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * 64 + t;
        const int i = e / b, j = e - (e / b) * b;
        at[q] = (e < bb && i > k && j >= i) ? i * 65 + j : -1;
        if (at[q] >= 0) {
          gi[q] = sG[k * 65 + i];
          gj[q] = sG[k * 65 + j];
          gij[q] = sG[at[q]];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (at[q] >= 0) sG[at[q]] = gij[q] - gi[q] * gj[q] * ip;
    }
    __syncthreads();
  }
  // the factorisation has consumed sG: column t of the inverse is built in place there
  // by back substitution (R_ii^{-1} from sdi; deflated rows and columns stay zero)
  if (t < b) {
    for (int i = b - 1; i >= 0; --i) {
      if (defl[i] || defl[t]) {
        sG[i * 65 + t] = 0.0;
        continue;
      }
      double v0 = (i == t) ? 1.0 : 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
      int j = i + 1;
      for (; j + 3 < b; j += 4) {
        v0 -= sR[i * 65 + j] * sG[j * 65 + t];
        v1 -= sR[i * 65 + j + 1] * sG[(j + 1) * 65 + t];
        v2 -= sR[i * 65 + j + 2] * sG[(j + 2) * 65 + t];
        v3 -= sR[i * 65 + j + 3] * sG[(j + 3) * 65 + t];
      }
      for (; j < b; ++j) v0 -= sR[i * 65 + j] * sG[j * 65 + t];
      sG[i * 65 + t] = ((v0 + v1) + (v2 + v3)) * sdi[i];
    }
  }
  __syncthreads();
  if (Rinv)
    for (int e = t; e < bb; e += 64) Rinv[e] = sG[(e / b) * 65 + e % b];
}

// One projection step of block Lanczos (classical Gram-Schmidt against V_{j-1} and
// V_j).  P stacks nbv + 1 b x b blocks: [V_{j-1}^T W'; V_j^T W'; W'^T W'] (nbv = 2) or
// [V_j^T W'; W'^T W'] (nbv = 1).  Outputs: Aout = sym(V_j^T W') (the diagonal block of
// T); Cc = [-P1; -A; I] so that W = [V_{j-1} V_j W'] Cc is the projected block; ref =
// max_i (W'^T W')_ii, the block's scale before projection.  The projected block's
// Gram is then taken from W itself: forming it by Pythagoras from these inner
// products fails as soon as the basis loses orthogonality (converged Ritz vectors).
__global__ __launch_bounds__(64) void k_lanczos_proj(int b, int nbv, const double* __restrict__ P,
                                                     double* __restrict__ Aout, double* __restrict__ Cc, int64_t gs,
                                                     double* __restrict__ ref_out) {
  // one workgroup per graph of a batch: every matrix of graph g sits gs doubles further
  const int64_t go = (int64_t)blockIdx.x * gs;
  P += go;
  Aout += go;
  Cc += go;
  const int t = threadIdx.x;
  const int bb = b * b;
  const bool hasP1 = nbv == 2;
  const double* Aj = P + (size_t)(nbv - 1) * bb;
  const double* Gp = P + (size_t)nbv * bb;
  for (int e = t; e < bb; e += 64) {
    const int i = e / b, j = e % b;
    const double a = 0.5 * (Aj[i * b + j] + Aj[j * b + i]);
    Aout[e] = a;
    if (hasP1) Cc[e] = -P[e];
    Cc[(size_t)(nbv - 1) * bb + e] = -a;
    Cc[(size_t)nbv * bb + e] = i == j ? 1.0 : 0.0;
  }
  if (t == 0 && ref_out) {
    double m = 0.0;
    for (int i = 0; i < b; ++i) m = fmax(m, Gp[i * b + i]);
    ref_out[go] = m;
  }
}

// Cholesky with deflation, one workgroup of 64 threads, b <= 64.
__global__ __launch_bounds__(64) void k_chol(int b, const double* __restrict__ G, double tol,
                                             const double* __restrict__ Aref, const double* __restrict__ Bref,
                                             double* __restrict__ R, double* __restrict__ Rinv,
                                             const double* __restrict__ Rprev, double* __restrict__ Bout,
                                             int64_t gs, double* __restrict__ ref_out, const double* ref_in,
                                             double post_tol, double* skip_out, double skip_ratio,
                                             const double* skip_in, int dg, const double* dref) {
  const int64_t go = (int64_t)blockIdx.x * gs;  // batch: graph g's matrices at +g gs
  if (ref_out) ref_out += go;
  if (ref_in) ref_in += go;
  if (skip_out) skip_out += go;
  if (skip_in) skip_in += go;
  const int t = threadIdx.x;
  if (skip_in && *skip_in != 0.0) {
    // second pass not needed: identity factors, Bout = Rprev (the first pass's factor)
    G += go;
    if (R) R += go;
    Rinv += go;
    if (Rprev) Rprev += go;
    if (Bout) Bout += go;
    for (int e = t; e < b * b; e += 64) {
      const double id = (e / b == e % b) ? 1.0 : 0.0;
      if (R) R[e] = id;
      Rinv[e] = id;
      if (Bout) Bout[e] = Rprev ? Rprev[e] : id;
    }
    return;
  }
  G += go;
  if (Aref) Aref += go;
  if (Bref) Bref += go;
  if (R) R += go;
  Rinv += go;
  if (Rprev) Rprev += go;
  if (Bout) Bout += go;
  if ((int)blockIdx.x == dg) {
    // A group of independent single-column processes (different operators side by
    // side): only the diagonal of G is meaningful.  Each column is factorised alone and
    // judged against its own scale (G_ii, A_ii^2 + B_ii^2, and for the later check the
    // diagonal of dref when given); one pass is exact, so no second pass is asked for.
    for (int e = t; e < b * b; e += 64) {
      if (R) R[e] = 0.0;
      Rinv[e] = 0.0;
      if (Bout) Bout[e] = 0.0;
    }
    __syncthreads();
    const double* dr = dref ? dref + go : nullptr;
    for (int i = t; i < b; i += 64) {
      const int d = i * b + i;
      const double g = G[d];
      double sref = g;
      if (Aref || Bref)
        sref = fmax(sref, (Aref ? Aref[d] * Aref[d] : 0.0) + (Bref ? Bref[d] * Bref[d] : 0.0));
      const bool keep = g > 0.0 && g > tol * sref;
      const double r = keep ? sqrt(g) : 0.0;
      double ri = keep ? 1.0 / r : 0.0;
      double bo = r * (Rprev ? Rprev[d] : 1.0);
      if (Bout && ref_in && post_tol > 0.0) {
        const double lim = post_tol * sqrt(fmax(dr ? dr[d] : ref_in[0], 0.0));
        if (fabs(bo) <= lim) {
          bo = 0.0;
          ri = 0.0;
        }
      }
      if (R) R[d] = r;
      Rinv[d] = ri;
      if (Bout) Bout[d] = bo;
    }
    if (t == 0) {
      if (ref_out) {
        double m = 0.0;
        for (int i = 0; i < b; ++i) m = fmax(m, G[i * b + i]);
        ref_out[0] = m;
      }
      if (skip_out) *skip_out = 1.0;
    }
    return;
  }
  __shared__ double sG[64 * 65];
  __shared__ double sR[64 * 65];
  __shared__ int defl[64];
  __shared__ double sref;
  // (t defined above)
  for (int e = t; e < b * b; e += 64) {
    const int i = e / b, j = e % b;
    sG[i * 65 + j] = 0.5 * (G[i * b + j] + G[j * b + i]);
    sR[i * 65 + j] = 0.0;
  }
  __syncthreads();
  {
    // reference scale: max diagonal of G and ||Aref||_F^2 + ||Bref||_F^2 over b, the
    // sums spread over the 64 lanes of the (single-wave) workgroup
    double m = 0.0, fa = 0.0;
    for (int i = t; i < b; i += 64) m = fmax(m, sG[i * 65 + i]);
    if (Aref)
      for (int e = t; e < b * b; e += 64) fa += Aref[e] * Aref[e];
    if (Bref)
      for (int e = t; e < b * b; e += 64) fa += Bref[e] * Bref[e];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      m = fmax(m, __shfl_xor(m, off, 64));
      fa += __shfl_xor(fa, off, 64);
    }
    if (t == 0) {
      sref = fmax(m, fa / b);
      if (ref_out) ref_out[0] = sref;  // reference scale for a later check
    }
  }
  __syncthreads();
  chol_deflate(b, sG, sR, defl, tol * sref, Rinv);
  for (int e = t; e < b * b; e += 64) {
    const int i = e / b, j = e % b;
    if (R) R[e] = sR[i * 65 + j];
  }
  // diagonal of Bout, kept on chip for the checks below (0 for a dropped component)
  __shared__ double sBd[64];
  if (Bout) {
    __syncthreads();
    if (Rprev) {  // the first pass's factor, staged (sG is free once Rinv is written)
      for (int e = t; e < b * b; e += 64) sG[(e / b) * 65 + e % b] = Rprev[e];
      __syncthreads();
    }
    if (t < b) {
      for (int j = 0; j < b; ++j) {
        double s;
        if (Rprev) {
          s = 0.0;
          for (int k = t; k <= j; ++k) s += sR[t * 65 + k] * sG[k * 65 + j];  // both upper triangular
        } else {
          s = sR[t * 65 + j];
        }
        Bout[t * b + j] = s;
        if (j == t) sBd[t] = s;
      }
    }
    // Bout is the R factor of the block as stored (R of its true Gram, or R2 R1 after a
    // second pass), so Bout_kk is the true norm of its k-th orthogonal component.
    // Components at the rounding level of the reference scale are dropped: column k of
    // Rinv and row k of Bout become zero, so the next basis block loses that column
    // instead of carrying normalised noise.
    if (ref_in && post_tol > 0.0) {
      const double lim = post_tol * sqrt(fmax(ref_in[0], 0.0));
      if (t < b && fabs(sBd[t]) <= lim) {
        for (int j = 0; j < b; ++j) Bout[t * b + j] = 0.0;
        for (int i = 0; i < b; ++i) Rinv[i * b + t] = 0.0;
        sBd[t] = 0.0;
      }
    }
  }
  // Is a second CholQR pass needed?  One pass with the Gram accumulated in FP64 leaves
  // the new block orthonormal to about u_64 kappa^2; kappa^2 is the ratio of the largest
  // to the smallest kept pivot.  skip_out = 1 when min / max >= skip_ratio.
  if (skip_out) {
    __syncthreads();
    double pmax = 0.0, pmin = INFINITY;
    for (int k = t; k < b; k += 64) {
      const double r = sR[k * 65 + k];
      const bool kept = r > 0.0 && !(Bout && sBd[k] == 0.0);
      if (kept) {
        pmax = fmax(pmax, r * r);
        pmin = fmin(pmin, r * r);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      pmax = fmax(pmax, __shfl_xor(pmax, off, 64));
      pmin = fmin(pmin, __shfl_xor(pmin, off, 64));
    }
    if (t == 0) *skip_out = (pmax == 0.0 || pmin >= skip_ratio * pmax) ? 1.0 : 0.0;
  }
}

__global__ void k_dadd(int count, const double* __restrict__ x, double* __restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) y[i] += x[i];
}
__global__ void k_dcopy(int count, const double* __restrict__ x, double* __restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) y[i] = x[i];
}

__global__ void k_dtranspose(int b, const double* __restrict__ x, double* __restrict__ y) {
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) y[(e % b) * b + e / b] = x[e];
}

template <typename T>
__global__ void k_fill(int64_t count, T value, T* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = value;
}

template <typename T>
__global__ void k_axpby_rows(int64_t n, int b, const T* __restrict__ w, const T* __restrict__ X, T beta,
                             const T* __restrict__ Y, T* __restrict__ Out) {
  const int64_t total = n * b;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / b;
    const T wr = w ? w[r] : T(1);
    Out[i] = wr * X[i] + beta * Y[i];
  }
}

template <typename T>
__global__ void k_degrees(int64_t n, const int32_t* __restrict__ rowptr, T* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (T)(rowptr[i + 1] - rowptr[i]);
}

// flags[0]: rowptr not monotone / out of range; [1]: column out of range;
// [2]: self loop; [3]: unsorted or duplicate column; [4]: missing reverse edge.
__global__ void k_validate(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                           const int32_t* __restrict__ colidx, int32_t* __restrict__ flags) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = rowptr[r], e = rowptr[r + 1];
    if (s > e || s < 0 || e > nnz) {
      atomicOr(&flags[0], 1);
      continue;
    }
    for (int64_t k = s; k < e; ++k) {
      const int32_t c = colidx[k];
      if (c < 0 || c >= n) {
        atomicOr(&flags[1], 1);
        continue;
      }
      if (c == r) atomicOr(&flags[2], 1);
      if (k > s && colidx[k - 1] >= c) atomicOr(&flags[3], 1);
      // reverse edge by binary search in row c
      int64_t lo = rowptr[c], hi = rowptr[c + 1] - 1;
      if (lo < 0 || hi >= nnz) {
        atomicOr(&flags[0], 1);
        continue;
      }
      bool found = false;
      while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t v = colidx[mid];
        if (v == r) {
          found = true;
          break;
        }
        if (v < r) lo = mid + 1; else hi = mid - 1;
      }
      if (!found) atomicOr(&flags[4], 1);
    }
  }
}

// ------------------------------------------------------------ Philox4x32-10
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

template <typename T>
__global__ void k_probes(int law, uint32_t k0, uint32_t k1, uint32_t stream, int64_t total, T* __restrict__ out) {
  const int64_t nq = (total + 3) / 4;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)q, (uint32_t)((uint64_t)q >> 32), stream, 0u};
    philox4x32_10(c, k0, k1);
    double v[4];
    if (law == WL_PROBE_RADEMACHER) {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (c[i] >> 31) ? -1.0 : 1.0;
    } else {
      const double two32i = 2.3283064365386963e-10;  // 2^-32
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        const double u1 = ((double)c[2 * pr] + 0.5) * two32i;
        const double u2 = ((double)c[2 * pr + 1] + 0.5) * two32i;
        const double rad = sqrt(-2.0 * log(u1));
        const double th = 6.283185307179586 * u2;
        v[2 * pr] = rad * cos(th);
        v[2 * pr + 1] = rad * sin(th);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t e = q * 4 + i;
      if (e < total) out[e] = (T)v[i];
    }
  }
}

// ------------------------------------------------------------ estimator rows
template <typename T>
__global__ void k_rowdot(int64_t n, int M, const T* __restrict__ Om, const T* __restrict__ Y,
                         double* __restrict__ dot, double* __restrict__ sq, int accumulate) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = accumulate ? dot[r] : 0.0, q = accumulate ? sq[r] : 0.0;
    const T* o = Om + r * M;
    const T* y = Y + r * M;
    for (int j = 0; j < M; ++j) {
      s += (double)o[j] * (double)y[j];
      q += (double)o[j] * (double)o[j];
    }
    dot[r] = s;
    sq[r] = q;
  }
}

// Diagonal estimate from the accumulated row sums s_r = sum_j Omega_rj Y_rj and
// q_r = sum_j Omega_rj^2 over M probes (modes as in k_cv_finish).
template <typename T>
__global__ void k_sums_finish(int64_t n, int M, const double* __restrict__ dot, const double* __restrict__ sq,
                              const T* __restrict__ g, int mode, T* __restrict__ diag) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const double s = dot[r], q = sq[r];
    double d;
    if (mode == 1) {
      d = s / q;
    } else if (mode == 2) {
      const double gr = (double)g[r];
      d = gr + (s - gr * q) / M;
    } else {
      d = s / M;
    }
    diag[r] = (T)d;
  }
}

// mode 0: Hutchinson, 1: BKS, 2: control variate (Hutchinson law)
template <typename T>
__global__ void k_cv_finish(int64_t n, int M, const T* __restrict__ Om, const T* __restrict__ Y,
                            const T* __restrict__ g, int mode, T* __restrict__ diag) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const T* o = Om + r * M;
    const T* y = Y + r * M;
    double s = 0.0, q = 0.0;
    for (int j = 0; j < M; ++j) {
      const double ov = (double)o[j];
      s += ov * (double)y[j];
      q += ov * ov;
    }
    double d;
    if (mode == 1) {
      d = s / q;
    } else if (mode == 2) {
      const double gr = (double)g[r];
      d = gr + (s - gr * q) / M;
    } else {
      d = s / M;
    }
    diag[r] = (T)d;
  }
}

// diag[r] = (y_r^T Q1 y_r + sum_j o_rj y_rj - y_r^T Q2 o_r) / M   (Q1, Q2 M x M, M <= 256)
template <typename T>
__global__ __launch_bounds__(256) void k_nys_diag(int64_t n, int M, const T* __restrict__ Om,
                                                  const T* __restrict__ Y, const double* __restrict__ Q1,
                                                  const double* __restrict__ Q2, T* __restrict__ diag) {
  extern __shared__ double sq[];  // Q1 then Q2 (only when 2*M*M*8 bytes fit)
  const bool staged = (int64_t)2 * M * M <= 8192;
  if (staged) {
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
      sq[e] = Q1[e];
      sq[M * M + e] = Q2[e];
    }
    __syncthreads();
  }
  const double* q1 = staged ? sq : Q1;
  const double* q2 = staged ? sq + M * M : Q2;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const T* o = Om + r * M;
    const T* y = Y + r * M;
    double tot = 0.0;
    for (int i = 0; i < M; ++i) {
      const double yi = (double)y[i];
      double a = 0.0, c = 0.0;
      for (int j = 0; j < M; ++j) {
        a += q1[i * M + j] * (double)y[j];
        c += q2[i * M + j] * (double)o[j];
      }
      tot += yi * (a - c) + (double)o[i] * yi;
    }
    diag[r] = (T)(tot / M);
  }
}

int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

int fin_grid(int E) {
  const int EB = E < 16 ? E : 16;
  return (E + EB - 1) / EB;
}

template <int B>
wl_status gram_B(wl_ctx* ctx, int64_t n, const void* X, bool isf, int ldx, int64_t sX, int nblk, const void* Y,
                 int ldy, int bx, int by, double* out, const double* skip = nullptr) {
  constexpr int E = B * B;
  if constexpr (B >= 16) {
    if (isf) {
      // matrix-core path, FP64 accumulation
      constexpr int NT = B / 16;
      const int64_t nchunks = (n + 15) / 16;
      int64_t blocks = (nchunks + 15) / 16;
      if (blocks > 1024) blocks = 1024;
      if (blocks < 1) blocks = 1;
      blocks = (blocks + 7) / 8 * 8;  // row sets: a multiple of the 8 XCDs
      const int nparts = (int)blocks;  // one partial per row set and block
      WL_TRY(ctx->partials.ensure((size_t)nparts * nblk * E * sizeof(double)));
      double* pp = ctx->partials.as<double>();
      const float* Xf = (const float*)X;
      const float* Yf = (const float*)Y;
      if (NT >= 4 || nblk == 1) {
        hipLaunchKernelGGL((k_gram_mfma<NT, 1>), dim3((unsigned)(blocks * nblk)), dim3(256), 0, ctx->stream, n, Xf,
                           ldx, sX, nblk, Yf, ldy, bx, by, pp, skip, (int)blocks, nblk);
      } else if (nblk == 2 || NT == 2) {
        const int ny = (nblk + 1) / 2;
        hipLaunchKernelGGL((k_gram_mfma<NT, 2>), dim3((unsigned)(blocks * ny)), dim3(256), 0, ctx->stream, n, Xf,
                           ldx, sX, nblk, Yf, ldy, bx, by, pp, skip, (int)blocks, ny);
      } else {
        const int ny = (nblk + 2) / 3;
        hipLaunchKernelGGL((k_gram_mfma<NT, 3>), dim3((unsigned)(blocks * ny)), dim3(256), 0, ctx->stream, n, Xf,
                           ldx, sX, nblk, Yf, ldy, bx, by, pp, skip, (int)blocks, ny);
      }
      WL_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_gram_finalize, dim3(fin_grid(E), nblk), dim3(256), 0, ctx->stream,
                         ctx->partials.as<double>(), nparts, B, bx, by, out, skip);
      WL_HIP(hipGetLastError());
      return WL_OK;
    }
  }
  if constexpr (B == 1) {
    const int W = isf ? 4 : 2;
    if (bx == 1 && by == 1 && ldx == 1 && ldy == 1 && sX % W == 0 &&
        ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15u) == 0) {
      int64_t parts = (n / W + 511) / 512;  // two vectors of 16 bytes per lane
      if (parts > 1024) parts = 1024;
      if (parts < 1) parts = 1;
      WL_TRY(ctx->partials.ensure((size_t)parts * nblk * sizeof(double)));
      const dim3 grid((unsigned)parts, (unsigned)((nblk + VDOT_KB - 1) / VDOT_KB));
      if (isf)
        hipLaunchKernelGGL(k_vdot<float>, grid, dim3(256), 0, ctx->stream, n, (const float*)X, sX, nblk,
                           (const float*)Y, ctx->partials.as<double>(), skip);
      else
        hipLaunchKernelGGL(k_vdot<double>, grid, dim3(256), 0, ctx->stream, n, (const double*)X, sX, nblk,
                           (const double*)Y, ctx->partials.as<double>(), skip);
      WL_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_gram_finalize, dim3(1, nblk), dim3(256), 0, ctx->stream, ctx->partials.as<double>(),
                         (int)parts, 1, 1, 1, out, skip);
      WL_HIP(hipGetLastError());
      return WL_OK;
    }
  }
  const int64_t ntiles = (n + GRAM_TR - 1) / GRAM_TR;
  int64_t cap = (int64_t)(1 << 22) / ((int64_t)E * nblk);
  if (cap < 32) cap = 32;
  if (cap > 512) cap = 512;
  int parts = (int)(ntiles < cap ? ntiles : cap);
  if (parts < 1) parts = 1;
  WL_TRY(ctx->partials.ensure((size_t)parts * nblk * E * sizeof(double)));
  dim3 grid(parts, nblk);
  hipLaunchKernelGGL(k_gram_partial<B>, grid, dim3(256), 0, ctx->stream, n,
                     isf ? (const float*)X : nullptr, isf ? nullptr : (const double*)X, ldx, sX,
                     isf ? (const float*)Y : nullptr, isf ? nullptr : (const double*)Y, ldy, bx, by,
                     ctx->partials.as<double>());
  WL_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_gram_finalize, dim3(fin_grid(E), nblk), dim3(256), 0, ctx->stream,
                     ctx->partials.as<double>(), parts, B, bx, by, out, nullptr);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

int pick_B(int b) {
  int B = 1;
  while (B < b) B <<= 1;
  return B;
}

template <typename T, int B>
wl_status update_B(wl_ctx* ctx, int64_t n, const T* X, int ldx, int64_t sX, int nblk, int bx, const double* C,
                   const T* Yin, int ldy, double alpha, const T* wv, double beta, T* Out, int by,
                   double* gram_out, const double* skip, const double* skip_gram) {
  constexpr int E = B * B;
  if constexpr (sizeof(T) == 4 && B == 16) {
    const bool al = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Out) |
                      reinterpret_cast<uintptr_t>(Yin)) & 15u) == 0 && (sX % 4) == 0;
    if (bx == 16 && by == 16 && ldx == 16 && ldy == 16 && al && nblk <= UPD_MFMA_MAXK && !(skip && gram_out)) {
      const int64_t nchunks = (n + 15) / 16;
      int64_t grid = (nchunks + 15) / 16;  // about four chunks per wave
      if (grid > 1024) grid = 1024;
      if (grid < 1) grid = 1;
      const size_t lds = (size_t)nblk * 64 * sizeof(float4);
      if (gram_out) {
        WL_TRY(ctx->partials.ensure((size_t)grid * 256 * sizeof(double)));
        hipLaunchKernelGGL(k_update_mfma16<true>, dim3((unsigned)grid), dim3(256), lds, ctx->stream, n,
                           (const float*)X, sX, nblk, C, (const float*)Yin, alpha, (const float*)wv, beta,
                           (float*)Out, ctx->partials.as<double>(), skip, skip_gram);
        WL_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_gram_finalize, dim3(fin_grid(256), 1), dim3(256), 0, ctx->stream,
                           ctx->partials.as<double>(), (int)grid, 16, 16, 16, gram_out, skip_gram);
        WL_HIP(hipGetLastError());
      } else {
        hipLaunchKernelGGL(k_update_mfma16<false>, dim3((unsigned)grid), dim3(256), lds, ctx->stream, n,
                           (const float*)X, sX, nblk, C, (const float*)Yin, alpha, (const float*)wv, beta,
                           (float*)Out, nullptr, skip, nullptr);
        WL_HIP(hipGetLastError());
      }
      return WL_OK;
    }
  }
  if constexpr (sizeof(T) == 4 && B == 32) {
    const bool al = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Out) |
                      reinterpret_cast<uintptr_t>(Yin)) & 15u) == 0 && (sX % 4) == 0;
    // chained launches overwrite Out before the later blocks are read: Out must not
    // be one of them
    const uintptr_t xo = reinterpret_cast<uintptr_t>(X), oo = reinterpret_cast<uintptr_t>(Out);
    const bool chain_alias = nblk > UPD32_MAXK && oo >= xo &&
                             oo < xo + ((uintptr_t)(nblk - 1) * (uintptr_t)sX + (uintptr_t)n * 32) * sizeof(float);
    if (bx == 32 && by == 32 && ldx == 32 && ldy == 32 && al && !(skip && gram_out) && !chain_alias) {
      const int64_t nchunks = (n + 15) / 16;
      int64_t grid = (nchunks + 15) / 16;  // about four chunks per wave
      if (grid > 1024) grid = 1024;
      if (grid < 1) grid = 1;
      if (gram_out) WL_TRY(ctx->partials.ensure((size_t)grid * 1024 * sizeof(double)));
      for (int k0 = 0; k0 < nblk; k0 += UPD32_MAXK) {
        const int kb = std::min(UPD32_MAXK, nblk - k0);
        const bool first = k0 == 0, last = k0 + kb == nblk;
        const float* Xk = (const float*)X + (int64_t)k0 * sX;
        const float* Yk = first ? (const float*)Yin : (const float*)Out;
        const double ak = first ? alpha : 1.0;
        const float* wk = first ? (const float*)wv : nullptr;
        const size_t lds = (size_t)kb * 256 * sizeof(float4);
        if (last && gram_out) {
          hipLaunchKernelGGL(k_update_mfma32<true>, dim3((unsigned)grid), dim3(256), lds, ctx->stream, n, Xk, sX, kb,
                             C + (int64_t)k0 * 1024, Yk, ak, wk, beta, (float*)Out, ctx->partials.as<double>(), skip,
                             skip_gram);
          WL_HIP(hipGetLastError());
          hipLaunchKernelGGL(k_gram_finalize, dim3(fin_grid(1024), 1), dim3(256), 0, ctx->stream,
                             ctx->partials.as<double>(), (int)grid, 32, 32, 32, gram_out, skip_gram);
        } else {
          hipLaunchKernelGGL(k_update_mfma32<false>, dim3((unsigned)grid), dim3(256), lds, ctx->stream, n, Xk, sX, kb,
                             C + (int64_t)k0 * 1024, Yk, ak, wk, beta, (float*)Out, nullptr, skip, nullptr);
        }
        WL_HIP(hipGetLastError());
      }
      return WL_OK;
    }
  }
  if constexpr (sizeof(T) == 4 && B >= 4) {
    const bool al = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Out) |
                      reinterpret_cast<uintptr_t>(Yin)) & 15u) == 0 && (sX % 4) == 0;
    if (bx == B && by == B && ldx == B && ldy == B && al) {
      constexpr int RPT = 256 / (B / 4);
      int64_t ntiles = (n + RPT - 1) / RPT;
      const int grid = (int)(ntiles < 1 ? 1 : (ntiles > 8192 ? 8192 : ntiles));
      // C blocks staged per workgroup: all of them if they fit in 48 KB
      const int kc = std::max(1, std::min(nblk, 12288 / (B * B)));
      const size_t lds = (size_t)kc * B * B * sizeof(float);
      hipLaunchKernelGGL((k_update_f4<B>), dim3(grid), dim3(256), lds, ctx->stream, n, (const float*)X, sX, nblk,
                         kc, C, (const float*)Yin, alpha, (const float*)wv, beta, (float*)Out, skip);
      WL_HIP(hipGetLastError());
      if (gram_out) return gram_B<B>(ctx, n, Out, true, B, 0, 1, Out, B, B, B, gram_out, skip_gram);
      return WL_OK;
    }
  }
  if constexpr (B == 1) {
    constexpr int W = sizeof(T) == 4 ? 4 : 2;
    // (an update that may be skipped and also yields a Gram takes the general path)
    if (bx == 1 && by == 1 && ldx == 1 && ldy == 1 && nblk <= VUPD_MAXK && sX % W == 0 && !(skip && gram_out) &&
        ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Out) | reinterpret_cast<uintptr_t>(Yin) |
          reinterpret_cast<uintptr_t>(wv)) & 15u) == 0) {
      int64_t grid = (n / W + 1023) / 1024;
      if (grid > (gram_out ? 512 : 2048)) grid = gram_out ? 512 : 2048;
      if (grid < 1) grid = 1;
      double* parts = nullptr;
      if (gram_out) {
        WL_TRY(ctx->partials.ensure((size_t)grid * sizeof(double)));
        parts = ctx->partials.as<double>();
      }
      hipLaunchKernelGGL(k_vupdate<T>, dim3((unsigned)grid), dim3(256), 0, ctx->stream, n, X, sX, nblk, C, Yin,
                         alpha, wv, beta, Out, parts, skip);
      WL_HIP(hipGetLastError());
      if (gram_out) {
        hipLaunchKernelGGL(k_gram_finalize, dim3(1, 1), dim3(256), 0, ctx->stream, parts, (int)grid, 1, 1, 1,
                           gram_out, skip_gram);
        WL_HIP(hipGetLastError());
      }
      return WL_OK;
    }
  }
  const int64_t ntiles = (n + 255) / 256;
  const int cap = gram_out ? 512 : 4096;
  const int grid = (int)(ntiles < cap ? (ntiles < 1 ? 1 : ntiles) : cap);
  double* parts = nullptr;
  if (gram_out) {
    WL_TRY(ctx->partials.ensure((size_t)grid * E * sizeof(double)));
    parts = ctx->partials.as<double>();
  }
  hipLaunchKernelGGL((k_update<T, B>), dim3(grid), dim3(256), 0, ctx->stream, n, X, ldx, sX, nblk, bx, C, Yin, ldy,
                     alpha, wv, beta, Out, by, parts);
  WL_HIP(hipGetLastError());
  if (gram_out) {
    hipLaunchKernelGGL(k_gram_finalize, dim3(fin_grid(E), 1), dim3(256), 0, ctx->stream, parts, grid, B, by, by,
                       gram_out, nullptr);
    WL_HIP(hipGetLastError());
  }
  return WL_OK;
}

}  // namespace

template <typename T>
wl_status launch_gram(wl_ctx* ctx, int64_t n, const T* X, int bx, int64_t sX, int nblk, const T* Y, int by,
                      double* out) {
  WL_CHECK(bx >= 1 && bx <= 64 && by >= 1 && by <= 64 && nblk >= 1, WL_EINVAL, "gram: block sizes out of range");
  const bool isf = sizeof(T) == 4;
  const int B = pick_B(bx > by ? bx : by);
  switch (B) {
    case 1: return gram_B<1>(ctx, n, X, isf, bx, sX, nblk, Y, by, bx, by, out);
    case 2: return gram_B<2>(ctx, n, X, isf, bx, sX, nblk, Y, by, bx, by, out);
    case 4: return gram_B<4>(ctx, n, X, isf, bx, sX, nblk, Y, by, bx, by, out);
    case 8: return gram_B<8>(ctx, n, X, isf, bx, sX, nblk, Y, by, bx, by, out);
    case 16: return gram_B<16>(ctx, n, X, isf, bx, sX, nblk, Y, by, bx, by, out);
    case 32: return gram_B<32>(ctx, n, X, isf, bx, sX, nblk, Y, by, bx, by, out);
    default: return gram_B<64>(ctx, n, X, isf, bx, sX, nblk, Y, by, bx, by, out);
  }
}

template <typename T>
wl_status launch_update_skip(wl_ctx* ctx, int64_t n, const T* X, int bx, int64_t sX, int nblk, const double* C,
                             const T* Yin, double alpha, const T* wv, double beta, T* Out, int by, double* gram_out,
                             const double* skip, const double* skip_gram) {
  WL_CHECK(bx >= 1 && bx <= 64 && by >= 1 && by <= 64, WL_EINVAL, "update: block sizes out of range");
  const int B = pick_B(bx > by ? bx : by);
  switch (B) {
    case 1: return update_B<T, 1>(ctx, n, X, bx, sX, nblk, bx, C, Yin, by, alpha, wv, beta, Out, by, gram_out,
                                                   skip, skip_gram);
    case 2: return update_B<T, 2>(ctx, n, X, bx, sX, nblk, bx, C, Yin, by, alpha, wv, beta, Out, by, gram_out,
                                                   skip, skip_gram);
    case 4: return update_B<T, 4>(ctx, n, X, bx, sX, nblk, bx, C, Yin, by, alpha, wv, beta, Out, by, gram_out,
                                                   skip, skip_gram);
    case 8: return update_B<T, 8>(ctx, n, X, bx, sX, nblk, bx, C, Yin, by, alpha, wv, beta, Out, by, gram_out,
                                                   skip, skip_gram);
    case 16: return update_B<T, 16>(ctx, n, X, bx, sX, nblk, bx, C, Yin, by, alpha, wv, beta, Out, by, gram_out,
                                                   skip, skip_gram);
    case 32: return update_B<T, 32>(ctx, n, X, bx, sX, nblk, bx, C, Yin, by, alpha, wv, beta, Out, by, gram_out,
                                                   skip, skip_gram);
    default: return update_B<T, 64>(ctx, n, X, bx, sX, nblk, bx, C, Yin, by, alpha, wv, beta, Out, by, gram_out,
                                                   skip, skip_gram);
  }
}

template <typename T>
wl_status launch_update(wl_ctx* ctx, int64_t n, const T* X, int bx, int64_t sX, int nblk, const double* C,
                        const T* Yin, double alpha, const T* wv, double beta, T* Out, int by, double* gram_out) {
  return launch_update_skip<T>(ctx, n, X, bx, sX, nblk, C, Yin, alpha, wv, beta, Out, by, gram_out, nullptr,
                               nullptr);
}

wl_status launch_lanczos_proj(wl_ctx* ctx, int b, int nbv, const double* P, double* Aout, double* Cc,
                              double* ref_out, int ngraphs, int64_t gs) {
  WL_CHECK(b >= 1 && b <= 64 && (nbv == 1 || nbv == 2) && ngraphs >= 1, WL_EINVAL,
           "lanczos projection: bad sizes");
  hipLaunchKernelGGL(k_lanczos_proj, dim3(ngraphs), dim3(64), 0, ctx->stream, b, nbv, P, Aout, Cc, gs, ref_out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status launch_chol(wl_ctx* ctx, int b, const double* G, double tol, const double* Aref, const double* Bref,
                      double* R, double* Rinv, const double* Rprev, double* Bout, int ngraphs, int64_t gs,
                      double* ref_out, const double* ref_in, double post_tol, double* skip_out, double skip_ratio,
                      const double* skip_in, int dg, const double* dref) {
  WL_CHECK(b >= 1 && b <= 64 && ngraphs >= 1, WL_EINVAL, "chol: b out of range");
  hipLaunchKernelGGL(k_chol, dim3(ngraphs), dim3(64), 0, ctx->stream, b, G, tol, Aref, Bref, R, Rinv, Rprev, Bout,
                     gs, ref_out, ref_in, post_tol, skip_out, skip_ratio, skip_in, dg, dref);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status launch_dadd(wl_ctx* ctx, int count, const double* x, double* y) {
  hipLaunchKernelGGL(k_dadd, dim3(grid_for(count, 256, 64)), dim3(256), 0, ctx->stream, count, x, y);
  WL_HIP(hipGetLastError());
  return WL_OK;
}
wl_status launch_dcopy(wl_ctx* ctx, int count, const double* x, double* y) {
  hipLaunchKernelGGL(k_dcopy, dim3(grid_for(count, 256, 64)), dim3(256), 0, ctx->stream, count, x, y);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status launch_dtranspose(wl_ctx* ctx, int b, const double* x, double* y) {
  hipLaunchKernelGGL(k_dtranspose, dim3(1), dim3(256), 0, ctx->stream, b, x, y);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_fill(wl_ctx* ctx, int64_t count, T value, T* out) {
  if (count <= 0) return WL_OK;
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(count, 256, 8192)), dim3(256), 0, ctx->stream, count, value, out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_axpby_rows(wl_ctx* ctx, int64_t n, int b, const T* w, const T* X, double beta, const T* Y,
                            T* Out) {
  if (n * b <= 0) return WL_OK;
  hipLaunchKernelGGL((k_axpby_rows<T>), dim3(grid_for(n * b, 256, 8192)), dim3(256), 0, ctx->stream, n, b, w, X,
                     (T)beta, Y, Out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_degrees(wl_graph* g, T* out) {
  if (g->n == 0) return WL_OK;
  hipLaunchKernelGGL((k_degrees<T>), dim3(grid_for(g->n, 256, 8192)), dim3(256), 0, g->ctx->stream, g->n, g->rowptr,
                     out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

wl_status launch_validate(wl_graph* g, int32_t* d_flags) {
  if (g->n == 0) return WL_OK;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(g->n, 256, 8192)), dim3(256), 0, g->ctx->stream, g->n, g->nnz,
                     g->rowptr, g->colidx, d_flags);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_probes(wl_ctx* ctx, int law, uint64_t seed, uint32_t stream, int64_t n, int M, T* out) {
  const int64_t total = n * (int64_t)M;
  if (total <= 0) return WL_OK;
  hipLaunchKernelGGL((k_probes<T>), dim3(grid_for((total + 3) / 4, 256, 8192)), dim3(256), 0, ctx->stream, law,
                     (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), stream, total, out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_rowdot(wl_ctx* ctx, int64_t n, int M, const T* Om, const T* Y, double* dot, double* sq,
                        int accumulate) {
  hipLaunchKernelGGL((k_rowdot<T>), dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, n, M, Om, Y, dot, sq,
                     accumulate);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_sums_finish(wl_ctx* ctx, int64_t n, int M, const double* dot, const double* sq, const T* g,
                             int mode, T* diag) {
  hipLaunchKernelGGL((k_sums_finish<T>), dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, n, M, dot, sq, g,
                     mode, diag);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_cv_finish(wl_ctx* ctx, int64_t n, int M, const T* Om, const T* Y, const T* g, int mode, T* diag) {
  hipLaunchKernelGGL((k_cv_finish<T>), dim3(grid_for(n, 256, 8192)), dim3(256), 0, ctx->stream, n, M, Om, Y, g, mode,
                     diag);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

template <typename T>
wl_status launch_nys_diag(wl_ctx* ctx, int64_t n, int M, const T* Om, const T* Y, const double* Q1,
                          const double* Q2, T* diag) {
  const size_t lds = ((int64_t)2 * M * M <= 8192) ? (size_t)2 * M * M * sizeof(double) : 0;
  hipLaunchKernelGGL((k_nys_diag<T>), dim3(grid_for(n, 256, 8192)), dim3(256), lds, ctx->stream, n, M, Om, Y, Q1, Q2,
                     diag);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

size_t gram_partials_bound(int64_t n, int prec, int b, int nblk) {
  const int64_t B = pick_B(b), E = B * B;
  nblk = std::max(nblk, 1);
  int64_t doubles = 0;
  // matrix-core Gram (FP32, B >= 16): one partial per workgroup, at most 1024
  const int64_t mfma_parts = std::min<int64_t>(1024, std::max<int64_t>(1, ((n + 15) / 16 + 15) / 16));
  if (prec == WL_FP32 && B >= 16) doubles = std::max(doubles, mfma_parts * nblk * E);
  // single-column dot products: at most 1024 partials per block
  if (B == 1) doubles = std::max<int64_t>(doubles, 1024 * nblk);
  // general tiles: one partial per 32-row tile, at most clamp(2^22 / (E nblk), 32, 512)
  const int64_t ntiles = std::max<int64_t>(1, (n + GRAM_TR - 1) / GRAM_TR);
  const int64_t cap = std::min<int64_t>(512, std::max<int64_t>(32, ((int64_t)1 << 22) / (E * nblk)));
  doubles = std::max<int64_t>(doubles, std::min(ntiles, cap) * nblk * E);
  return (size_t)doubles * sizeof(double);
}

size_t update_partials_bound(int64_t n, int prec, int b) {
  const int64_t B = pick_B(b), E = B * B;
  // matrix-core update with its Gram (FP32, 16 wide): one 256-value partial per workgroup
  const int64_t mfma_grid = std::min<int64_t>(1024, std::max<int64_t>(1, ((n + 15) / 16 + 15) / 16));
  int64_t doubles = (prec == WL_FP32 && B == 16) ? mfma_grid * 256 : 0;
  doubles = std::max<int64_t>(doubles, 512);  // single-column updates
  // general tiles with the Gram: one partial per 256-row tile, at most 512
  doubles = std::max<int64_t>(doubles, std::min<int64_t>(512, std::max<int64_t>(1, (n + 255) / 256)) * E);
  // updates that take a separate Gram of their output
  doubles = std::max<int64_t>(doubles, (int64_t)gram_partials_bound(n, prec, b, 1) / (int64_t)sizeof(double));
  return (size_t)doubles * sizeof(double);
}

#define WL_INST(T)                                                                                                   \
  template wl_status launch_gram<T>(wl_ctx*, int64_t, const T*, int, int64_t, int, const T*, int, double*);        \
  template wl_status launch_update<T>(wl_ctx*, int64_t, const T*, int, int64_t, int, const double*, const T*,      \
                                      double, const T*, double, T*, int, double*);                                 \
  template wl_status launch_update_skip<T>(wl_ctx*, int64_t, const T*, int, int64_t, int, const double*, const T*, \
                                           double, const T*, double, T*, int, double*, const double*,             \
                                           const double*);                                                         \
  template wl_status launch_fill<T>(wl_ctx*, int64_t, T, T*);                                                      \
  template wl_status launch_axpby_rows<T>(wl_ctx*, int64_t, int, const T*, const T*, double, const T*, T*);       \
  template wl_status launch_degrees<T>(wl_graph*, T*);                                                              \
  template wl_status launch_probes<T>(wl_ctx*, int, uint64_t, uint32_t, int64_t, int, T*);                         \
  template wl_status launch_rowdot<T>(wl_ctx*, int64_t, int, const T*, const T*, double*, double*, int);           \
  template wl_status launch_sums_finish<T>(wl_ctx*, int64_t, int, const double*, const double*, const T*, int, T*); \
  template wl_status launch_cv_finish<T>(wl_ctx*, int64_t, int, const T*, const T*, const T*, int, T*);            \
  template wl_status launch_nys_diag<T>(wl_ctx*, int64_t, int, const T*, const T*, const double*, const double*,  \
                                        T*);
WL_INST(float)
WL_INST(double)
