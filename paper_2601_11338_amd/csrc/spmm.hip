// CSR x tall-skinny block product with fused epilogues, for gfx950 (CDNA4).
//
// Y = A X for an unweighted symmetric CSR adjacency A (no value array: the sum of
// gathered neighbour rows) and a row-major n x b block X.  This is the matrix
// product every Krylov step of the method is built on (Sec. 4.1); the epilogue
// fuses the vector work of one step of
//   * the backtrack-downweighted recurrence  q_{k+1} = A q_k + mu (mu I - D) q_{k-1}
//     with running sum S += c_{k+1} q_{k+1}          (eq. qrec, Prop. "whe-we-converge"),
//   * the deformed Laplacian A_mu(alpha) X = (1 - mu^2 a^2) X - a A X + a^2 mu D X
//     (eq. deformed, general mu),
//   * the block Lanczos three-term subtraction  W = Op(V_j) - V_{j-1} B_{j-1}^T,
//   * the walk-Laplacian finish  L X = w * X - phi X  (eq. f-laplacian).
//
// Work decomposition (64-wide wavefronts, 256-thread workgroups):
//   * a row is owned by a group of G lanes (G | 64).  Inside the group, LPN lanes
//     cover one neighbour row segment of TILE = VW * LPN contiguous values with
//     VW-wide vector loads (16 bytes per lane), and the G / LPN neighbour slots walk
//     the row's column list in parallel; the slots are summed with xor-shuffles
//     (wave-shuffle row reduction) and slot 0 applies the epilogue;
//   * rows whose degree exceeds a threshold are listed (decreasing degree) and each
//     is processed by one whole workgroup (256 / LPN slots, shuffles inside each
//     wave, LDS across the four waves), so hub rows of heavy-tailed graphs do not
//     serialise a single group.  Those workgroups come first in the grid;
//   * blocks wider than one tile are processed as column tiles (grid y).
#include "wl_internal.h"

namespace {

template <typename T, int VW>
struct VecType;
template <>
struct VecType<float, 1> { typedef float type; };
template <>
struct VecType<float, 4> { typedef float4 type; };
template <>
struct VecType<double, 1> { typedef double type; };
template <>
struct VecType<double, 2> { typedef double2 type; };

template <typename T, int VW>
struct Frag {
  T v[VW];
};

template <typename T, int VW>
__device__ __forceinline__ Frag<T, VW> ldf(const T* p) {
  typedef typename VecType<T, VW>::type V;
  static_assert(sizeof(V) == sizeof(Frag<T, VW>), "fragment size");
  V x = *reinterpret_cast<const V*>(p);
  Frag<T, VW> f;
  __builtin_memcpy(&f, &x, sizeof(f));
  return f;
}

template <typename T, int VW>
__device__ __forceinline__ void stf(T* p, const Frag<T, VW>& f) {
  typedef typename VecType<T, VW>::type V;
  V x;
  __builtin_memcpy(&x, &f, sizeof(f));
  *reinterpret_cast<V*>(p) = x;
}

// Masked fragment load: lanes whose columns lie past the block read nothing.  With
// VW > 1 the block width is a multiple of VW, so a fragment is wholly in or out.
template <typename T, int VW, bool MASK>
__device__ __forceinline__ Frag<T, VW> ldf_m(const T* p, bool ok) {
  if constexpr (MASK && VW == 1) {
    Frag<T, VW> f;
    f.v[0] = ok ? p[0] : T(0);
    return f;
  } else if constexpr (MASK) {
    Frag<T, VW> f;
    if (ok) {
      f = ldf<T, VW>(p);
    } else {
#pragma unroll
      for (int i = 0; i < VW; ++i) f.v[i] = T(0);
    }
    return f;
  } else {
    return ldf<T, VW>(p);
  }
}

// Streaming (non-temporal) accesses for row-aligned blocks that no later gather reads
// (the running sum, P_{k-2}, the Laplacian finish input): they should not displace
// the gathered block from the caches.
template <typename T, int VW>
__device__ __forceinline__ Frag<T, VW> ldf_nt(const T* p) {
  Frag<T, VW> f;
  if constexpr (VW == 1) {
    f.v[0] = __builtin_nontemporal_load(p);
  } else {
    typedef T V __attribute__((ext_vector_type(VW)));
    V x = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
#pragma unroll
    for (int i = 0; i < VW; ++i) f.v[i] = x[i];
  }
  return f;
}

template <typename T, int VW>
__device__ __forceinline__ void stf_nt(T* p, const Frag<T, VW>& f) {
  if constexpr (VW == 1) {
    __builtin_nontemporal_store(f.v[0], p);
  } else {
    typedef T V __attribute__((ext_vector_type(VW)));
    V x;
#pragma unroll
    for (int i = 0; i < VW; ++i) x[i] = f.v[i];
    __builtin_nontemporal_store(x, reinterpret_cast<V*>(p));
  }
}

template <typename T, int VW>
__device__ __forceinline__ void zero(Frag<T, VW>& f) {
#pragma unroll
  for (int i = 0; i < VW; ++i) f.v[i] = T(0);
}

template <typename T, int VW>
__device__ __forceinline__ void add_shfl_xor(Frag<T, VW>& f, int off) {
#pragma unroll
  for (int i = 0; i < VW; ++i) f.v[i] += __shfl_xor(f.v[i], off, 64);
}

// Epilogue for row r on columns [col, col + VW) (tile-local column cl).
// Block-diagonal C term y -= Z2_row(group) C_group for the VW columns of this lane.
template <typename T, int VW>
__device__ __forceinline__ void c_term(int64_t r, int ld, int b, int col, int cl, int TILE, const EpiArgs<T>& ep,
                                       const T* sC, T* y) {
  const T* z2 = ep.Z2 + r * (int64_t)ld;
  const int kw = ep.ctab ? ep.cgw : b;                    // rows of C that meet this column
  if (ep.ctab) z2 += (col / ep.cgw) * ep.cgw;             // the operator's own segment
  constexpr int ZV = 16 / (int)sizeof(T);                 // values per 16-byte load
  int k = 0;
  if ((reinterpret_cast<uintptr_t>(z2) & 15u) == 0) {
    // the segment in 16-byte loads (the lanes of one row read the same lines)
    for (; k + ZV <= kw; k += ZV) {
      const Frag<T, ZV> zf = ldf<T, ZV>(z2 + k);
#pragma unroll
      for (int u = 0; u < ZV; ++u)
#pragma unroll
        for (int i = 0; i < VW; ++i) y[i] -= zf.v[u] * sC[(k + u) * TILE + cl + i];
    }
  }
  for (; k < kw; ++k) {
    const T zk = z2[k];
#pragma unroll
    for (int i = 0; i < VW; ++i) y[i] -= zk * sC[k * TILE + cl + i];
  }
}

// Epilogue with per-column operators (ep.cmap): the VW columns of a lane may belong to
// different operators, each with its own coefficients and finish.  The caller has
// returned for lanes past the block (with VW > 1 a fragment lies wholly inside it).
// Deferred normalisation: y (this lane's VW columns of a 16-column group) <- u N with u
// the group's 16 values (its 16 / VW consecutive lanes exchange theirs) and N the
// group's block staged in LDS as sN[k * TILE + tile column].
template <typename T, int VW>
__device__ __forceinline__ void right_factor(T* y, int cl, int TILE, const T* sN) {
  constexpr int LG = 16 / VW;  // lanes holding one group's row segment
  const int lane = threadIdx.x & 63;
  const int base = lane & ~(LG - 1);
  T out[VW];
#pragma unroll
  for (int i = 0; i < VW; ++i) out[i] = T(0);
#pragma unroll
  for (int t = 0; t < LG; ++t) {  // lane base + t's VW values, rows t VW .. of N
    T ut[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) ut[k] = __shfl(y[k], base + t, 64);
#pragma unroll
    for (int k = 0; k < VW; ++k)
#pragma unroll
      for (int i = 0; i < VW; ++i) out[i] += ut[k] * sN[(t * VW + k) * TILE + cl + i];
  }
#pragma unroll
  for (int i = 0; i < VW; ++i) y[i] = out[i];
}

// Epilogue variants (template bits of the kernel): per-column operators (ep.cmap) and
// the deferred-normalisation right factor (ep.Nm).
constexpr int EPI_COLS = 1, EPI_NFAC = 2;

// Per-column coefficients of one column tile, resolved through ep.cmap once per
// workgroup into LDS (the epilogue then reads them with a few LDS loads instead of
// global loads per column and row).  fin holds the finishing operator (-1: none).
template <typename T, int TILE>
struct ColCoef {
  T a[TILE], sc[TILE], z0[TILE], z1[TILE];
  int fin[TILE];
};

template <typename T, int TILE>
__device__ __forceinline__ void stage_col_coef(const EpiArgs<T>& ep, int c0, int b, ColCoef<T, TILE>& cc) {
  for (int j = threadIdx.x; j < TILE; j += 256) {
    const int c = c0 + j;
    const int q = c < b ? ep.cmap[c] : -1;
    if (q >= 0) {  // else a padding column: all zero
      const double* k = ep.ctab + 5 * (int64_t)q;
      cc.a[j] = (T)k[0];
      cc.z0[j] = (T)k[1];
      cc.z1[j] = (T)k[2];
      cc.sc[j] = (T)k[3];
      cc.fin[j] = ep.wv != nullptr && k[4] != 0.0 ? q : -1;
    } else {
      cc.a[j] = T(0);
      cc.z0[j] = T(0);
      cc.z1[j] = T(0);
      cc.sc[j] = T(0);
      cc.fin[j] = -1;
    }
  }
}

template <typename T, int VW, int TILE, bool NF>
__device__ __forceinline__ void epilogue_cols(int64_t r, int ld, int b, int col, int cl, T deg,
                                              const Frag<T, VW>& acc, const EpiArgs<T>& ep, const T* sC,
                                              const T* sN, const ColCoef<T, TILE>& cc, T* Y) {
  const int64_t off = r * (int64_t)ld + col;
  T y[VW];
#pragma unroll
  for (int i = 0; i < VW; ++i) y[i] = cc.a[cl + i] * acc.v[i];
  if (ep.Z) {
    Frag<T, VW> z = ldf<T, VW>(ep.Z + off);
#pragma unroll
    for (int i = 0; i < VW; ++i) y[i] += (cc.z0[cl + i] + cc.z1[cl + i] * deg) * z.v[i];
  }
  if constexpr (NF && VW > 1) right_factor<T, VW>(y, cl, TILE, sN);
  if (ep.C) c_term<T, VW>(r, ld, b, col, cl, TILE, ep, sC, y);
  if (Y) {
    Frag<T, VW> o;
#pragma unroll
    for (int i = 0; i < VW; ++i) o.v[i] = y[i];
    stf<T, VW>(Y + off, o);
  }
  if (ep.Sout) {
    Frag<T, VW> s, xw;
    if (ep.Sin)
      s = ldf_nt<T, VW>(ep.Sin + off);
    else
      zero(s);
    if (ep.wv) xw = ldf_nt<T, VW>(ep.Xw + off);
    const T s0 = (T)ep.s0;
#pragma unroll
    for (int i = 0; i < VW; ++i) {
      T v = s0 * s.v[i] + cc.sc[cl + i] * y[i];
      const int q = cc.fin[cl + i];
      if (q >= 0) v = ep.wv[r * (int64_t)ep.wld + q] * xw.v[i] - v;
      s.v[i] = v;
    }
    stf_nt<T, VW>(ep.Sout + off, s);
  }
}

template <typename T, int VW, bool MASK, int E, int TILE_>
__device__ __forceinline__ void epilogue(int64_t r, int ld, int b, int col, int cl, int TILE, T deg,
                                         const Frag<T, VW>& acc, const EpiArgs<T>& ep, const T* sC, const T* sN,
                                         const ColCoef<T, TILE_>& cc, T* Y) {
  if (MASK && col >= b) return;
  if constexpr ((E & EPI_COLS) != 0) {  // separate instantiations: their registers do not weigh on the others
    epilogue_cols<T, VW, TILE_, (E & EPI_NFAC) != 0>(r, ld, b, col, cl, deg, acc, ep, sC, sN, cc, Y);
    return;
  }
  const int64_t off = r * (int64_t)ld + col;
  double ca = ep.a, cb0 = ep.b0, cb1 = ep.b1, csc = ep.sc;
  bool fin = ep.wv != nullptr;
  if (ep.gid) {
    const double* c = ep.gtab + 5 * (int64_t)ep.gid[r];
    ca = c[0];
    cb0 = c[1];
    cb1 = c[2];
    csc = c[3];
    fin = fin && c[4] != 0.0;
  }
  if (ep.ctab) {  // the VW columns of this lane lie in one operator's group
    const double* c = ep.ctab + 5 * (col / ep.cgw);
    ca = c[0];
    cb0 = c[1];
    cb1 = c[2];
    csc = c[3];
    fin = fin && c[4] != 0.0;
  }
  T y[VW];
  const T a = (T)ca;
#pragma unroll
  for (int i = 0; i < VW; ++i) y[i] = a * acc.v[i];
  if (ep.Z) {
    const T coef = (T)(cb0 + cb1 * (double)deg);
    Frag<T, VW> z = ldf_m<T, VW, MASK>(ep.Z + off, true);
#pragma unroll
    for (int i = 0; i < VW; ++i) y[i] += coef * z.v[i];
  }
  if constexpr ((E & EPI_NFAC) != 0 && VW > 1) right_factor<T, VW>(y, cl, TILE, sN);
  if (ep.C) c_term<T, VW>(r, ld, b, col, cl, TILE, ep, sC, y);
  if (Y) {
    Frag<T, VW> o;
#pragma unroll
    for (int i = 0; i < VW; ++i) o.v[i] = y[i];
    if constexpr (MASK && VW == 1) {
      Y[off] = o.v[0];
    } else {
      stf<T, VW>(Y + off, o);
    }
  }
  if (ep.Sout) {
    Frag<T, VW> s;
    if (ep.Sin)
      s = (MASK && VW == 1) ? ldf_m<T, VW, MASK>(ep.Sin + off, true) : ldf_nt<T, VW>(ep.Sin + off);
    else
      zero(s);
    const T s0 = (T)ep.s0, sc = (T)csc;
#pragma unroll
    for (int i = 0; i < VW; ++i) s.v[i] = s0 * s.v[i] + sc * y[i];
    if (fin) {
      const T wr = ep.wld ? ep.wv[r * (int64_t)ep.wld + col / ep.cgw] : ep.wv[r];
      Frag<T, VW> xw = (MASK && VW == 1) ? ldf_m<T, VW, MASK>(ep.Xw + off, true) : ldf_nt<T, VW>(ep.Xw + off);
#pragma unroll
      for (int i = 0; i < VW; ++i) s.v[i] = wr * xw.v[i] - s.v[i];
    } else if (ep.jw) {
      const T jr = ep.jw[r];
      Frag<T, VW> xj = (MASK && VW == 1) ? ldf_m<T, VW, MASK>(ep.jx + off, true) : ldf_nt<T, VW>(ep.jx + off);
#pragma unroll
      for (int i = 0; i < VW; ++i) s.v[i] = xj.v[i] + jr * s.v[i];
    }
    if constexpr (MASK && VW == 1) {
      ep.Sout[off] = s.v[0];
    } else {
      stf_nt<T, VW>(ep.Sout + off, s);
    }
  }
}

// Sum of the neighbour row segments X[colidx[k], col : col + VW] over k = k0, k0 + stride,
// ... < e.  The column indices of U neighbours are loaded first (one round trip), then
// the U gathers are issued together (one more): a short row costs two memory
// latencies instead of two per neighbour.  Lanes past the end of their row are masked
// off, so they issue no traffic.  The summation order is k order.
template <typename T, int VW, bool MASK, int U>
__device__ __forceinline__ void gather_sum(const int32_t* __restrict__ colidx, int k0, int e, int stride,
                                           const T* __restrict__ X, int ld, int col, bool colok,
                                           Frag<T, VW>& acc) {
  for (int k = k0; k < e; k += U * stride) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = k + u * stride < e ? colidx[k + u * stride] : 0;
    Frag<T, VW> x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (k + u * stride < e)
        x[u] = ldf_m<T, VW, MASK>(X + (int64_t)j[u] * ld + col, colok);
      else
        zero(x[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < VW; ++i) acc.v[i] += x[u].v[i];
  }
}

template <typename T, int VW>
constexpr int gather_unroll() {
  return VW == 1 && sizeof(T) == 4 ? 16 : 8;
}

template <typename T, int VW, int LPN, int G, bool MASK, int E>
__global__ __launch_bounds__(256) void k_spmm(const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colidx, int64_t n, int ld, int b,
                                              const T* __restrict__ X, T* Y, EpiArgs<T> ep,
                                              const int32_t* __restrict__ long_rows, int n_long,
                                              int long_thr) {
  constexpr int TILE = VW * LPN;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sC = reinterpret_cast<T*>(smem_raw);
  __shared__ Frag<T, VW> red[4][LPN];
  constexpr bool CM = (E & EPI_COLS) != 0;
  __shared__ ColCoef<T, CM ? TILE : 1> cc;

  const int c0 = blockIdx.y * TILE;
  if constexpr (CM) {
    stage_col_coef<T, TILE>(ep, c0, b, cc);
    if (!ep.C) __syncthreads();  // else the C staging below synchronises
  }
  if (ep.C) {
    const int kw = ep.ctab ? ep.cgw : b;
    for (int e = threadIdx.x; e < kw * TILE; e += 256) {
      const int k = e / TILE, j = e - (e / TILE) * TILE;
      const int c = c0 + j;
      double v = 0.0;
      if (c < b) {
        if (ep.ctab) {  // block-diagonal C: operator q = c / cgw, local column jc
          const int q = c / ep.cgw, jc = c - q * ep.cgw;
          const double* Cq = ep.C + q * ep.cgs;
          v = ep.transC ? Cq[(int64_t)jc * ep.cgw + k] : Cq[(int64_t)k * ep.cgw + jc];
        } else {
          v = ep.transC ? ep.C[(int64_t)c * b + k] : ep.C[(int64_t)k * b + c];
        }
      }
      sC[e] = (T)v;
    }
  }
  // deferred normalisation factor: group q's block of Nm, row k, tile column j
  T* sN = sC + (ep.C ? (ep.ctab ? ep.cgw : b) * TILE : 0);
  if (ep.Nm) {
    for (int e = threadIdx.x; e < 16 * TILE; e += 256) {
      const int k = e / TILE, j = e - (e / TILE) * TILE;
      const int c = c0 + j;
      double v = 0.0;
      if (c < b) {
        const int q = c / 16, jc = c - q * 16;
        v = ep.Nm[q * ep.cgs + k * 16 + jc];
      }
      sN[e] = (T)v;
    }
  }
  if (ep.C || ep.Nm) __syncthreads();
  const int lane = threadIdx.x & 63;
  const int v = lane % LPN;
  const int cl = v * VW;
  const int col = c0 + cl;
  const bool colok = !MASK || col < b;

  if ((int)blockIdx.x < n_long) {
    constexpr int NSLOT = 256 / LPN;
    const int64_t r = long_rows[blockIdx.x];
    if (ep.gid) {  // whole workgroup decides together
      const double* c = ep.gtab + 5 * (int64_t)ep.gid[r];
      if (c[0] == 0.0 && c[3] == 0.0) return;
    }
    const int slot = threadIdx.x / LPN;
    const int s = rowptr[r], e = rowptr[r + 1];
    Frag<T, VW> acc;
    zero(acc);
    gather_sum<T, VW, MASK, gather_unroll<T, VW>()>(colidx, s + slot, e, NSLOT, X, ld, col, colok, acc);
#pragma unroll
    for (int off = LPN; off < 64; off <<= 1) add_shfl_xor(acc, off);
    const int wave = threadIdx.x >> 6;
    if (lane < LPN) red[wave][lane] = acc;
    __syncthreads();
    if (threadIdx.x < LPN) {
      Frag<T, VW> tot = red[0][lane];
#pragma unroll
      for (int w = 1; w < 4; ++w)
#pragma unroll
        for (int i = 0; i < VW; ++i) tot.v[i] += red[w][lane].v[i];
      epilogue<T, VW, MASK, E>(r, ld, b, col, cl, TILE, (T)(e - s), tot, ep, sC, sN, cc, Y);
    }
    return;
  }

  constexpr int RPB = 256 / G;
  constexpr int NS = G / LPN;
  int64_t tile = (int64_t)blockIdx.x - n_long;
  if (ep.tile_map) {
    tile = ep.tile_map[tile];
    if (tile < 0) return;  // idle block of the XCD placement (whole workgroup)
  }
  const int64_t r = tile * RPB + threadIdx.x / G;
  if (r >= n) return;  // whole group leaves together: all its lanes share r
  const int s = rowptr[r], e = rowptr[r + 1];
  if (e - s > long_thr) return;
  if (ep.gid) {  // graph finished its recurrence: nothing to gather or write
    const double* c = ep.gtab + 5 * (int64_t)ep.gid[r];
    if (c[0] == 0.0 && c[3] == 0.0) return;
  }
  const int slot = (lane % G) / LPN;
  Frag<T, VW> acc;
  zero(acc);
  gather_sum<T, VW, MASK, gather_unroll<T, VW>()>(colidx, s + slot, e, NS, X, ld, col, colok, acc);
#pragma unroll
  for (int off = LPN; off < G; off <<= 1) add_shfl_xor(acc, off);
  if (slot == 0) epilogue<T, VW, MASK, E>(r, ld, b, col, cl, TILE, (T)(e - s), acc, ep, sC, sN, cc, Y);
}

template <typename T, int VW, int LPN, int G, bool MASK>
wl_status run(wl_graph* g, const T* X, T* Y, int b, const EpiArgs<T>& ep, int long_thr) {
  constexpr int TILE = VW * LPN;
  const int tiles = (b + TILE - 1) / TILE;
  // rows above the threshold, taken from the decreasing-degree list
  int n_long = 0;
  if (long_thr < g->long_min_thr) long_thr = g->long_min_thr;
  {
    const auto& dd = g->h_long_deg;
    int lo = 0, hi = (int)dd.size();
    while (lo < hi) {  // first index with degree <= long_thr
      int mid = (lo + hi) / 2;
      if (dd[mid] > long_thr) lo = mid + 1; else hi = mid;
    }
    n_long = lo;
  }
  constexpr int RPB = 256 / G;
  int64_t nshort = (g->n + RPB - 1) / RPB;
  EpiArgs<T> epx = ep;
  if (ep.xmap) {  // XCD-aware order of the short-row tiles
    int64_t blocks = 0;
    WL_TRY(const_cast<XcdTileMap*>(ep.xmap)->get(RPB, n_long, &epx.tile_map, &blocks));
    nshort = blocks;
  }
  if (ep.prepare_only) return WL_OK;
  const int64_t gx = nshort + n_long;
  WL_CHECK(gx < (1ll << 31) && tiles < 65536, WL_ERANGE, "spmm grid too large");
  const size_t lds = ((ep.C ? (size_t)(ep.ctab ? ep.cgw : b) : 0) + (ep.Nm ? 16 : 0)) * TILE * sizeof(T);  // C, N
  dim3 grid((unsigned)gx, (unsigned)tiles);
  wl_ctx* ctx = g->ctx;
  KernelStats* ks = nullptr;
  WL_TRY(kstats_begin(ctx, ep.kclass, &ks));
  const int32_t* lr = g->long_rows.as<int32_t>();
  if constexpr (VW == 4) {  // the right factor exists for 16-byte vectors of FP32 only
    if (ep.Nm && ep.cmap)
      hipLaunchKernelGGL((k_spmm<T, VW, LPN, G, MASK, EPI_COLS | EPI_NFAC>), grid, dim3(256), lds, ctx->stream,
                         g->rowptr, g->colidx, g->n, b, b, X, Y, epx, lr, n_long, long_thr);
    else if (ep.Nm)
      hipLaunchKernelGGL((k_spmm<T, VW, LPN, G, MASK, EPI_NFAC>), grid, dim3(256), lds, ctx->stream, g->rowptr,
                         g->colidx, g->n, b, b, X, Y, epx, lr, n_long, long_thr);
  }
  if (ep.Nm && VW != 4) {
    wl_set_error("spmm: the deferred-normalisation factor needs FP32 16-byte vectors");
    return WL_EINTERNAL;
  }
  if (!ep.Nm && ep.cmap)
    hipLaunchKernelGGL((k_spmm<T, VW, LPN, G, MASK, EPI_COLS>), grid, dim3(256), lds, ctx->stream, g->rowptr,
                       g->colidx, g->n, b, b, X, Y, epx, lr, n_long, long_thr);
  else if (!ep.Nm)
    hipLaunchKernelGGL((k_spmm<T, VW, LPN, G, MASK, 0>), grid, dim3(256), lds, ctx->stream, g->rowptr,
                       g->colidx, g->n, b, b, X, Y, epx, lr, n_long, long_thr);
  WL_HIP(hipGetLastError());
  if (ks) {
    // algorithmic bytes: CSR once, the gathered block once (compulsory), every row stream once
    const double s = sizeof(T), nb = (double)g->n * b;
    int streams = 1 + (Y ? 1 : 0) + (ep.Z ? 1 : 0) + (ep.C ? 1 : 0) + (ep.Sin ? 1 : 0) + (ep.Sout ? 1 : 0) +
                  (ep.Xw ? 1 : 0) + (ep.jx ? 1 : 0);
    WL_TRY(kstats_end(ctx, ks, 4.0 * g->nnz + 4.0 * (g->n + 1) + s * nb * streams + (ep.wv ? s * g->n : 0.0) +
                                   (ep.jw ? s * g->n : 0.0)));
  }
  return WL_OK;
}

template <typename T, int VW, int LPN, bool MASK>
wl_status run_g(wl_graph* g, const T* X, T* Y, int b, const EpiArgs<T>& ep, int G, int long_thr) {
  int Gc = G < LPN ? LPN : G;
  if (Gc < 4) Gc = 4;
  if constexpr (LPN <= 4) {
    if (Gc <= 4) return run<T, VW, LPN, 4, MASK>(g, X, Y, b, ep, long_thr);
  }
  if constexpr (LPN <= 8) {
    if (Gc <= 8) return run<T, VW, LPN, 8, MASK>(g, X, Y, b, ep, long_thr);
  }
  if constexpr (LPN <= 16) {
    if (Gc <= 16) return run<T, VW, LPN, 16, MASK>(g, X, Y, b, ep, long_thr);
  }
  if (Gc <= 32) return run<T, VW, LPN, 32, MASK>(g, X, Y, b, ep, long_thr);
  return run<T, VW, LPN, 64, MASK>(g, X, Y, b, ep, long_thr);
}

template <typename T>
constexpr int vec_width() {
  return 16 / (int)sizeof(T);
}

bool aligned16(const void* p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

template <typename T>
wl_status launch_spmm(wl_graph* g, const T* X, T* Y, int b, const EpiArgs<T>& ep, const SpmmShape& sh) {
  if (g->n == 0) return WL_OK;
  constexpr int VW = vec_width<T>();
  const bool vec_ok = (b % VW == 0) && (!ep.ctab || ep.cgw % VW == 0) && aligned16(X) && aligned16(Y) &&
                      aligned16(ep.Z) && aligned16(ep.Sin) && aligned16(ep.Sout) && aligned16(ep.Xw) &&
                      aligned16(ep.jx);
  if (vec_ok) {
    const int lanes = b / VW;  // lanes needed for the whole row segment
    if (lanes == 1) return run_g<T, VW, 1, false>(g, X, Y, b, ep, sh.G, sh.long_thr);
    if (lanes == 2) return run_g<T, VW, 2, false>(g, X, Y, b, ep, sh.G, sh.long_thr);
    if (lanes <= 4 && lanes % 4 == 0) return run_g<T, VW, 4, false>(g, X, Y, b, ep, sh.G, sh.long_thr);
    if (lanes % 16 == 0) return run_g<T, VW, 16, false>(g, X, Y, b, ep, sh.G, sh.long_thr);
    // 17..31 vectors (e.g. 96 FP32 values): with 32 or more lanes per row one 32-lane
    // segment covers the whole row (idle lanes masked), each neighbour's row gathered by
    // one group in one go; with fewer the row is cut into column tiles (below)
    if (lanes > 16 && lanes < 32 && sh.G >= 32) return run_g<T, VW, 32, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
    // 12 vectors (48 FP32 values): one 16-lane segment with the last four lanes idle
    // gathers each neighbour row once, where three 4-lane tiles would gather it thrice
    if (lanes == 12) return run_g<T, VW, 16, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
    if (lanes % 8 == 0) return run_g<T, VW, 8, false>(g, X, Y, b, ep, sh.G, sh.long_thr);
    if (lanes % 4 == 0) return run_g<T, VW, 4, false>(g, X, Y, b, ep, sh.G, sh.long_thr);
    // other segments below 16 vectors (e.g. 20, 28 or 60 FP32 values): one masked
    // segment of the next power of two, so each neighbour row is still gathered once
    // with 16-byte loads
    if (lanes < 4) return run_g<T, VW, 4, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
    if (lanes < 8) return run_g<T, VW, 8, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
    if (lanes < 16) return run_g<T, VW, 16, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
  }
  // scalar path with column masking for any b
  if (b == 1) return run_g<T, 1, 1, false>(g, X, Y, b, ep, sh.G, sh.long_thr);
  if (b <= 2) return run_g<T, 1, 2, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
  if (b <= 4) return run_g<T, 1, 4, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
  if (b <= 8) return run_g<T, 1, 8, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
  return run_g<T, 1, 16, true>(g, X, Y, b, ep, sh.G, sh.long_thr);
}

template wl_status launch_spmm<float>(wl_graph*, const float*, float*, int, const EpiArgs<float>&, const SpmmShape&);
template wl_status launch_spmm<double>(wl_graph*, const double*, double*, int, const EpiArgs<double>&,
                                       const SpmmShape&);

wl_status XcdTileMap::get(int rpb, int lead, const int32_t** map, int64_t* blocks) {
  auto key = std::make_pair(rpb, lead % NXCD);
  auto it = cache.find(key);
  if (it == cache.end()) {
    std::vector<std::vector<int32_t>> tiles(NXCD);
    for (size_t p = 0; p < start.size(); ++p)
      for (int64_t t = start[p] / rpb; t < (end[p] + rpb - 1) / rpb; ++t) tiles[xcd[p]].push_back((int32_t)t);
    size_t per = 0;
    for (const auto& v : tiles) per = std::max(per, v.size());
    // block s (after lead other blocks) runs on XCD (s + lead) mod 8 and is the
    // (s / 8)-th block of that XCD
    std::vector<int32_t> h((size_t)NXCD * per, -1);
    for (size_t s = 0; s < h.size(); ++s) {
      const int x = (int)((s + (size_t)lead) % NXCD);
      const size_t k = s / NXCD;
      if (k < tiles[x].size()) h[s] = tiles[x][k];
    }
    Entry& e = cache[key];
    WL_TRY(e.map.ensure(std::max<size_t>(h.size(), 1) * 4));
    if (!h.empty() && hipMemcpy(e.map.p, h.data(), h.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      cache.erase(key);
      wl_set_error("XCD tile map upload failed");
      return WL_EDEVICE;
    }
    e.blocks = (int64_t)h.size();
    it = cache.find(key);
  }
  *map = it->second.map.as<int32_t>();
  *blocks = it->second.blocks;
  return WL_OK;
}
