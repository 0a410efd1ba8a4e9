// Multigrid-preconditioned conjugate gradients on the deformed Laplacian (Sec. 4.2).
//
// phi X = c0 A_mu(alpha)^{-1} X with A_mu(alpha) = c0 I - alpha A + alpha^2 mu D,
// c0 = 1 - mu^2 alpha^2 (eq. deformed, general mu): CG on every column of X, preconditioned
// by one V-cycle of the aggregation hierarchy built on the host (amg_host.cpp).
//
// Device side, FP64 throughout (the paper's double-precision solver):
//   * level 0 is applied implicitly from the graph through the tuned CSR kernel
//     (launch_spmm): the epilogue forms A_mu(alpha) x, the residual b - A_mu x, or a whole
//     l1-Jacobi sweep x + M^-1 (b - A_mu x), M = diag(c0 + alpha^2 mu d + alpha d);
//   * coarse levels, prolongators and restrictions are explicit CSR with values
//     (k_wspmm: 16 lanes per row, TB columns per lane group, neighbour slots reduced by
//     shuffles, the same fused modes);
//   * CG's inner products are column sums with per-workgroup partials reduced in a fixed
//     order; the step lengths stay on the device, and the host reads the residual norms
//     once per iteration to stop.
#include <chrono>
#include <cmath>

#include "wl_amg.h"

namespace {

enum { WM_APPLY = 0, WM_ADD = 1, WM_RES = 2, WM_SWEEP = 3 };

// Y = mode(M X) for an explicit CSR M: APPLY M X, ADD Z + M X, RES Z - M X, SWEEP
// X + jw (Z - M X).  16 lanes per row; lane l takes column tile column l % TB and
// neighbour slot l / TB.  Y may alias Z (each element is read and written by one lane),
// never X.
template <int TB>
__global__ __launch_bounds__(256) void k_wspmm(int64_t n, const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci, const double* __restrict__ v,
                                               const double* __restrict__ X, int b, int mode, const double* Z,
                                               const double* __restrict__ jw, double* Y) {
  constexpr int S = 16 / TB;
  const int lane = threadIdx.x & 15;
  const int64_t r = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  if (r >= n) return;  // all 16 lanes of the row leave together
  const int c = blockIdx.y * TB + lane % TB;
  const int s = lane / TB;
  const bool ok = c < b;
  double acc = 0.0;
  const int e1 = rp[r + 1];
  for (int e = rp[r] + s; e < e1; e += S) {
    const int j = ci[e];
    if (ok) acc += v[e] * X[(int64_t)j * b + c];
  }
#pragma unroll
  for (int off = TB; off < 16; off <<= 1) acc += __shfl_xor(acc, off, 16);
  if (s == 0 && ok) {
    const int64_t o = r * b + c;
    double out = acc;
    if (mode == WM_ADD)
      out = Z[o] + acc;
    else if (mode == WM_RES)
      out = Z[o] - acc;
    else if (mode == WM_SWEEP)
      out = X[o] + jw[r] * (Z[o] - acc);
    Y[o] = out;
  }
}

// X = jw (.) B row-wise (the first l1-Jacobi sweep from zero)
__global__ __launch_bounds__(256) void k_rowscale(int64_t n, int b, const double* __restrict__ jw,
                                                  const double* __restrict__ B, double* __restrict__ X) {
  const int64_t total = n * b;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256)
    X[e] = jw[e / b] * B[e];
}

__global__ __launch_bounds__(256) void k_copy64(int64_t count, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) y[e] = x[e];
}

// Column sums over row-major n x b blocks.  A workgroup owns a contiguous run of rows;
// lane t handles column t % bp (bp = b rounded up to a power of two, lanes past b idle)
// of rows t / bp, t / bp + 256 / bp, ...; per-column totals of the workgroup go to
// partials[blockIdx.x * b + c] in a fixed order.
__device__ __forceinline__ void block_colsum(double mine, int b, int bp, double* partials) {
  __shared__ double red[256];
  red[threadIdx.x] = mine;
  __syncthreads();
  if ((int)threadIdx.x < b) {
    double s = 0.0;
    for (int k = threadIdx.x; k < 256; k += bp) s += red[k];
    partials[(int64_t)blockIdx.x * b + threadIdx.x] = s;
  }
}

struct RowRange {
  int64_t lo, hi;
};
__device__ __forceinline__ RowRange rows_of_block(int64_t n) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  return {lo, lo + per < n ? lo + per : n};
}

// partials of sum_i X_ic Y_ic
__global__ __launch_bounds__(256) void k_coldot(int64_t n, int b, int bp, const double* __restrict__ X,
                                                const double* __restrict__ Y, double* __restrict__ partials) {
  const RowRange rr = rows_of_block(n);
  const int c = threadIdx.x % bp;
  double s = 0.0;
  if (c < b)
    for (int64_t r = rr.lo + threadIdx.x / bp; r < rr.hi; r += 256 / bp) s += X[r * b + c] * Y[r * b + c];
  block_colsum(s, b, bp, partials);
}

// x += a p, r -= a q with a_c = rz_c / pq_c (0 where pq_c = 0); partials of sum r_c^2
__global__ __launch_bounds__(256) void k_cg_xr(int64_t n, int b, int bp, const double* __restrict__ rz,
                                               const double* __restrict__ pq, double* __restrict__ x,
                                               double* __restrict__ r, const double* __restrict__ p,
                                               const double* __restrict__ q, double* __restrict__ partials) {
  const RowRange rr = rows_of_block(n);
  const int c = threadIdx.x % bp;
  double s = 0.0;
  if (c < b) {
    const double a = pq[c] > 0.0 ? rz[c] / pq[c] : 0.0;
    for (int64_t i = rr.lo + threadIdx.x / bp; i < rr.hi; i += 256 / bp) {
      const int64_t o = i * b + c;
      x[o] += a * p[o];
      const double rn = r[o] - a * q[o];
      r[o] = rn;
      s += rn * rn;
    }
  }
  block_colsum(s, b, bp, partials);
}

// p = z + beta p with beta_c = rz_new_c / rz_old_c (0 where rz_old_c = 0)
__global__ __launch_bounds__(256) void k_cg_p(int64_t n, int b, const double* __restrict__ rz_new,
                                              const double* __restrict__ rz_old, const double* __restrict__ z,
                                              double* __restrict__ p) {
  const int64_t total = n * b;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int c = (int)(e % b);
    const double beta = rz_old[c] > 0.0 ? rz_new[c] / rz_old[c] : 0.0;
    p[e] = z[e] + beta * p[e];
  }
}

// out[c] = sum over workgroups of partials (fixed order)
__global__ void k_colsum_finish(int nparts, int b, const double* __restrict__ partials, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b) return;
  double s = 0.0;
  for (int k = 0; k < nparts; ++k) s += partials[(int64_t)k * b + c];
  out[c] = s;
}

// Y = c0 x (phi X), or Y = w (.) Xw - c0 x (L X)
__global__ __launch_bounds__(256) void k_amg_finish(int64_t n, int b, double c0, const double* __restrict__ x,
                                                    const double* __restrict__ w, const double* __restrict__ Xw,
                                                    double* __restrict__ Y) {
  const int64_t total = n * b;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256)
    Y[e] = w ? w[e / b] * Xw[e] - c0 * x[e] : c0 * x[e];
}

unsigned grid_elems(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

int pow2_at_least(int b) {
  int p = 1;
  while (p < b) p <<= 1;
  return p;
}

constexpr int kDotParts = 1024;

unsigned dot_grid(int64_t n) {
  int64_t g = (n + 1023) / 1024;
  if (g > kDotParts) g = kDotParts;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
T* devp(DevBuf& b) {
  return b.as<T>();
}

wl_status upload(DevBuf& d, const void* h, size_t bytes) {
  WL_TRY(d.ensure(std::max<size_t>(bytes, 8)));
  if (bytes) WL_HIP(hipMemcpy(d.p, h, bytes, hipMemcpyHostToDevice));
  return WL_OK;
}

wl_status upload_csr(const HostCSR& A, DevBuf& rp, DevBuf& ci, DevBuf& v) {
  WL_CHECK(A.rp.back() < (1ll << 31), WL_ERANGE, "multigrid: a level has more than 2^31 entries");
  std::vector<int32_t> r32(A.rp.begin(), A.rp.end());
  WL_TRY(upload(rp, r32.data(), r32.size() * 4));
  WL_TRY(upload(ci, A.ci.data(), A.ci.size() * 4));
  WL_TRY(upload(v, A.v.data(), A.v.size() * 8));
  return WL_OK;
}

wl_status launch_wspmm(wl_ctx* ctx, int64_t n, const DevBuf& rp, const DevBuf& ci, const DevBuf& v,
                       const double* X, int b, int mode, const double* Z, const double* jw, double* Y) {
  if (n == 0) return WL_OK;
  const int TB = std::min(16, pow2_at_least(b));
  dim3 grid((unsigned)((n + 15) / 16), (unsigned)((b + TB - 1) / TB));
  switch (TB) {
    case 1:
      hipLaunchKernelGGL(k_wspmm<1>, grid, dim3(256), 0, ctx->stream, n, rp.as<int32_t>(), ci.as<int32_t>(),
                         v.as<double>(), X, b, mode, Z, jw, Y);
      break;
    case 2:
      hipLaunchKernelGGL(k_wspmm<2>, grid, dim3(256), 0, ctx->stream, n, rp.as<int32_t>(), ci.as<int32_t>(),
                         v.as<double>(), X, b, mode, Z, jw, Y);
      break;
    case 4:
      hipLaunchKernelGGL(k_wspmm<4>, grid, dim3(256), 0, ctx->stream, n, rp.as<int32_t>(), ci.as<int32_t>(),
                         v.as<double>(), X, b, mode, Z, jw, Y);
      break;
    case 8:
      hipLaunchKernelGGL(k_wspmm<8>, grid, dim3(256), 0, ctx->stream, n, rp.as<int32_t>(), ci.as<int32_t>(),
                         v.as<double>(), X, b, mode, Z, jw, Y);
      break;
    default:
      hipLaunchKernelGGL(k_wspmm<16>, grid, dim3(256), 0, ctx->stream, n, rp.as<int32_t>(), ci.as<int32_t>(),
                         v.as<double>(), X, b, mode, Z, jw, Y);
      break;
  }
  WL_HIP(hipGetLastError());
  return WL_OK;
}

// column sums of X (.) Y into out (b device doubles)
wl_status coldot(wl_ctx* ctx, AmgState& st, int64_t n, int b, const double* X, const double* Y, double* out) {
  const unsigned g = dot_grid(n);
  hipLaunchKernelGGL(k_coldot, dim3(g), dim3(256), 0, ctx->stream, n, b, pow2_at_least(b), X, Y,
                     st.partials.as<double>());
  WL_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_colsum_finish, dim3((b + 63) / 64), dim3(64), 0, ctx->stream, (int)g, b,
                     st.partials.as<double>(), out);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

// Level-0 products through the graph's CSR kernel (A_mu applied implicitly).
//   mode WM_APPLY: Y = A_mu X;  WM_RES: Y = Bv - A_mu X;  WM_SWEEP: Y = X + jw (Bv - A_mu X)
wl_status level0(wl_op* op, AmgState& st, const double* X, int b, int mode, const double* Bv, double* Y) {
  wl_graph* g = op->g;
  EpiArgs<double> ep;
  ep.Z = X;
  ep.kclass = WL_KC_AMG;
  if (mode == WM_APPLY) {
    ep.a = -st.alpha;
    ep.b0 = st.c0;
    ep.b1 = st.am;
    WL_TRY(launch_spmm<double>(g, X, Y, b, ep, shape_for(g, WL_FP64, b)));
  } else {
    // b - A_mu x = b + alpha A x - (c0 + am d) x, into the running-sum output
    ep.a = st.alpha;
    ep.b0 = -st.c0;
    ep.b1 = -st.am;
    ep.Sin = Bv;
    ep.Sout = Y;
    ep.s0 = 1.0;
    ep.sc = 1.0;
    if (mode == WM_SWEEP) {
      ep.jw = st.lv[0]->jw.as<double>();
      ep.jx = X;
    }
    WL_TRY(launch_spmm<double>(g, X, nullptr, b, ep, shape_for(g, WL_FP64, b)));
  }
  st.products += (double)g->nnz * b;
  return WL_OK;
}

// One V-cycle from zero at level l: out = B_l bv (out must not be level l's x or r).
wl_status vcycle(wl_op* op, AmgState& st, int l, const double* bv, double* out, int b) {
  wl_ctx* ctx = op->g->ctx;
  AmgDevLevel& L = *st.lv[l];
  const int64_t n = L.n;
  double* x = L.x.as<double>();
  double* r = L.r.as<double>();
  const bool last = l + 1 == (int)st.lv.size();
  auto sweep = [&](const double* xin, double* xout) -> wl_status {
    if (l == 0) return level0(op, st, xin, b, WM_SWEEP, bv, xout);
    st.products += (double)L.nnz * b;
    return launch_wspmm(ctx, n, L.rp, L.ci, L.v, xin, b, WM_SWEEP, bv, L.jw.as<double>(), xout);
  };
  // first sweep from zero: x = M^-1 b
  hipLaunchKernelGGL(k_rowscale, dim3(grid_elems(n * b)), dim3(256), 0, ctx->stream, n, b, L.jw.as<double>(), bv,
                     last && st.prm.coarse_sweeps == 1 ? out : x);
  WL_HIP(hipGetLastError());
  if (last) {
    // coarsest solve: the remaining sweeps, alternating x and r, the last into out
    const double* cur = x;
    for (int s = 1; s < st.prm.coarse_sweeps; ++s) {
      double* nxt = s + 1 == st.prm.coarse_sweeps ? out : (cur == x ? r : x);
      WL_TRY(sweep(cur, nxt));
      cur = nxt;
    }
    return WL_OK;
  }
  // residual, restriction, coarse correction, prolongation, post-smoothing
  if (l == 0) {
    WL_TRY(level0(op, st, x, b, WM_RES, bv, r));
  } else {
    st.products += (double)L.nnz * b;
    WL_TRY(launch_wspmm(ctx, n, L.rp, L.ci, L.v, x, b, WM_RES, bv, nullptr, r));
  }
  AmgDevLevel& C = *st.lv[l + 1];
  st.products += (double)L.pnnz * b * 2;
  WL_TRY(launch_wspmm(ctx, C.n, L.rrp, L.rci, L.rv, r, b, WM_APPLY, nullptr, nullptr, C.b.as<double>()));
  WL_TRY(vcycle(op, st, l + 1, C.b.as<double>(), C.y.as<double>(), b));
  WL_TRY(launch_wspmm(ctx, n, L.prp, L.pci, L.pv, C.y.as<double>(), b, WM_ADD, x, nullptr, x));
  return sweep(x, out);
}

wl_status ensure_blocks(wl_op* op, AmgState& st, int b) {
  if (st.nb >= b) return WL_OK;
  const int64_t n = op->g->n;
  const size_t blk = (size_t)std::max<int64_t>(n, 1) * b * 8;
  WL_TRY(st.x.ensure(blk));
  WL_TRY(st.r.ensure(blk));
  WL_TRY(st.z.ensure(blk));
  WL_TRY(st.p.ensure(blk));
  WL_TRY(st.q.ensure(blk));
  WL_TRY(st.scal.ensure((size_t)6 * b * 8));
  WL_TRY(st.partials.ensure((size_t)kDotParts * b * 8));
  for (auto& Lp : st.lv) {
    AmgDevLevel& L = *Lp;
    const size_t lb = (size_t)std::max<int64_t>(L.n, 1) * b * 8;
    WL_TRY(L.x.ensure(lb));
    WL_TRY(L.r.ensure(lb));
    WL_TRY(L.b.ensure(lb));
    WL_TRY(L.y.ensure(lb));
    L.nb = b;
  }
  st.nb = b;
  return WL_OK;
}

}  // namespace

wl_status amg_setup(wl_op* op) {
  wl_graph* g = op->g;
  const auto t0 = std::chrono::steady_clock::now();
  auto* st = new AmgState;
  op->amg = st;
  const double mu = op->d.mu, a = op->d.param;
  st->c0 = 1.0 - mu * mu * a * a;
  st->alpha = a;
  st->am = a * a * mu;
  const int64_t n = g->n;
  std::vector<int32_t> rp(n + 1), ci((size_t)g->nnz);
  WL_HIP(hipStreamSynchronize(g->ctx->stream));
  WL_HIP(hipMemcpy(rp.data(), g->rowptr, (n + 1) * 4, hipMemcpyDeviceToHost));
  if (g->nnz) WL_HIP(hipMemcpy(ci.data(), g->colidx, g->nnz * 4, hipMemcpyDeviceToHost));
  HostCSR A0;
  amg_deformed_matrix(n, rp.data(), ci.data(), mu, a, A0);
  std::vector<AmgHostLevel> hl;
  amg_build(A0, st->prm, hl, nullptr);
  for (size_t l = 0; l < hl.size(); ++l) st->lv.emplace_back(new AmgDevLevel);
  for (size_t l = 0; l < hl.size(); ++l) {
    AmgDevLevel& D = *st->lv[l];
    const AmgHostLevel& H = hl[l];
    D.n = H.A.n;
    D.nnz = (int64_t)H.A.ci.size();
    std::vector<double> jw(H.m.size());
    for (size_t i = 0; i < jw.size(); ++i) jw[i] = 1.0 / H.m[i];
    WL_TRY(upload(D.jw, jw.data(), jw.size() * 8));
    if (l > 0) WL_TRY(upload_csr(H.A, D.rp, D.ci, D.v));
    if (l + 1 < hl.size()) {
      D.pnnz = (int64_t)H.P.ci.size();
      WL_TRY(upload_csr(H.P, D.prp, D.pci, D.pv));
      WL_TRY(upload_csr(H.R, D.rrp, D.rci, D.rv));
    }
  }
  st->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return WL_OK;
}

void amg_destroy(wl_op* op) {
  delete op->amg;
  op->amg = nullptr;
}

template <>
wl_status phi_amg<float>(wl_op*, const float*, float*, int, const float*, const float*) {
  wl_set_error("the multigrid-preconditioned CG runs in double precision");
  return WL_EUNSUPPORTED;
}

template <>
wl_status phi_amg<double>(wl_op* op, const double* X, double* Y, int b, const double* wv, const double* Xw) {
  WL_CHECK(op->amg, WL_EINTERNAL, "multigrid hierarchy missing");
  AmgState& st = *op->amg;
  wl_graph* g = op->g;
  wl_ctx* ctx = g->ctx;
  const int64_t n = g->n;
  if (n == 0) return WL_OK;
  WL_TRY(ensure_blocks(op, st, b));
  double* x = st.x.as<double>();
  double* r = st.r.as<double>();
  double* z = st.z.as<double>();
  double* p = st.p.as<double>();
  double* q = st.q.as<double>();
  double* S = st.scal.as<double>();
  double* pq = S;
  double* rzA = S + b;
  double* rzB = S + 2 * b;
  double* rr = S + 3 * b;
  double* rr0 = S + 4 * b;
  const int bp = pow2_at_least(b);
  const double tol = op->d.tol > 0 ? op->d.tol : 1e-9;
  const int maxit = op->K > 0 ? op->K : 1000;
  // x = 0, r = X, rr0 = |X_c|^2
  WL_TRY(launch_fill<double>(ctx, n * b, 0.0, x));
  hipLaunchKernelGGL(k_copy64, dim3(grid_elems(n * b)), dim3(256), 0, ctx->stream, n * b, X, r);
  WL_HIP(hipGetLastError());
  WL_TRY(coldot(ctx, st, n, b, X, X, rr0));
  WL_TRY(vcycle(op, st, 0, r, z, b));
  WL_TRY(coldot(ctx, st, n, b, r, z, rzA));
  hipLaunchKernelGGL(k_copy64, dim3(grid_elems(n * b)), dim3(256), 0, ctx->stream, n * b, z, p);
  WL_HIP(hipGetLastError());
  std::vector<double> h(2 * b);
  WL_HIP(hipMemcpyAsync(h.data() + b, rr0, b * 8, hipMemcpyDeviceToHost, ctx->stream));
  WL_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<double> ref(h.begin() + b, h.end());
  double* rz = rzA;
  double* rz_next = rzB;
  int it = 0;
  double worst = 0.0;
  bool done = true;
  for (int c = 0; c < b; ++c) done = done && ref[c] == 0.0;
  while (!done) {
    if (it == maxit) {
      wl_set_error("multigrid CG: no convergence in %d iterations (relative residual %.3g > %.3g)", maxit, worst, tol);
      return WL_ENOCONV;
    }
    ++it;
    WL_TRY(level0(op, st, p, b, WM_APPLY, nullptr, q));
    WL_TRY(coldot(ctx, st, n, b, p, q, pq));
    const unsigned gd = dot_grid(n);
    hipLaunchKernelGGL(k_cg_xr, dim3(gd), dim3(256), 0, ctx->stream, n, b, bp, rz, pq, x, r, p, q,
                       st.partials.as<double>());
    WL_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_colsum_finish, dim3((b + 63) / 64), dim3(64), 0, ctx->stream, (int)gd, b,
                       st.partials.as<double>(), rr);
    WL_HIP(hipGetLastError());
    WL_HIP(hipMemcpyAsync(h.data(), rr, b * 8, hipMemcpyDeviceToHost, ctx->stream));
    WL_HIP(hipStreamSynchronize(ctx->stream));
    done = true;
    worst = 0.0;
    for (int c = 0; c < b; ++c) {
      WL_CHECK(std::isfinite(h[c]), WL_ENUMERIC, "multigrid CG: non-finite residual");
      const double rel = ref[c] > 0.0 ? std::sqrt(h[c] / ref[c]) : 0.0;
      worst = std::max(worst, rel);
      done = done && rel <= tol;
    }
    if (done) break;
    WL_TRY(vcycle(op, st, 0, r, z, b));
    WL_TRY(coldot(ctx, st, n, b, r, z, rz_next));
    hipLaunchKernelGGL(k_cg_p, dim3(grid_elems(n * b)), dim3(256), 0, ctx->stream, n, b, rz_next, rz, z, p);
    WL_HIP(hipGetLastError());
    std::swap(rz, rz_next);
  }
  st.last_iters = it;
  st.last_relres = worst;
  hipLaunchKernelGGL(k_amg_finish, dim3(grid_elems(n * b)), dim3(256), 0, ctx->stream, n, b, st.c0, x, wv, Xw, Y);
  WL_HIP(hipGetLastError());
  return WL_OK;
}

extern "C" {

wl_status wl_amg_info(const wl_op* op, wl_amg_stats* out) {
  WL_CHECK(op && out, WL_EINVAL, "wl_amg_info: null argument");
  WL_CHECK(op->amg, WL_EINVAL, "wl_amg_info: the operator does not use WL_M_AMG_CG");
  const AmgState& st = *op->amg;
  *out = wl_amg_stats{};
  out->levels = (int32_t)st.lv.size();
  double fine = 0.0, total = 0.0;
  for (size_t l = 0; l < st.lv.size() && l < WL_AMG_MAX_LEVELS; ++l) {
    out->rows[l] = st.lv[l]->n;
    out->nnz[l] = l == 0 ? op->g->nnz + op->g->n : st.lv[l]->nnz;
    total += (double)out->nnz[l];
    if (l == 0) fine = (double)out->nnz[l];
  }
  out->operator_complexity = fine > 0 ? total / fine : 1.0;
  out->setup_ms = st.setup_ms;
  out->iterations = st.last_iters;
  out->rel_residual = st.last_relres;
  out->products = st.products;
  return WL_OK;
}

wl_status wl_amg_describe(int64_t n, const int32_t* rowptr, const int32_t* colidx, double mu, double alpha,
                          int32_t max_levels, int32_t* levels, int64_t* rows, int64_t* nnz, int32_t* agg0) {
  WL_CHECK(n >= 1 && rowptr && (rowptr[n] == 0 || colidx) && levels, WL_EINVAL, "wl_amg_describe: bad arguments");
  WL_CHECK(max_levels >= 1 && max_levels <= WL_AMG_MAX_LEVELS, WL_EINVAL, "wl_amg_describe: bad max_levels");
  HostCSR A0;
  amg_deformed_matrix(n, rowptr, colidx, mu, alpha, A0);
  AmgParams prm;
  prm.max_levels = max_levels;
  std::vector<AmgHostLevel> hl;
  std::vector<int64_t> agg;
  amg_build(A0, prm, hl, &agg);
  *levels = (int32_t)hl.size();
  for (size_t l = 0; l < hl.size(); ++l) {
    if (rows) rows[l] = hl[l].A.n;
    if (nnz) nnz[l] = (int64_t)hl[l].A.ci.size();
  }
  if (agg0) {
    for (int64_t i = 0; i < n; ++i) agg0[i] = agg.empty() ? -1 : (int32_t)agg[i];
  }
  return WL_OK;
}

}  // extern "C"
