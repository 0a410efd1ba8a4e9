// Small dense FP64 linear algebra on the host for the projected Krylov matrices
// (the cheap "f(H_k) since k << n" step of Sec. 4.1): symmetric eigendecomposition
// by Householder tridiagonalisation followed by the implicit QL iteration with
// Wilkinson-type shifts, tridiagonal eigenvalues, and a block Cholesky solve for
// block tridiagonal SPD matrices.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "wl_internal.h"

namespace {

// Host threads for the dense work: the hardware's, at most 16 and at most
// OMP_NUM_THREADS when that is set, and at most cap.
int host_threads(int cap) {
  int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(e);
    if (v > 0) hw = std::min(hw, v);
  }
  return std::max(1, std::min({cap, 16, hw}));
}

// Barrier of a fixed team of threads (generation counter; spins, then yields).
class SpinBarrier {
 public:
  void reset(int n) { n_ = n; }
  void wait() {
    if (n_ == 1) return;
    const int g = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
      count_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_release);
      return;
    }
    int spins = 0;
    while (gen_.load(std::memory_order_acquire) == g)
      if (++spins > 512) std::this_thread::yield();
  }

 private:
  int n_ = 1;
  std::atomic<int> count_{0};
  std::atomic<int> gen_{0};
};

// Runs f(tid, team) on a team of up to nth threads (the caller's is tid 0).  The
// threads wait until the team is complete; if one cannot be started the team is
// smaller, and bar is sized for the team that runs.
template <typename F>
void run_team(int nth, SpinBarrier& bar, F f) {
  std::atomic<int> go{0};
  int team = nth;
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < nth; ++t)
      pool.emplace_back([&, t] {
        while (!go.load(std::memory_order_acquire)) std::this_thread::yield();
        f(t, team);
      });
  } catch (...) {
    team = 1 + (int)pool.size();
  }
  bar.reset(team);
  go.store(1, std::memory_order_release);
  f(0, team);
  for (auto& th : pool) th.join();
}

// Implicit QL on a symmetric tridiagonal matrix (diagonal d[0..m), off-diagonal
// e[0..m-1) with e[i] = T[i][i+1]).  If Zt is given (m x cols row-major, rows are the
// current basis vectors, or their first cols components), every plane rotation is
// applied to rows i, i+1 of Zt.
int tql(int m, double* d, double* e_in, double* Zt, int cols = -1, SymEig* log = nullptr) {
  if (cols < 0) cols = m;
  std::vector<double> e(m, 0.0);
  for (int i = 0; i + 1 < m; ++i) e[i] = e_in[i];
  // absolute floor for negligible couplings (exactly decoupled blocks with zero
  // diagonal, as left by an exhausted Krylov space, must not stall the iteration)
  double scale = 0.0;
  for (int i = 0; i < m; ++i) scale = std::max(scale, std::fabs(d[i]) + (i + 1 < m ? std::fabs(e[i]) : 0.0));
  const double floor_abs = 1e-16 * scale;
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    while (true) {
      int mm = l;
      for (; mm < m - 1; ++mm) {
        const double dd = std::fabs(d[mm]) + std::fabs(d[mm + 1]);
        if (std::fabs(e[mm]) <= 1e-16 * dd || std::fabs(e[mm]) <= floor_abs) break;
      }
      if (mm == l) break;
      if (++iter > 60) return 1;
      // shift from the leading 2x2 block
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[mm] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = mm - 1;
      bool underflow = false;
      for (; i >= l; --i) {
        double f = s * e[i];
        const double bq = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[mm] = 0.0;
          underflow = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * bq;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - bq;
        if (log) {
          log->ri.push_back(i);
          log->rc.push_back(c);
          log->rs.push_back(s);
        }
        if (Zt) {
          double* zi = Zt + (size_t)i * cols;
          double* zj = Zt + (size_t)(i + 1) * cols;
          for (int k = 0; k < cols; ++k) {
            const double fz = zj[k];
            zj[k] = s * zi[k] + c * fz;
            zi[k] = c * zi[k] - s * fz;
          }
        }
      }
      if (underflow) continue;
      d[l] -= p;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
  return 0;
}

}  // namespace

int tridiag_eigvals(int m, const double* a, const double* b, double* lam) {
  std::vector<double> d(a, a + m), e(m > 1 ? m - 1 : 1, 0.0);
  for (int i = 0; i + 1 < m; ++i) e[i] = b[i];
  if (tql(m, d.data(), e.data(), nullptr)) return 1;
  for (int i = 0; i < m; ++i) lam[i] = d[i];
  return 0;
}

namespace {

// Householder tridiagonalisation of the symmetric part of A (m x m row-major):
// A = Q T Q^T with Q = H_0 H_1 ..., T = tridiag(e, d, e); vs[k] the unit reflector
// of H_k acting on indices k+1.. (empty: identity).
void householder_tridiag(int m, const double* A_in, std::vector<double>& d, std::vector<double>& e,
                         std::vector<std::vector<double>>& vs) {
  std::vector<double> A(A_in, A_in + (size_t)m * m);
  // symmetrise
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) {
      const double v = 0.5 * (A[(size_t)i * m + j] + A[(size_t)j * m + i]);
      A[(size_t)i * m + j] = A[(size_t)j * m + i] = v;
    }
  // Householder reduction: for column k, reflect x = A[k+1:, k] onto alpha e_1.  The
  // two O(len^2) passes of a step (p = A22 v and the rank-2 update) split the rows of
  // A22 over a team of threads; every row is computed exactly as by one thread.
  const int steps = std::max(0, m - 2);
  vs.assign(steps, std::vector<double>());
  d.assign(m, 0.0);
  e.assign(m, 0.0);
  std::vector<double> p(m), q(m), v(m);
  std::vector<char> skip(std::max(steps, 1), 0);
  double K = 0.0;
  SpinBarrier bar;
  auto work = [&](int tid, int nth) {
    for (int k = 0; k < steps; ++k) {
      const int len = m - k - 1;
      if (tid == 0) {
        double nx = 0.0, tail = 0.0;
        for (int i = 0; i < len; ++i) {
          v[i] = A[(size_t)(k + 1 + i) * m + k];
          nx += v[i] * v[i];
          if (i > 0) tail += v[i] * v[i];
        }
        nx = std::sqrt(nx);
        skip[k] = nx == 0.0 || tail == 0.0;  // identity reflector
        if (!skip[k]) {
          const double alpha = v[0] >= 0 ? -nx : nx;
          v[0] -= alpha;
          double nv = 0.0;
          for (int i = 0; i < len; ++i) nv += v[i] * v[i];
          nv = std::sqrt(nv);
          for (int i = 0; i < len; ++i) v[i] /= nv;
          // column / row k become alpha e_1 (A22 is not touched by this)
          A[(size_t)(k + 1) * m + k] = alpha;
          A[(size_t)k * m + k + 1] = alpha;
          for (int i = 1; i < len; ++i) {
            A[(size_t)(k + 1 + i) * m + k] = 0.0;
            A[(size_t)k * m + k + 1 + i] = 0.0;
          }
        }
      }
      bar.wait();
      if (skip[k]) continue;
      const int r0 = (int)((int64_t)len * tid / nth), r1 = (int)((int64_t)len * (tid + 1) / nth);
      // p = A22 v
      for (int i = r0; i < r1; ++i) {
        const double* row = &A[(size_t)(k + 1 + i) * m + k + 1];
        double sum = 0.0;
        for (int j = 0; j < len; ++j) sum += row[j] * v[j];
        p[i] = sum;
      }
      bar.wait();
      if (tid == 0) {  // K = v^T p, q = p - K v
        K = 0.0;
        for (int i = 0; i < len; ++i) K += v[i] * p[i];
        for (int i = 0; i < len; ++i) q[i] = p[i] - K * v[i];
        vs[k].assign(v.begin(), v.begin() + len);
      }
      bar.wait();
      // A22 <- A22 - 2 (v q^T + q v^T)
      for (int i = r0; i < r1; ++i) {
        double* row = &A[(size_t)(k + 1 + i) * m + k + 1];
        const double vi = v[i], qi = q[i];
        for (int j = 0; j < len; ++j) row[j] -= 2.0 * (vi * q[j] + qi * v[j]);
      }
      bar.wait();
    }
  };
  run_team(m >= 160 ? host_threads(m / 32) : 1, bar, work);
  for (int i = 0; i < m; ++i) d[i] = A[(size_t)i * m + i];
  for (int i = 0; i + 1 < m; ++i) e[i] = A[(size_t)i * m + i + 1];
}

}  // namespace

// A = U diag(lam) U^T; U row-major, column i is the eigenvector of lam[i].
int dense_syev(int m, const double* A_in, double* lam, double* U) {
  if (m <= 0) return 0;
  std::vector<double> d, e;
  std::vector<std::vector<double>> vs;
  householder_tridiag(m, A_in, d, e, vs);
  // Zt = Q^T with Q = H_0 H_1 ... ; rows of Zt are columns of Q.
  // Build Q by applying the reflectors in reverse to the identity, stored transposed.
  std::vector<double> Zt((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Zt[(size_t)i * m + i] = 1.0;
  for (int k = (int)vs.size() - 1; k >= 0; --k) {
    const auto& v = vs[k];
    if (v.empty()) continue;
    const int off = k + 1, len = m - off;
    // Q <- H_k Q, H_k acts on rows off.. of Q, i.e. on columns off.. of Zt
    for (int r = 0; r < m; ++r) {
      double* z = &Zt[(size_t)r * m + off];
      double s = 0.0;
      for (int i = 0; i < len; ++i) s += z[i] * v[i];
      s *= 2.0;
      for (int i = 0; i < len; ++i) z[i] -= s * v[i];
    }
  }
  if (tql(m, d.data(), e.data(), Zt.data())) return 1;
  // sort ascending
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int c = 0; c < m; ++c) {
    const int s = idx[c];
    lam[c] = d[s];
    for (int r = 0; r < m; ++r) U[(size_t)r * m + c] = Zt[(size_t)s * m + r];
  }
  return 0;
}

// Eigenvalues (ascending) and the first kr rows of the eigenvector matrix:
// Ur (kr x m row-major), Ur[r][c] = component r of the eigenvector of lam[c].  The
// rows of Q needed are e_r^T H_0 H_1 ..., and the QL rotations act on kr components
// only: O(m^3) for the reduction, O(kr m^2) for the vectors.
int dense_syev_rows(int m, const double* A_in, int kr, double* lam, double* Ur) {
  if (m <= 0) return 0;
  kr = std::min(kr, m);
  std::vector<double> d, e;
  std::vector<std::vector<double>> vs;
  householder_tridiag(m, A_in, d, e, vs);
  // Zt (m x kr): Zt[j][r] = Q[r][j]
  std::vector<double> Zt((size_t)m * kr, 0.0), x(m);
  for (int r = 0; r < kr; ++r) {
    std::fill(x.begin(), x.end(), 0.0);
    x[r] = 1.0;
    for (size_t k = 0; k < vs.size(); ++k) {
      const auto& v = vs[k];
      if (v.empty()) continue;
      const int off = (int)k + 1, len = m - off;
      double s = 0.0;
      for (int i = 0; i < len; ++i) s += x[off + i] * v[i];
      s *= 2.0;
      for (int i = 0; i < len; ++i) x[off + i] -= s * v[i];
    }
    for (int j = 0; j < m; ++j) Zt[(size_t)j * kr + r] = x[j];
  }
  if (tql(m, d.data(), e.data(), Zt.data(), kr)) return 1;
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int c = 0; c < m; ++c) {
    const int s = idx[c];
    lam[c] = d[s];
    for (int r = 0; r < kr; ++r) Ur[(size_t)r * m + c] = Zt[(size_t)s * kr + r];
  }
  return 0;
}

int sym_eig_factor(int m, const double* A_in, SymEig& E) {
  E = SymEig();
  E.m = m;
  if (m <= 0) return 0;
  std::vector<double> d, e;
  householder_tridiag(m, A_in, d, e, E.vs);
  if (tql(m, d.data(), e.data(), nullptr, -1, &E)) return 1;
  E.lam = std::move(d);
  return 0;
}

namespace {

constexpr int SYM_COLS = 8;  // columns moved through the reflectors and rotations together

// Applies f(x) to the m x b block X in groups of SYM_COLS columns: x holds the group
// row-major (m x SYM_COLS, missing columns zero), so a reflector or rotation updates
// SYM_COLS independent values per row; the groups are split over host threads.
template <typename F>
void per_column_group(int m, int b, double* X, F f) {
  const int ng = (b + SYM_COLS - 1) / SYM_COLS;
  auto groups = [&](int g0, int g1) {
    std::vector<double> x((size_t)m * SYM_COLS);
    for (int gi = g0; gi < g1; ++gi) {
      const int c0 = gi * SYM_COLS, nc = std::min(SYM_COLS, b - c0);
      for (int i = 0; i < m; ++i)
        for (int c = 0; c < SYM_COLS; ++c) x[(size_t)i * SYM_COLS + c] = c < nc ? X[(size_t)i * b + c0 + c] : 0.0;
      f(x.data());
      for (int i = 0; i < m; ++i)
        for (int c = 0; c < nc; ++c) X[(size_t)i * b + c0 + c] = x[(size_t)i * SYM_COLS + c];
    }
  };
  const int nth = (int64_t)m * m * b < (1 << 22) ? 1 : host_threads(ng);
  std::vector<std::thread> pool;
  int started = 1;
  try {
    for (; started < nth; ++started) pool.emplace_back(groups, ng * started / nth, ng * (started + 1) / nth);
  } catch (...) {  // no thread to be had: the caller's thread takes the rest
  }
  groups(0, ng / nth);
  for (auto& th : pool) th.join();
  if (started < nth) groups(ng * started / nth, ng);
}

// x (rows of SYM_COLS values) <- H x for the reflector v acting on rows off..
inline void reflect_rows(double* x, int off, const std::vector<double>& v) {
  double s[SYM_COLS] = {};
  for (size_t i = 0; i < v.size(); ++i) {
    const double* r = x + (size_t)(off + i) * SYM_COLS;
    for (int c = 0; c < SYM_COLS; ++c) s[c] += r[c] * v[i];
  }
  for (int c = 0; c < SYM_COLS; ++c) s[c] *= 2.0;
  for (size_t i = 0; i < v.size(); ++i) {
    double* r = x + (size_t)(off + i) * SYM_COLS;
    for (int c = 0; c < SYM_COLS; ++c) r[c] -= s[c] * v[i];
  }
}

}  // namespace

void sym_eig_apply_ut(const SymEig& E, int b, double* X) {
  const int m = E.m;
  if (m <= 0 || b <= 0) return;
  per_column_group(m, b, X, [&](double* x) {
    // Q^T = H_last ... H_0: reflectors in order
    for (size_t k = 0; k < E.vs.size(); ++k)
      if (!E.vs[k].empty()) reflect_rows(x, (int)k + 1, E.vs[k]);
    // then the QL rotations in the order they were made
    for (size_t r = 0; r < E.ri.size(); ++r) {
      double* xi = x + (size_t)E.ri[r] * SYM_COLS;
      double* xj = xi + SYM_COLS;
      const double c = E.rc[r], s = E.rs[r];
      for (int q = 0; q < SYM_COLS; ++q) {
        const double a = xi[q], bq = xj[q];
        xj[q] = s * a + c * bq;
        xi[q] = c * a - s * bq;
      }
    }
  });
}

void sym_eig_apply_u(const SymEig& E, int b, double* X) {
  const int m = E.m;
  if (m <= 0 || b <= 0) return;
  per_column_group(m, b, X, [&](double* x) {
    // the transposed rotations in reverse order
    for (size_t r = E.ri.size(); r-- > 0;) {
      double* xi = x + (size_t)E.ri[r] * SYM_COLS;
      double* xj = xi + SYM_COLS;
      const double c = E.rc[r], s = E.rs[r];
      for (int q = 0; q < SYM_COLS; ++q) {
        const double a = xi[q], bq = xj[q];
        xi[q] = c * a + s * bq;
        xj[q] = c * bq - s * a;
      }
    }
    // Q = H_0 ... H_last: reflectors in reverse order
    for (size_t k = E.vs.size(); k-- > 0;)
      if (!E.vs[k].empty()) reflect_rows(x, (int)k + 1, E.vs[k]);
  });
}

namespace {
// lower Cholesky in place of a b x b SPD block; returns nonzero if not SPD
int chol_lower(int b, double* A) {
  for (int j = 0; j < b; ++j) {
    double s = A[j * b + j];
    for (int k = 0; k < j; ++k) s -= A[j * b + k] * A[j * b + k];
    if (!(s > 0.0)) return 1;
    const double ljj = std::sqrt(s);
    A[j * b + j] = ljj;
    for (int i = j + 1; i < b; ++i) {
      double t = A[i * b + j];
      for (int k = 0; k < j; ++k) t -= A[i * b + k] * A[j * b + k];
      A[i * b + j] = t / ljj;
    }
    for (int k = j + 1; k < b; ++k) A[j * b + k] = 0.0;
  }
  return 0;
}
// X <- L^{-1} X (X is b x nrhs)
void lsolve(int b, const double* L, double* X, int nrhs) {
  for (int i = 0; i < b; ++i) {
    for (int c = 0; c < nrhs; ++c) {
      double s = X[i * nrhs + c];
      for (int k = 0; k < i; ++k) s -= L[i * b + k] * X[k * nrhs + c];
      X[i * nrhs + c] = s / L[i * b + i];
    }
  }
}
// X <- L^{-T} X
void ltsolve(int b, const double* L, double* X, int nrhs) {
  for (int i = b - 1; i >= 0; --i) {
    for (int c = 0; c < nrhs; ++c) {
      double s = X[i * nrhs + c];
      for (int k = i + 1; k < b; ++k) s -= L[k * b + i] * X[k * nrhs + c];
      X[i * nrhs + c] = s / L[i * b + i];
    }
  }
}
}  // namespace

int block_tridiag_solve(int K, int b, const double* Ad, const double* Bo, const double* B, int nrhs, double* X) {
  const int bb = b * b;
  std::vector<double> L((size_t)K * bb), Mb((size_t)K * bb, 0.0);
  for (int j = 0; j < K; ++j) {
    double* Lj = &L[(size_t)j * bb];
    std::memcpy(Lj, Ad + (size_t)j * bb, sizeof(double) * bb);
    for (int r = 0; r < b; ++r)  // symmetrise
      for (int c = r + 1; c < b; ++c) Lj[r * b + c] = Lj[c * b + r] = 0.5 * (Lj[r * b + c] + Lj[c * b + r]);
    if (j > 0) {
      // M_j = B_{j-1} L_{j-1}^{-T}:  solve M L^T = B  <=>  L M^T = B^T
      double* Mj = &Mb[(size_t)j * bb];
      std::vector<double> Bt(bb);
      const double* Bj = Bo + (size_t)(j - 1) * bb;
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) Bt[r * b + c] = Bj[c * b + r];
      lsolve(b, &L[(size_t)(j - 1) * bb], Bt.data(), b);  // Bt = M^T
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) Mj[r * b + c] = Bt[c * b + r];
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) {
          double s = 0.0;
          for (int k = 0; k < b; ++k) s += Mj[r * b + k] * Mj[c * b + k];
          Lj[r * b + c] -= s;
        }
    }
    if (chol_lower(b, Lj)) return 1;
  }
  std::memcpy(X, B, sizeof(double) * (size_t)K * b * nrhs);
  for (int j = 0; j < K; ++j) {
    double* xj = X + (size_t)j * b * nrhs;
    if (j > 0) {
      const double* xp = X + (size_t)(j - 1) * b * nrhs;
      const double* Mj = &Mb[(size_t)j * bb];
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < nrhs; ++c) {
          double s = 0.0;
          for (int k = 0; k < b; ++k) s += Mj[r * b + k] * xp[k * nrhs + c];
          xj[r * nrhs + c] -= s;
        }
    }
    lsolve(b, &L[(size_t)j * bb], xj, nrhs);
  }
  for (int j = K - 1; j >= 0; --j) {
    double* xj = X + (size_t)j * b * nrhs;
    if (j + 1 < K) {
      const double* xn = X + (size_t)(j + 1) * b * nrhs;
      const double* Mn = &Mb[(size_t)(j + 1) * bb];
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < nrhs; ++c) {
          double s = 0.0;
          for (int k = 0; k < b; ++k) s += Mn[k * b + r] * xn[k * nrhs + c];
          xj[r * nrhs + c] -= s;
        }
    }
    ltsolve(b, &L[(size_t)j * bb], xj, nrhs);
  }
  return 0;
}

// ------------------------------------------------------------------ deflating Cholesky
void host_chol_deflate(int M, const std::vector<double>& G, double tol, double ref, std::vector<double>& R,
                       std::vector<double>& Rinv, std::vector<char>& keep) {
  R.assign((size_t)M * M, 0.0);
  Rinv.assign((size_t)M * M, 0.0);
  keep.assign(M, 0);
  for (int k = 0; k < M; ++k) {
    double d = G[(size_t)k * M + k];
    for (int i = 0; i < k; ++i) d -= R[(size_t)i * M + k] * R[(size_t)i * M + k];
    if (!(d > tol * ref)) continue;
    keep[k] = 1;
    const double rkk = std::sqrt(d);
    R[(size_t)k * M + k] = rkk;
    for (int j = k + 1; j < M; ++j) {
      double s = G[(size_t)k * M + j];
      for (int i = 0; i < k; ++i) s -= R[(size_t)i * M + k] * R[(size_t)i * M + j];
      R[(size_t)k * M + j] = s / rkk;
    }
  }
  // Rinv: R Rinv = I on the kept indices (upper triangular, back substitution)
  for (int c = 0; c < M; ++c) {
    if (!keep[c]) continue;
    for (int i = c; i >= 0; --i) {
      if (!keep[i]) continue;
      double s = (i == c) ? 1.0 : 0.0;
      for (int j = i + 1; j <= c; ++j)
        if (keep[j]) s -= R[(size_t)i * M + j] * Rinv[(size_t)j * M + c];
      Rinv[(size_t)i * M + c] = s / R[(size_t)i * M + i];
    }
  }
}

// ------------------------------------------------------------------ phi_1 of a general matrix
namespace {

typedef double wl_v4d __attribute__((vector_size(32)));  // four doubles (GCC / Clang vector extension)

// C = A B for m x m row-major matrices on rows [r0, r1): 4 x 8 register tiles, k in
// blocks of 128 rows of B (which stay in cache while a thread's rows pass over them).
#define WL_MATMUL_ROWS_BODY                                                                              \
  constexpr int KB = 128;                                                                                \
  for (int i = r0; i < r1; ++i) std::fill(C + (size_t)i * m, C + (size_t)i * m + m, 0.0);                 \
  for (int k0 = 0; k0 < m; k0 += KB) {                                                                   \
    const int k1 = std::min(m, k0 + KB);                                                                 \
    for (int i = r0; i < r1; i += 4) {                                                                   \
      const int ni = std::min(4, r1 - i);                                                                \
      for (int j = 0; j < m; j += 8) {                                                                   \
        const int nj = std::min(8, m - j);                                                               \
        if (ni == 4 && nj == 8) { /* eight 4-wide accumulators in registers */                            \
          const double* a0 = A + (size_t)i * m;                                                          \
          wl_v4d c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00, c20 = c00, c21 = c00, c30 = c00,      \
                 c31 = c00;                                                                              \
          for (int k = k0; k < k1; ++k) {                                                                \
            const double* b = B + (size_t)k * m + j;                                                     \
            wl_v4d b0, b1;                                                                               \
            __builtin_memcpy(&b0, b, sizeof(b0));                                                        \
            __builtin_memcpy(&b1, b + 4, sizeof(b1));                                                    \
            const double x0 = a0[k], x1 = a0[m + k], x2 = a0[2 * (size_t)m + k], x3 = a0[3 * (size_t)m + k]; \
            c00 += x0 * b0;                                                                              \
            c01 += x0 * b1;                                                                              \
            c10 += x1 * b0;                                                                              \
            c11 += x1 * b1;                                                                              \
            c20 += x2 * b0;                                                                              \
            c21 += x2 * b1;                                                                              \
            c30 += x3 * b0;                                                                              \
            c31 += x3 * b1;                                                                              \
          }                                                                                              \
          const wl_v4d cs[4][2] = {{c00, c01}, {c10, c11}, {c20, c21}, {c30, c31}};                      \
          for (int ii = 0; ii < 4; ++ii) {                                                               \
            double* cr = C + (size_t)(i + ii) * m + j;                                                   \
            for (int jj = 0; jj < 8; ++jj) cr[jj] += cs[ii][jj >> 2][jj & 3];                            \
          }                                                                                              \
        } else {                                                                                         \
          for (int ii = 0; ii < ni; ++ii)                                                                \
            for (int k = k0; k < k1; ++k) {                                                              \
              const double x = A[(size_t)(i + ii) * m + k];                                              \
              for (int jj = 0; jj < nj; ++jj) C[(size_t)(i + ii) * m + j + jj] += x * B[(size_t)k * m + j + jj]; \
            }                                                                                            \
        }                                                                                                \
      }                                                                                                  \
    }                                                                                                    \
  }

// P <- (L U)^{-1} Pi P on columns [c0, c1) (P m x m row-major): the recorded row swaps,
// then the unit lower triangle L and the upper triangle U of the factored Q, row by row
// (each row of P takes the earlier rows' multiples, reading a row of Q at a time).
#define WL_LU_SOLVE_COLS_BODY                                                                            \
  for (int k = 0; k < m; ++k)                                                                            \
    if (piv[k] != k)                                                                                     \
      for (int j = c0; j < c1; ++j) std::swap(P[(size_t)piv[k] * m + j], P[(size_t)k * m + j]);          \
  for (int i = 1; i < m; ++i) {                                                                          \
    double* pi = P + (size_t)i * m;                                                                      \
    const double* qi = Q + (size_t)i * m;                                                                \
    for (int k = 0; k < i; ++k) {                                                                        \
      const double f = qi[k];                                                                            \
      if (f == 0.0) continue;                                                                            \
      const double* pk = P + (size_t)k * m;                                                              \
      for (int j = c0; j < c1; ++j) pi[j] -= f * pk[j];                                                  \
    }                                                                                                    \
  }                                                                                                      \
  for (int i = m - 1; i >= 0; --i) {                                                                     \
    double* pi = P + (size_t)i * m;                                                                      \
    const double* qi = Q + (size_t)i * m;                                                                \
    for (int k = i + 1; k < m; ++k) {                                                                    \
      const double f = qi[k];                                                                            \
      if (f == 0.0) continue;                                                                            \
      const double* pk = P + (size_t)k * m;                                                              \
      for (int j = c0; j < c1; ++j) pi[j] -= f * pk[j];                                                  \
    }                                                                                                    \
    const double inv = 1.0 / qi[i];                                                                      \
    for (int j = c0; j < c1; ++j) pi[j] *= inv;                                                          \
  }

void matmul_rows_base(int m, const double* A, const double* B, double* C, int r0, int r1) { WL_MATMUL_ROWS_BODY }
void lu_solve_cols_base(int m, const double* Q, const int* piv, double* P, int c0, int c1) {
  WL_LU_SOLVE_COLS_BODY
}
#if !defined(__HIP_DEVICE_COMPILE__) && (defined(__x86_64__) || defined(_M_X64))
// the same code compiled for AVX2 with FMA, taken when the host has them
__attribute__((target("avx2,fma"))) void matmul_rows_avx2(int m, const double* A, const double* B, double* C, int r0,
                                                          int r1) {
  WL_MATMUL_ROWS_BODY
}
__attribute__((target("avx2,fma"))) void lu_solve_cols_avx2(int m, const double* Q, const int* piv, double* P,
                                                            int c0, int c1) {
  WL_LU_SOLVE_COLS_BODY
}
bool host_has_avx2() {
  static const bool yes = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
  return yes;
}
#endif
#undef WL_MATMUL_ROWS_BODY
#undef WL_LU_SOLVE_COLS_BODY

void matmul_rows(int m, const double* A, const double* B, double* C, int r0, int r1) {
#if !defined(__HIP_DEVICE_COMPILE__) && (defined(__x86_64__) || defined(_M_X64))
  if (host_has_avx2()) return matmul_rows_avx2(m, A, B, C, r0, r1);
#endif
  matmul_rows_base(m, A, B, C, r0, r1);
}

void lu_solve_cols(int m, const double* Q, const int* piv, double* P, int c0, int c1) {
#if !defined(__HIP_DEVICE_COMPILE__) && (defined(__x86_64__) || defined(_M_X64))
  if (host_has_avx2()) return lu_solve_cols_avx2(m, Q, piv, P, c0, c1);
#endif
  lu_solve_cols_base(m, Q, piv, P, c0, c1);
}

// exp(A) by scaling and squaring with the [13/13] Pade approximant (Higham, SIAM J.
// Matrix Anal. Appl. 26, 2005): s with ||A / 2^s||_1 <= theta_13, r_13 = (V - U)^{-1}
// (V + U) from the even and odd parts, then s squarings.  One team of host threads does
// it all: the products by row ranges, the LU factorisation of V - U (partial pivoting)
// by rows below the pivot, the triangular solves by column ranges of V + U.
int dense_expm(int m, std::vector<double>& A) {
  static const double b[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0, 1187353796428800.0,
                               129060195264000.0,   10559470521600.0,    670442572800.0,     33522128640.0,
                               1323241920.0,        40840800.0,          960960.0,           16380.0,
                               182.0,               1.0};
  const double theta13 = 5.371920351148152;
  double nrm = 0.0;
  for (int j = 0; j < m; ++j) {
    double c = 0.0;
    for (int i = 0; i < m; ++i) c += std::fabs(A[(size_t)i * m + j]);
    nrm = std::max(nrm, c);
  }
  if (!std::isfinite(nrm)) return 1;
  int sq = 0;
  if (nrm > theta13) sq = (int)std::ceil(std::log2(nrm / theta13));
  const double sc = std::ldexp(1.0, -sq);
  for (double& x : A) x *= sc;
  const size_t mm = (size_t)m * m;
  std::vector<double> A2(mm), A4(mm), A6(mm), T1(mm), U(mm), V(mm), W(mm);
  std::vector<int> piv(m);
  std::atomic<int> singular{0};
  SpinBarrier bar;
  const int nth = m >= 96 ? host_threads(m / 32) : 1;
  run_team(nth, bar, [&](int tid, int team) {
    const int per = (m + team - 1) / team;
    const int r0 = std::min(m, tid * per), r1 = std::min(m, r0 + per);
    auto mul = [&](const double* X, const double* Y, double* Z) {
      matmul_rows(m, X, Y, Z, r0, r1);
      bar.wait();
    };
    auto rows = [&](auto f) {  // elementwise work on this thread's rows, then the barrier
      for (int i = r0; i < r1; ++i) f(i);
      bar.wait();
    };
    mul(A.data(), A.data(), A2.data());
    mul(A2.data(), A2.data(), A4.data());
    mul(A4.data(), A2.data(), A6.data());
    rows([&](int i) {
      for (size_t e = (size_t)i * m; e < (size_t)(i + 1) * m; ++e) T1[e] = b[13] * A6[e] + b[11] * A4[e] + b[9] * A2[e];
    });
    mul(A6.data(), T1.data(), W.data());
    rows([&](int i) {
      for (size_t e = (size_t)i * m; e < (size_t)(i + 1) * m; ++e) W[e] += b[7] * A6[e] + b[5] * A4[e] + b[3] * A2[e];
      W[(size_t)i * m + i] += b[1];
    });
    mul(A.data(), W.data(), U.data());  // the odd part U = A (...)
    rows([&](int i) {
      for (size_t e = (size_t)i * m; e < (size_t)(i + 1) * m; ++e) T1[e] = b[12] * A6[e] + b[10] * A4[e] + b[8] * A2[e];
    });
    mul(A6.data(), T1.data(), V.data());
    // P = V + U (into A2), Q = V - U (into A4)
    rows([&](int i) {
      for (size_t e = (size_t)i * m; e < (size_t)(i + 1) * m; ++e) {
        const double v = V[e] + b[6] * A6[e] + b[4] * A4[e] + b[2] * A2[e] + (e == (size_t)i * m + i ? b[0] : 0.0);
        A2[e] = v + U[e];
        A4[e] = v - U[e];
      }
    });
    double* P = A2.data();
    double* Q = A4.data();
    // Q = L U with partial pivoting, the row swaps recorded (rows swapped whole, so the
    // multipliers move with them)
    for (int k = 0; k < m; ++k) {
      if (tid == 0) {
        int p = k;
        for (int i = k + 1; i < m; ++i)
          if (std::fabs(Q[(size_t)i * m + k]) > std::fabs(Q[(size_t)p * m + k])) p = i;
        piv[k] = p;
        if (Q[(size_t)p * m + k] == 0.0) {
          singular.store(1);
        } else if (p != k) {
          for (int j = 0; j < m; ++j) std::swap(Q[(size_t)p * m + j], Q[(size_t)k * m + j]);
        }
      }
      bar.wait();
      if (singular.load()) return;
      const double inv = 1.0 / Q[(size_t)k * m + k];
      const int rem = m - k - 1, per2 = (rem + team - 1) / team;
      const int i0 = k + 1 + std::min(rem, tid * per2), i1 = k + 1 + std::min(rem, (tid + 1) * per2);
      for (int i = i0; i < i1; ++i) {
        const double f = Q[(size_t)i * m + k] * inv;
        Q[(size_t)i * m + k] = f;
        if (f == 0.0) continue;
        for (int j = k + 1; j < m; ++j) Q[(size_t)i * m + j] -= f * Q[(size_t)k * m + j];
      }
      bar.wait();
    }
    // P <- Q^{-1} P on this thread's columns: the swaps, then L, then U
    const int cper = (m + team - 1) / team;
    const int c0 = std::min(m, tid * cper), c1 = std::min(m, c0 + cper);
    if (c0 < c1) lu_solve_cols(m, Q, piv.data(), P, c0, c1);
    bar.wait();
    double* cur = P;
    double* nxt = T1.data();
    for (int k = 0; k < sq; ++k) {
      mul(cur, cur, nxt);
      std::swap(cur, nxt);
    }
    if (tid == 0) std::copy(cur, cur + mm, A.begin());
  });
  return singular.load() ? 1 : 0;
}

}  // namespace

int dense_phi1_times(int m, const double* M, int k, const double* B, double* out) {
  // phi_1(M) B is the top-right block of exp([[M, B], [0, 0]])
  const int a = m + k;
  std::vector<double> E((size_t)a * a, 0.0);
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) E[(size_t)i * a + j] = M[(size_t)i * m + j];
    for (int j = 0; j < k; ++j) E[(size_t)i * a + m + j] = B[(size_t)i * k + j];
  }
  if (dense_expm(a, E)) return 1;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < k; ++j) out[(size_t)i * k + j] = E[(size_t)i * a + m + j];
  return 0;
}
