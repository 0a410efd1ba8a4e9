// Host-side numerical kernels of the library (dense eigensolvers, block-tridiagonal
// solve, CholQR deflation, phi_1, AAA poles of exp(-x), the multigrid hierarchy)
// driven on small inputs, for a build with AddressSanitizer and UndefinedBehavior-
// Sanitizer.  Each case also checks its defining property (residual, orthogonality,
// reconstruction), so a memory error, undefined behaviour or a wrong result all end in
// a non-zero exit status.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "wl_amg.h"
#include "wl_internal.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what, double v) {
  std::printf("%-52s %s (%.3g)\n", what, ok ? "ok" : "FAILED", v);
  if (!ok) ++failures;
}

std::vector<double> random_symmetric(int m, std::mt19937_64& rng) {
  std::normal_distribution<double> nd;
  std::vector<double> A((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) A[(size_t)i * m + j] = A[(size_t)j * m + i] = nd(rng);
  return A;
}

// max |A U - U diag(lam)| and max |U^T U - I|
void eig_residuals(int m, const std::vector<double>& A, const std::vector<double>& lam, const std::vector<double>& U,
                   double* res, double* orth) {
  *res = *orth = 0.0;
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < m; ++k) {
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += A[(size_t)i * m + j] * U[(size_t)j * m + k];
      *res = std::max(*res, std::fabs(s - lam[k] * U[(size_t)i * m + k]));
    }
  for (int a = 0; a < m; ++a)
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += U[(size_t)i * m + a] * U[(size_t)i * m + c];
      *orth = std::max(*orth, std::fabs(s - (a == c ? 1.0 : 0.0)));
    }
}

void check_dense(std::mt19937_64& rng) {
  for (int m : {1, 2, 7, 64, 150}) {
    std::vector<double> A = random_symmetric(m, rng), lam(m), U((size_t)m * m);
    const int st = dense_syev(m, A.data(), lam.data(), U.data());
    double res, orth;
    eig_residuals(m, A, lam, U, &res, &orth);
    char what[96];
    std::snprintf(what, sizeof(what), "dense_syev m=%d", m);
    expect(st == 0 && res < 1e-10 * m && orth < 1e-12 * m, what, res + orth);
    // the first kr rows only
    const int kr = std::max(1, m / 3);
    std::vector<double> lam2(m), Ur((size_t)kr * m);
    const int st2 = dense_syev_rows(m, A.data(), kr, lam2.data(), Ur.data());
    double d = 0.0;
    for (int i = 0; i < m; ++i) d = std::max(d, std::fabs(lam2[i] - lam[i]));
    // rows agree up to the sign of each eigenvector
    for (int k = 0; k < m; ++k) {
      double sgn = 0.0;
      for (int i = 0; i < kr && sgn == 0.0; ++i)
        if (std::fabs(U[(size_t)i * m + k]) > 1e-6) sgn = (U[(size_t)i * m + k] > 0) == (Ur[(size_t)i * m + k] > 0) ? 1 : -1;
      if (sgn == 0.0) sgn = 1.0;
      for (int i = 0; i < kr; ++i) d = std::max(d, std::fabs(sgn * Ur[(size_t)i * m + k] - U[(size_t)i * m + k]));
    }
    std::snprintf(what, sizeof(what), "dense_syev_rows m=%d kr=%d", m, kr);
    expect(st2 == 0 && d < 1e-8, what, d);
    // tridiagonal eigenvalues against the dense solver
    std::vector<double> a(m), b(std::max(m - 1, 1)), T((size_t)m * m, 0.0), lt(m), lu(m), Ut((size_t)m * m);
    std::normal_distribution<double> nd;
    for (int i = 0; i < m; ++i) a[i] = T[(size_t)i * m + i] = nd(rng);
    for (int i = 0; i + 1 < m; ++i) b[i] = T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = nd(rng);
    const int st3 = tridiag_eigvals(m, a.data(), b.data(), lt.data());
    dense_syev(m, T.data(), lu.data(), Ut.data());
    std::sort(lt.begin(), lt.end());
    std::sort(lu.begin(), lu.end());
    d = 0.0;
    for (int i = 0; i < m; ++i) d = std::max(d, std::fabs(lt[i] - lu[i]));
    std::snprintf(what, sizeof(what), "tridiag_eigvals m=%d", m);
    expect(st3 == 0 && d < 1e-10 * m, what, d);
  }
}

// the factored eigendecomposition: U (U^T X) = X and U diag(lam) U^T X = A X, on a dense
// matrix and on a block tridiagonal one (the shape of the projected Krylov matrices)
void check_sym_eig(std::mt19937_64& rng) {
  std::normal_distribution<double> nd;
  for (int m : {1, 3, 150, 400, 1280}) {
    const int b = m >= 1000 ? 8 : 5;
    std::vector<double> A((size_t)m * m, 0.0);
    const int band = m >= 400 ? 32 : m;  // block tridiagonal bandwidth for the large cases
    for (int i = 0; i < m; ++i)
      for (int j = std::max(0, i - band); j <= i; ++j) A[(size_t)i * m + j] = A[(size_t)j * m + i] = nd(rng);
    SymEig E;
    const int st = sym_eig_factor(m, A.data(), E);
    std::vector<double> X((size_t)m * b), Y, Z;
    for (double& v : X) v = nd(rng);
    Y = X;
    sym_eig_apply_ut(E, b, Y.data());
    Z = Y;
    sym_eig_apply_u(E, b, Z.data());
    double orth = 0.0;
    for (size_t i = 0; i < X.size(); ++i) orth = std::max(orth, std::fabs(Z[i] - X[i]));
    for (int i = 0; i < m; ++i)
      for (int c = 0; c < b; ++c) Y[(size_t)i * b + c] *= E.lam[i];
    sym_eig_apply_u(E, b, Y.data());
    double res = 0.0;
    for (int i = 0; i < m; ++i)
      for (int c = 0; c < b; ++c) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += A[(size_t)i * m + j] * X[(size_t)j * b + c];
        res = std::max(res, std::fabs(s - Y[(size_t)i * b + c]));
      }
    char what[96];
    std::snprintf(what, sizeof(what), "sym_eig factored m=%d b=%d", m, b);
    expect(st == 0 && (int)E.lam.size() == m && orth < 1e-11 && res < 1e-10 * std::sqrt((double)m), what,
           std::max(orth, res));
  }
}

void check_block_tridiag(std::mt19937_64& rng) {
  std::normal_distribution<double> nd;
  for (int K : {1, 3, 9}) {
    const int b = 4, m = K * b, nrhs = 3;
    // SPD block tridiagonal: diagonally dominant blocks
    std::vector<double> Ad((size_t)K * b * b), Bo((size_t)std::max(K - 1, 1) * b * b), T((size_t)m * m, 0.0);
    for (int j = 0; j + 1 < K; ++j)
      for (int e = 0; e < b * b; ++e) Bo[(size_t)j * b * b + e] = 0.3 * nd(rng);
    for (int j = 0; j < K; ++j) {
      for (int r = 0; r < b; ++r)
        for (int c = 0; c <= r; ++c) {
          const double v = r == c ? 8.0 + std::fabs(nd(rng)) : 0.2 * nd(rng);
          Ad[(size_t)j * b * b + r * b + c] = Ad[(size_t)j * b * b + c * b + r] = v;
        }
    }
    for (int j = 0; j < K; ++j)
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) {
          T[(size_t)(j * b + r) * m + j * b + c] = Ad[(size_t)j * b * b + r * b + c];
          if (j + 1 < K) {
            const double v = Bo[(size_t)j * b * b + r * b + c];  // T_{j+1, j}
            T[(size_t)((j + 1) * b + r) * m + j * b + c] = v;
            T[(size_t)(j * b + c) * m + (j + 1) * b + r] = v;
          }
        }
    std::vector<double> B((size_t)m * nrhs), X((size_t)m * nrhs);
    for (double& v : B) v = nd(rng);
    const int st = block_tridiag_solve(K, b, Ad.data(), Bo.data(), B.data(), nrhs, X.data());
    double res = 0.0;
    for (int i = 0; i < m; ++i)
      for (int c = 0; c < nrhs; ++c) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += T[(size_t)i * m + j] * X[(size_t)j * nrhs + c];
        res = std::max(res, std::fabs(s - B[(size_t)i * nrhs + c]));
      }
    char what[96];
    std::snprintf(what, sizeof(what), "block_tridiag_solve K=%d b=%d", K, b);
    expect(st == 0 && res < 1e-12, what, res);
  }
}

void check_chol_deflate(std::mt19937_64& rng) {
  std::normal_distribution<double> nd;
  const int n = 40, M = 6;
  std::vector<double> W((size_t)n * M);
  for (double& v : W) v = nd(rng);
  for (int i = 0; i < n; ++i) W[(size_t)i * M + 4] = W[(size_t)i * M + 1];  // a dependent column
  for (int i = 0; i < n; ++i) W[(size_t)i * M + 5] = 0.0;                  // a zero column
  std::vector<double> G((size_t)M * M, 0.0), R, Ri;
  std::vector<char> keep;
  double ref = 0.0;
  for (int a = 0; a < M; ++a)
    for (int c = 0; c < M; ++c) {
      for (int i = 0; i < n; ++i) G[(size_t)a * M + c] += W[(size_t)i * M + a] * W[(size_t)i * M + c];
      if (a == c) ref = std::max(ref, G[(size_t)a * M + c]);
    }
  host_chol_deflate(M, G, 1e-12, ref, R, Ri, keep);
  // Q = W Rinv has orthonormal kept columns and zero dropped ones
  double orth = 0.0;
  int kept = 0;
  for (int a = 0; a < M; ++a) kept += keep[a] ? 1 : 0;
  std::vector<double> Q((size_t)n * M, 0.0);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < M; ++c)
      for (int k = 0; k < M; ++k) Q[(size_t)i * M + c] += W[(size_t)i * M + k] * Ri[(size_t)k * M + c];
  for (int a = 0; a < M; ++a)
    for (int c = 0; c < M; ++c) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += Q[(size_t)i * M + a] * Q[(size_t)i * M + c];
      orth = std::max(orth, std::fabs(s - (a == c && keep[a] ? 1.0 : 0.0)));
    }
  expect(kept == 4 && !keep[4] && !keep[5] && orth < 1e-10, "host_chol_deflate (dependent and zero column)", orth);
}

void check_phi1(std::mt19937_64& rng) {
  std::normal_distribution<double> nd;
  // small sizes run on one thread, the larger ones on a team (ragged register tiles:
  // m + k not a multiple of 4 or 8; B's columns put their 1-norms above theta_13, so
  // the squarings run too)
  for (int m : {1, 5, 12, 101, 203}) {
    const int k = m > 12 ? 3 : 2;
    std::vector<double> Mx((size_t)m * m), B((size_t)m * k), out((size_t)m * k);
    const double sc = m > 12 ? (m > 150 ? 0.9 : 0.4) / std::sqrt((double)m) : 0.4;
    for (double& v : Mx) v = sc * nd(rng);
    for (double& v : B) v = nd(rng);
    const int st = dense_phi1_times(m, Mx.data(), k, B.data(), out.data());
    // phi_1(M) B = sum_j M^j B / (j + 1)!
    std::vector<double> term = B, acc((size_t)m * k, 0.0), nxt((size_t)m * k);
    double fact = 1.0;
    for (int j = 0; j < 60; ++j) {
      fact *= (j + 1);
      for (size_t e = 0; e < acc.size(); ++e) acc[e] += term[e] / fact;
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < k; ++c) {
          double s = 0.0;
          for (int q = 0; q < m; ++q) s += Mx[(size_t)r * m + q] * term[(size_t)q * k + c];
          nxt[(size_t)r * k + c] = s;
        }
      term.swap(nxt);
    }
    double d = 0.0, big = 1.0;
    for (size_t e = 0; e < acc.size(); ++e) {
      d = std::max(d, std::fabs(acc[e] - out[e]));
      big = std::max(big, std::fabs(acc[e]));
    }
    char what[96];
    std::snprintf(what, sizeof(what), "dense_phi1_times m=%d", m);
    expect(st == 0 && d < 1e-12 * big, what, d / big);
  }
}

void check_aaa() {
  for (double xmax : {0.5, 20.0, 570.0}) {
    std::vector<std::complex<double>> poles;
    double err = 0.0;
    const int st = exp_poles(xmax, 1e-13, 100, poles, &err);
    // closed under conjugation, none on [0, xmax]
    int unmatched = 0, on_interval = 0;
    for (const auto& p : poles) {
      bool found = false;
      for (const auto& q : poles)
        if (std::abs(q - std::conj(p)) <= 1e-8 * std::max(1.0, std::abs(p))) found = true;
      unmatched += found ? 0 : 1;
      if (std::fabs(p.imag()) < 1e-12 && p.real() >= 0.0 && p.real() <= xmax) ++on_interval;
    }
    char what[96];
    std::snprintf(what, sizeof(what), "exp_poles xmax=%g (%zu poles)", xmax, poles.size());
    expect(st == 0 && !poles.empty() && unmatched == 0 && on_interval == 0 && err < 1e-11, what, err);
  }
  // a rational function with known poles: 1 / ((x + 2)(x + 5)) on [0, 10]
  std::vector<double> Z(400), F(400), z, f, w;
  for (int i = 0; i < 400; ++i) {
    Z[i] = 10.0 * i / 399.0;
    F[i] = 1.0 / ((Z[i] + 2.0) * (Z[i] + 5.0));
  }
  double err = 0.0;
  const int st = aaa_real(400, Z.data(), F.data(), 1e-13, 50, z, f, w, &err);
  std::vector<std::complex<double>> poles;
  const int st2 = aaa_poles(z, w, poles);
  double d2 = 1e9, d5 = 1e9;
  for (const auto& p : poles) {
    d2 = std::min(d2, std::abs(p + 2.0));
    d5 = std::min(d5, std::abs(p + 5.0));
  }
  expect(st == 0 && st2 == 0 && err < 1e-12 && d2 < 1e-8 && d5 < 1e-8, "aaa_real / aaa_poles on 1/((x+2)(x+5))",
         std::max(d2, d5));
}

void check_amg(std::mt19937_64& rng) {
  // a 40 x 40 lattice with 30% of the edges removed, and a Barabasi-Albert-like graph
  for (int kind = 0; kind < 2; ++kind) {
    const int side = 40;
    const int64_t n = kind == 0 ? side * side : 1500;
    std::vector<std::vector<int32_t>> adj(n);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    auto add = [&](int64_t a, int64_t b) {
      if (a == b) return;
      for (int32_t x : adj[a])
        if (x == b) return;
      adj[a].push_back((int32_t)b);
      adj[b].push_back((int32_t)a);
    };
    if (kind == 0) {
      for (int r = 0; r < side; ++r)
        for (int c = 0; c < side; ++c) {
          if (c + 1 < side && u(rng) < 0.7) add(r * side + c, r * side + c + 1);
          if (r + 1 < side && u(rng) < 0.7) add(r * side + c, (r + 1) * side + c);
        }
    } else {
      std::vector<int64_t> ends;
      for (int64_t v = 1; v < 4; ++v) add(v, 0), ends.push_back(v), ends.push_back(0);
      for (int64_t v = 4; v < n; ++v)
        for (int e = 0; e < 3; ++e) {
          const int64_t t = ends[std::uniform_int_distribution<size_t>(0, ends.size() - 1)(rng)];
          add(v, t);
          ends.push_back(v);
          ends.push_back(t);
        }
    }
    std::vector<int32_t> rp(n + 1, 0), ci;
    for (int64_t i = 0; i < n; ++i) {
      std::sort(adj[i].begin(), adj[i].end());
      rp[i + 1] = rp[i] + (int32_t)adj[i].size();
      ci.insert(ci.end(), adj[i].begin(), adj[i].end());
    }
    for (double frac : {0.01, 0.5, 0.99}) {
      // alpha from a cheap bound: rho(Z_1) <= max degree
      int32_t dmax = 1;
      for (int64_t i = 0; i < n; ++i) dmax = std::max(dmax, rp[i + 1] - rp[i]);
      // the lattice's rho(Z_1) is below its largest degree; the preferential-attachment
      // graph's is far below (about 0.2 times the inverse of alpha here)
      const double alpha = kind == 0 ? frac / dmax : 0.2 * frac;
      HostCSR A;
      amg_deformed_matrix(n, rp.data(), ci.data(), 1.0, alpha, A);
      AmgParams prm;
      prm.coarse_size = 50;
      std::vector<AmgHostLevel> levels;
      std::vector<int64_t> agg;
      const int st = amg_build(A, prm, levels, &agg);
      bool ok = st == (int)levels.size() && !levels.empty() && levels[0].A.n == n;
      for (size_t l = 0; ok && l + 1 < levels.size(); ++l) {
        const HostCSR& P = levels[l].P;
        const HostCSR& R = levels[l].R;
        ok = P.n == levels[l].A.n && P.m == levels[l + 1].A.n && R.n == P.m && R.m == P.n &&
             levels[l + 1].A.n < levels[l].A.n && (int64_t)P.rp.size() == P.n + 1;
        for (int64_t e = 0; ok && e < P.rp.back(); ++e) ok = P.ci[e] >= 0 && P.ci[e] < P.m;
      }
      char what[96];
      std::snprintf(what, sizeof(what), "amg_build %s n=%lld alpha=%.4f (%zu levels)",
                    kind == 0 ? "lattice" : "ba", (long long)n, alpha, levels.size());
      expect(ok, what, (double)levels.size());
    }
  }
}

}  // namespace

// The library's error hook (defined in the device part of the library).
void wl_set_error(const char*, ...) {}

int main() {
  std::mt19937_64 rng(20260111);
  check_dense(rng);
  check_sym_eig(rng);
  check_block_tridiag(rng);
  check_chol_deflate(rng);
  check_phi1(rng);
  check_aaa();
  check_amg(rng);
  std::printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}
