// AAA rational approximation on real data, and the poles of the approximant (host, FP64).
//
// AAA (Nakatsukasa, Sete and Trefethen, SIAM J. Sci. Comput. 40, 2018), the pole
// construction Alg. 1 cites: support points are chosen greedily where the current
// barycentric approximant r(x) = sum_j w_j f_j / (x - z_j) / sum_j w_j / (x - z_j) errs
// most; the weights w are the right singular vector of the smallest singular value of
// the Loewner matrix (F_i - f_k) / (Z_i - z_k) over the points not yet chosen.  With
// real points and values the Loewner matrix is real; its smallest singular pair comes
// from a one-sided Jacobi SVD (accurate for the small singular values AAA needs) of
// the triangular factor of its Householder QR.
// The poles are the zeros of the denominator sum_j w_j / (x - z_j), i.e. of the
// polynomial sum_j w_j prod_{i != j} (x - z_i), found by the Aberth-Ehrlich
// simultaneous iteration on that product form.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "wl_internal.h"

namespace {

// Right singular vector of the smallest singular value of the rows x m matrix A
// (column-major, leading dimension rows) by one-sided Jacobi: columns are rotated
// pairwise until mutually orthogonal; V accumulates the rotations.
void jacobi_min_right_vector(int64_t rows, int m, std::vector<double>& A, std::vector<double>& v) {
  std::vector<double> V((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  const double eps = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        double* ap = &A[(size_t)p * rows];
        double* aq = &A[(size_t)q * rows];
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int64_t i = 0; i < rows; ++i) {
          al += ap[i] * ap[i];
          be += aq[i] * aq[i];
          ga += ap[i] * aq[i];
        }
        if (std::fabs(ga) <= eps * std::sqrt(al * be) || ga == 0.0) continue;
        rotated = true;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int64_t i = 0; i < rows; ++i) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        for (int i = 0; i < m; ++i) {
          double* vp = &V[(size_t)p * m + i];
          double* vq = &V[(size_t)q * m + i];
          const double x = *vp, y = *vq;
          *vp = c * x - s * y;
          *vq = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
  int kmin = 0;
  double smin = INFINITY;
  for (int k = 0; k < m; ++k) {
    double s = 0.0;
    for (int64_t i = 0; i < rows; ++i) s += A[(size_t)k * rows + i] * A[(size_t)k * rows + i];
    if (s < smin) {
      smin = s;
      kmin = k;
    }
  }
  v.assign(V.begin() + (size_t)kmin * m, V.begin() + (size_t)(kmin + 1) * m);
}

// R (m x m, column-major) of a Householder QR of the rows x m column-major A: A and R
// share their right singular vectors, and the Jacobi sweeps then run on m rows only.
void householder_r(int64_t rows, int m, std::vector<double>& A, std::vector<double>& R) {
  std::vector<double> v(rows);
  for (int k = 0; k < m && k < rows; ++k) {
    double* a = &A[(size_t)k * rows];
    double nx = 0.0;
    for (int64_t i = k; i < rows; ++i) nx += a[i] * a[i];
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const double alpha = a[k] >= 0 ? -nx : nx;
    for (int64_t i = k; i < rows; ++i) v[i] = a[i];
    v[k] -= alpha;
    double vv = 0.0;
    for (int64_t i = k; i < rows; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int c = k; c < m; ++c) {
      double* col = &A[(size_t)c * rows];
      double s = 0.0;
      for (int64_t i = k; i < rows; ++i) s += v[i] * col[i];
      s = 2.0 * s / vv;
      for (int64_t i = k; i < rows; ++i) col[i] -= s * v[i];
    }
  }
  R.assign((size_t)m * m, 0.0);
  for (int c = 0; c < m; ++c)
    for (int r = 0; r <= c && r < rows; ++r) R[(size_t)c * m + r] = A[(size_t)c * rows + r];
}

}  // namespace

int aaa_real(int64_t N, const double* Z, const double* F, double tol, int mmax, std::vector<double>& z,
             std::vector<double>& f, std::vector<double>& w, double* max_err) {
  z.clear();
  f.clear();
  w.clear();
  if (N < 2 || mmax < 1) return -1;
  std::vector<char> free_pt(N, 1);
  std::vector<double> R(N);
  double mean = 0.0, scale = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    mean += F[i];
    scale = std::max(scale, std::fabs(F[i]));
  }
  mean /= N;
  std::fill(R.begin(), R.end(), mean);
  double err = INFINITY;
  std::vector<int64_t> rows;
  std::vector<double> A, v;
  for (int m = 1; m <= mmax && m < N; ++m) {
    int64_t j = -1;
    double best = -1.0;
    for (int64_t i = 0; i < N; ++i)
      if (free_pt[i] && std::fabs(F[i] - R[i]) > best) {
        best = std::fabs(F[i] - R[i]);
        j = i;
      }
    z.push_back(Z[j]);
    f.push_back(F[j]);
    free_pt[j] = 0;
    rows.clear();
    for (int64_t i = 0; i < N; ++i)
      if (free_pt[i]) rows.push_back(i);
    const int64_t nr = (int64_t)rows.size();
    A.assign((size_t)nr * m, 0.0);
    for (int k = 0; k < m; ++k)
      for (int64_t r = 0; r < nr; ++r) {
        const int64_t i = rows[r];
        A[(size_t)k * nr + r] = (F[i] - f[k]) / (Z[i] - z[k]);
      }
    if (nr > 2 * m) {
      std::vector<double> Rm;
      householder_r(nr, m, A, Rm);
      jacobi_min_right_vector(m, m, Rm, v);
    } else {
      jacobi_min_right_vector(nr, m, A, v);
    }
    w = v;
    err = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      if (!free_pt[i]) {
        R[i] = F[i];
        continue;
      }
      double num = 0.0, den = 0.0;
      for (int k = 0; k < m; ++k) {
        const double c = w[k] / (Z[i] - z[k]);
        num += c * f[k];
        den += c;
      }
      R[i] = num / den;
      err = std::max(err, std::fabs(F[i] - R[i]));
    }
    if (err <= tol * scale) break;
  }
  if (max_err) *max_err = err;
  return 0;
}

int aaa_poles(const std::vector<double>& z, const std::vector<double>& w, std::vector<std::complex<double>>& poles) {
  using cd = std::complex<double>;
  poles.clear();
  const int m = (int)z.size();
  if (m < 2) return 0;
  double wsum = 0.0, wabs = 0.0, zlo = z[0], zhi = z[0];
  for (int j = 0; j < m; ++j) {
    wsum += w[j];
    wabs += std::fabs(w[j]);
    zlo = std::min(zlo, z[j]);
    zhi = std::max(zhi, z[j]);
  }
  // degree of p(x) = sum_j w_j prod_{i != j} (x - z_i): m - 1 unless the leading
  // coefficient sum_j w_j vanishes (then a pole has gone to infinity)
  const int deg = std::fabs(wsum) <= 1e-14 * wabs ? m - 2 : m - 1;
  if (deg <= 0) return 0;
  // work in x' = (x - ctr) / rad so that every factor is O(1); p is evaluated in this
  // product form (no singularity at the support points, unlike the barycentric ratio)
  const double ctr = 0.5 * (zlo + zhi), rad = std::max(0.5 * (zhi - zlo), 1e-300);
  std::vector<double> zs(m);
  for (int i = 0; i < m; ++i) zs[i] = (z[i] - ctr) / rad;
  // p(x) = sum_j w_j prod_{i != j} f_i and p'(x), f_i = x - z_i, in O(m) from prefix
  // and suffix products of the f_i and their derivatives (product rule, f_i' = 1)
  std::vector<cd> pre(m + 1), pred(m + 1), suf(m + 1), sufd(m + 1);
  auto p_and_dp = [&](cd x, cd* p, cd* dp) {
    pre[0] = 1.0;
    pred[0] = 0.0;
    for (int i = 0; i < m; ++i) {
      const cd f = x - zs[i];
      pred[i + 1] = pred[i] * f + pre[i];
      pre[i + 1] = pre[i] * f;
    }
    suf[m] = 1.0;
    sufd[m] = 0.0;
    for (int i = m - 1; i >= 0; --i) {
      const cd f = x - zs[i];
      sufd[i] = sufd[i + 1] * f + suf[i + 1];
      suf[i] = suf[i + 1] * f;
    }
    cd P(0.0), D(0.0);
    for (int j = 0; j < m; ++j) {
      P += w[j] * (pre[j] * suf[j + 1]);
      D += w[j] * (pred[j] * suf[j + 1] + pre[j] * sufd[j + 1]);
    }
    *p = P;
    *dp = D;
  };
  std::vector<cd> r(deg);
  for (int k = 0; k < deg; ++k) {
    const double th = 2.0 * M_PI * (k + 0.25) / deg + 0.4;
    r[k] = 1.3 * cd(std::cos(th), std::sin(th));
  }
  // Aberth-Ehrlich: r_k -= N / (1 - N sum_{j != k} 1 / (r_k - r_j)), N = p / p';
  // stop once every correction is at the rounding level of its root
  for (int it = 0; it < 500; ++it) {
    double mx = 0.0;
    for (int k = 0; k < deg; ++k) {
      cd P, D;
      p_and_dp(r[k], &P, &D);
      if (D == cd(0.0)) continue;
      const cd nwt = P / D;
      cd s(0.0);
      for (int j = 0; j < deg; ++j)
        if (j != k) s += 1.0 / (r[k] - r[j]);
      const cd delta = nwt / (1.0 - nwt * s);
      r[k] -= delta;
      mx = std::max(mx, std::abs(delta) / (1.0 + std::abs(r[k])));
    }
    if (mx <= 1e-15) break;
  }
  for (const cd& x : r) {
    const cd y = x * rad + ctr;
    if (std::isfinite(y.real()) && std::isfinite(y.imag())) poles.push_back(y);
  }
  return 0;
}

void exp_sample_points(double xmax, std::vector<double>& Z) {
  // equispaced points plus points graded geometrically towards 0, as one sorted set
  const int count = 1000;
  Z.clear();
  const double step = xmax / (count - 1);
  for (int i = 0; i < count; ++i) Z.push_back(i == count - 1 ? xmax : i * step);
  for (int i = 0; i < count; ++i) {
    const double e = i == count - 1 ? 0.0 : -6.0 + i * (6.0 / (count - 1));
    Z.push_back(xmax * std::pow(10.0, e));
  }
  std::sort(Z.begin(), Z.end());
  Z.erase(std::unique(Z.begin(), Z.end()), Z.end());
}

int exp_poles(double xmax, double tol, int mmax, std::vector<std::complex<double>>& poles, double* max_err) {
  std::vector<double> Z, F, z, f, w;
  exp_sample_points(xmax, Z);
  F.resize(Z.size());
  for (size_t i = 0; i < Z.size(); ++i) F[i] = std::exp(-Z[i]);
  if (aaa_real((int64_t)Z.size(), Z.data(), F.data(), tol, mmax, z, f, w, max_err)) return -1;
  std::vector<std::complex<double>> all;
  aaa_poles(z, w, all);
  poles.clear();
  for (const auto& p : all) {
    // real poles on the sampled interval are spurious pole-zero pairs and cannot be
    // shifts of a matrix whose spectrum the interval covers
    const bool on = std::fabs(p.imag()) <= 1e-8 * xmax && p.real() >= 0.0 && p.real() <= xmax;
    if (!on) poles.push_back(p);
  }
  return 0;
}
