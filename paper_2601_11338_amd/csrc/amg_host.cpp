// Aggregation multigrid hierarchy for the deformed Laplacian, built on the host.
//
// Sec. 4.2 preconditions CG on A_mu(alpha) (eq. deformed, an M-matrix) with an
// aggregation AMG: Vanek-Mandel-Brezina aggregation, a V-cycle with one l1-Jacobi sweep
// before and after the coarse correction, 30 sweeps as the coarsest solver.  The setup is
// sequential graph work on a few sparse matrices (aggregation, two sparse products per
// level), done once per operator on the host; the device applies the hierarchy.
//
// Per level:
//   * strong couplings: j != i with |a_ij| >= theta sqrt(a_ii a_jj);
//   * aggregation over the nodes with a strong neighbour (others get no coarse unknown):
//     1. in node order, a node whose strong neighbourhood holds no aggregated node roots
//        an aggregate made of that neighbourhood;
//     2. every node still free joins the step-1 aggregate of its most strongly coupled
//        step-1-aggregated neighbour (largest |a_ij|, ties to the lower column);
//     3. in node order, a node still free forms an aggregate with its free neighbours;
//   * tentative prolongator: piecewise constant, columns of unit norm;
//   * smoothed prolongator P = (I - omega D^-1 A) P_t, omega = 4 / (3 ||D^-1 A||_inf);
//   * Galerkin coarse matrix P^T A P;
//   * levels are added while the coarse size is below 0.9 of the fine one and the fine
//     level is larger than coarse_size.
// Entries that sum to exactly zero are not stored.  Rows are sorted by column.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "wl_amg.h"

namespace {

// Y = A B for CSR A (na x k) and CSR B (k x m), rows accumulated in column order.
void spgemm(const HostCSR& A, const HostCSR& B, int64_t m, HostCSR& C) {
  C.n = A.n;
  C.m = m;
  C.rp.assign(A.n + 1, 0);
  C.ci.clear();
  C.v.clear();
  std::vector<double> acc(m, 0.0);
  std::vector<char> used(m, 0);
  std::vector<int32_t> cols;
  for (int64_t i = 0; i < A.n; ++i) {
    cols.clear();
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int32_t k = A.ci[e];
      const double a = A.v[e];
      for (int64_t f = B.rp[k]; f < B.rp[k + 1]; ++f) {
        const int32_t j = B.ci[f];
        if (!used[j]) {
          used[j] = 1;
          cols.push_back(j);
        }
        acc[j] += a * B.v[f];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols) {
      if (acc[j] != 0.0) {
        C.ci.push_back(j);
        C.v.push_back(acc[j]);
      }
      acc[j] = 0.0;
      used[j] = 0;
    }
    C.rp[i + 1] = (int64_t)C.ci.size();
  }
}

void transpose(const HostCSR& A, HostCSR& T) {
  T.n = A.m;
  T.m = A.n;
  T.rp.assign(T.n + 1, 0);
  for (int32_t j : A.ci) ++T.rp[j + 1];
  for (int64_t j = 0; j < T.n; ++j) T.rp[j + 1] += T.rp[j];
  T.ci.resize(A.ci.size());
  T.v.resize(A.v.size());
  std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int64_t i = 0; i < A.n; ++i)  // rows in order: every column of T comes out sorted
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int64_t p = pos[A.ci[e]]++;
      T.ci[p] = (int32_t)i;
      T.v[p] = A.v[e];
    }
}

std::vector<double> diagonal(const HostCSR& A) {
  std::vector<double> d(A.n, 0.0);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e)
      if (A.ci[e] == i) d[i] = A.v[e];
  return d;
}

}  // namespace

std::vector<double> amg_l1_diagonal(const HostCSR& A) {
  std::vector<double> m(A.n, 0.0);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) m[i] += std::fabs(A.v[e]);
  return m;
}

int64_t amg_aggregate(const HostCSR& A, double theta, std::vector<int64_t>& agg) {
  const int64_t n = A.n;
  const std::vector<double> d = diagonal(A);
  // strong neighbours of every row (CSR of the strength graph, sorted columns)
  std::vector<int64_t> srp(n + 1, 0);
  std::vector<int32_t> sci;
  std::vector<double> sv;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int32_t j = A.ci[e];
      if (j == i) continue;
      if (std::fabs(A.v[e]) >= theta * std::sqrt(std::fabs(d[i] * d[j]))) {
        sci.push_back(j);
        sv.push_back(std::fabs(A.v[e]));
      }
    }
    srp[i + 1] = (int64_t)sci.size();
  }
  agg.assign(n, -1);
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i) {  // 1: roots with wholly free neighbourhoods
    if (srp[i] == srp[i + 1] || agg[i] >= 0) continue;
    bool free = true;
    for (int64_t e = srp[i]; e < srp[i + 1] && free; ++e) free = agg[sci[e]] < 0;
    if (!free) continue;
    agg[i] = k;
    for (int64_t e = srp[i]; e < srp[i + 1]; ++e) agg[sci[e]] = k;
    ++k;
  }
  const std::vector<int64_t> first(agg);
  for (int64_t i = 0; i < n; ++i) {  // 2: the most strongly coupled step-1 aggregate
    if (srp[i] == srp[i + 1] || agg[i] >= 0) continue;
    int64_t best = -1;
    double bv = -1.0;
    for (int64_t e = srp[i]; e < srp[i + 1]; ++e)
      if (first[sci[e]] >= 0 && sv[e] > bv) {
        best = sci[e];
        bv = sv[e];
      }
    if (best >= 0) agg[i] = first[best];
  }
  for (int64_t i = 0; i < n; ++i) {  // 3: leftovers with their free strong neighbours
    if (srp[i] == srp[i + 1] || agg[i] >= 0) continue;
    agg[i] = k;
    for (int64_t e = srp[i]; e < srp[i + 1]; ++e)
      if (agg[sci[e]] < 0) agg[sci[e]] = k;
    ++k;
  }
  return k;
}

void amg_deformed_matrix(int64_t n, const int32_t* rowptr, const int32_t* colidx, double mu, double alpha,
                         HostCSR& A) {
  // A_mu(alpha) = (1 - mu^2 alpha^2) I - alpha A + alpha^2 mu D, diagonal stored in place
  const double c0 = 1.0 - mu * mu * alpha * alpha;
  A.n = A.m = n;
  A.rp.assign(n + 1, 0);
  A.ci.clear();
  A.v.clear();
  A.ci.reserve((size_t)rowptr[n] + n);
  A.v.reserve((size_t)rowptr[n] + n);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t s = rowptr[i], e = rowptr[i + 1];
    bool diag_done = false;
    for (int32_t k = s; k <= e; ++k) {
      if (!diag_done && (k == e || colidx[k] > i)) {
        A.ci.push_back((int32_t)i);
        A.v.push_back(c0 + alpha * alpha * mu * (double)(e - s));
        diag_done = true;
      }
      if (k < e) {
        A.ci.push_back(colidx[k]);
        A.v.push_back(-alpha);
      }
    }
    A.rp[i + 1] = (int64_t)A.ci.size();
  }
}

int amg_build(const HostCSR& A0, const AmgParams& prm, std::vector<AmgHostLevel>& levels, std::vector<int64_t>* agg0) {
  levels.clear();
  levels.emplace_back();
  levels[0].A = A0;
  for (;;) {
    AmgHostLevel& L = levels.back();
    L.m = amg_l1_diagonal(L.A);
    const int64_t n = L.A.n;
    if (n <= prm.coarse_size || (int)levels.size() >= prm.max_levels) break;
    std::vector<int64_t> agg;
    const int64_t nagg = amg_aggregate(L.A, prm.theta, agg);
    if (levels.size() == 1 && agg0) *agg0 = agg;
    if (nagg == 0 || (double)nagg > 0.9 * (double)n) break;
    // tentative prolongator (unit-norm piecewise constants)
    std::vector<double> size(nagg, 0.0);
    for (int64_t i = 0; i < n; ++i)
      if (agg[i] >= 0) size[agg[i]] += 1.0;
    HostCSR Pt;
    Pt.n = n;
    Pt.m = nagg;
    Pt.rp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      if (agg[i] >= 0) {
        Pt.ci.push_back((int32_t)agg[i]);
        Pt.v.push_back(1.0 / std::sqrt(size[agg[i]]));
      }
      Pt.rp[i + 1] = (int64_t)Pt.ci.size();
    }
    // P = Pt - omega D^-1 (A Pt)
    const std::vector<double> d = diagonal(L.A);
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t e = L.A.rp[i]; e < L.A.rp[i + 1]; ++e) s += std::fabs(L.A.v[e]);
      nrm = std::max(nrm, s / d[i]);
    }
    const double omega = 4.0 / (3.0 * nrm);
    HostCSR APt;
    spgemm(L.A, Pt, nagg, APt);
    HostCSR& P = L.P;
    P.n = n;
    P.m = nagg;
    P.rp.assign(n + 1, 0);
    P.ci.clear();
    P.v.clear();
    for (int64_t i = 0; i < n; ++i) {
      // merge row i of Pt (at most one entry) with row i of -omega D^-1 A Pt
      const bool has = Pt.rp[i + 1] > Pt.rp[i];
      const int32_t pc = has ? Pt.ci[Pt.rp[i]] : -1;
      const double pv = has ? Pt.v[Pt.rp[i]] : 0.0;
      bool done = !has;
      for (int64_t e = APt.rp[i]; e <= APt.rp[i + 1]; ++e) {
        const bool end = e == APt.rp[i + 1];
        const int32_t c = end ? -1 : APt.ci[e];
        if (!done && (end || c >= pc)) {
          double v = pv;
          if (!end && c == pc) v -= (omega / d[i]) * APt.v[e];
          if (v != 0.0) {
            P.ci.push_back(pc);
            P.v.push_back(v);
          }
          done = true;
          if (!end && c == pc) continue;
        }
        if (end) break;
        const double v = 0.0 - (omega / d[i]) * APt.v[e];
        if (v != 0.0) {
          P.ci.push_back(c);
          P.v.push_back(v);
        }
      }
      P.rp[i + 1] = (int64_t)P.ci.size();
    }
    transpose(P, L.R);
    HostCSR AP, Ac;
    spgemm(L.A, P, nagg, AP);
    spgemm(L.R, AP, nagg, Ac);
    levels.emplace_back();
    levels.back().A = std::move(Ac);
  }
  return (int)levels.size();
}
