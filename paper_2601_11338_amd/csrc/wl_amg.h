// Aggregation multigrid for the deformed Laplacian: host setup and device hierarchy.
// Internal to the library.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "wl_internal.h"

// Compressed sparse rows with values (n rows, m columns).
struct HostCSR {
  int64_t n = 0, m = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

struct AmgParams {
  double theta = 0.01;      // strength of connection
  int64_t coarse_size = 256;  // a level this small is the coarsest
  int max_levels = 20;
  int coarse_sweeps = 30;   // l1-Jacobi sweeps of the coarsest-level solver
};

struct AmgHostLevel {
  HostCSR A;              // level matrix (diagonal stored)
  HostCSR P, R;           // prolongator from the next level and its transpose (empty on the last)
  std::vector<double> m;  // l1 diagonal, sum_j |a_ij|
};

// A_mu(alpha) of a CSR graph as an explicit matrix (diagonal stored in column order).
void amg_deformed_matrix(int64_t n, const int32_t* rowptr, const int32_t* colidx, double mu, double alpha,
                         HostCSR& A);
// Aggregate of every row (-1: no strong neighbour); returns the number of aggregates.
int64_t amg_aggregate(const HostCSR& A, double theta, std::vector<int64_t>& agg);
std::vector<double> amg_l1_diagonal(const HostCSR& A);
// Levels from A0; agg0 (optional) receives the aggregates of the finest level.
int amg_build(const HostCSR& A0, const AmgParams& prm, std::vector<AmgHostLevel>& levels,
              std::vector<int64_t>* agg0);

// Device copy of one level (FP64 values, int32 columns and row pointers).
struct AmgDevLevel {
  int64_t n = 0, nnz = 0, pnnz = 0;
  DevBuf rp, ci, v;    // level matrix (unused on level 0, applied implicitly from the graph)
  DevBuf prp, pci, pv;  // P
  DevBuf rrp, rci, rv;  // R = P^T
  DevBuf jw;           // 1 / (l1 diagonal)
  DevBuf b, x, r, y;   // n x b work blocks
  int64_t nb = 0;      // block width the work blocks were sized for
};

struct AmgState {
  AmgParams prm;
  double c0 = 1.0, alpha = 0.0, am = 0.0;  // A_mu(alpha) = c0 I - alpha A + am D
  std::vector<std::unique_ptr<AmgDevLevel>> lv;
  double setup_ms = 0.0;
  // CG work blocks (n x b) and per-column scalars
  DevBuf x, r, z, p, q, scal, partials;
  int64_t nb = 0;
  int last_iters = 0;           // iterations of the last solve (largest over columns)
  double last_relres = 0.0;     // largest relative residual at its end
  double products = 0.0;        // sum over sparse products of nnz x columns (work tally)
};

wl_status amg_setup(wl_op* op);
void amg_destroy(wl_op* op);
template <typename T>
wl_status phi_amg(wl_op* op, const T* X, T* Y, int b, const T* wv, const T* Xw);
