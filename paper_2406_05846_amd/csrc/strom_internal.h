// strom_internal.h -- data shared by the host setup, the C ABI layer and the HIP kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/strom.h"

namespace strom {

// Task types of the triangular solves.
enum : int32_t { kTaskLevels = 0, kTaskDense = 1 };

// Host result of the one-time analysis of an SDP instance.
struct HostAnalysis {
  int32_t m = 0;
  int64_t nsvec = 0;
  int32_t nblocks = 0;
  std::vector<int32_t> bsize;
  std::vector<int64_t> boff;
  // A^T in CSR (row c = svec column c of A): for A^* y.
  std::vector<int64_t> Atrp;
  std::vector<int32_t> Atci;
  std::vector<double> Atv;
  // Row ordering: perm[new] = old, pinv[old] = new.
  std::vector<int32_t> perm, pinv;
  // eps*I + A A^* (permuted) = L D L^T, L unit lower triangular.
  double eps = 0.0;
  std::vector<int64_t> Lrp;   // CSR of strict lower L (rows in new order, columns ascending)
  std::vector<int32_t> Lci;
  std::vector<double> Lv;
  std::vector<int64_t> Urp;   // CSR of L^T (row j lists i > j), columns ascending
  std::vector<int32_t> Uci;
  std::vector<double> Uv;
  std::vector<double> D;
  // Solve tasks: contiguous row ranges of the new order.
  std::vector<int32_t> task_r0, task_r1, task_type;
  std::vector<int32_t> task_flev0, task_fnlev, task_blev0, task_bnlev;  // level tasks
  std::vector<int64_t> task_inv;                                        // dense tasks
  std::vector<int32_t> flevptr, frows, blevptr, brows;                  // level lists (absolute rows)
  std::vector<double> inv;   // dense inverses of diagonal blocks, column-major
  std::vector<double> invT;  // same, transposed (row-major), for the backward GEMV
  // Launch schedule: task ids grouped by dependency depth.
  std::vector<int32_t> fwd_order, fwd_gptr, bwd_order, bwd_gptr;
  int32_t max_task_rows = 0;
  int32_t max_dense_rows = 0;
  int64_t nnzL = 0;
};

// Validates the CSR, orders, factors and analyses.  Returns STROM_OK or an error with `err`.
strom_status analyze_instance(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
                              const int32_t *col, const double *val, double eps_reg, HostAnalysis &H,
                              std::string &err);

}  // namespace strom
