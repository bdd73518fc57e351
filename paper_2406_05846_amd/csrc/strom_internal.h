// strom_internal.h -- data shared by the host setup, the C ABI layer and the HIP kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/strom.h"

namespace strom {

// Phase types of the triangular solves.
enum : int32_t { kPhaseLevels = 0, kPhaseDense = 1 };
constexpr int32_t kSolveThreads = 512;     // workgroup size of the solve kernels
constexpr int32_t kMaxDenseRows = 256;     // rows of one dense phase
constexpr int32_t kMaxLdsTaskRows = 14336; // task values kept in LDS up to this many rows

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
  // Solve tasks: contiguous row ranges of the new order (rows sorted by dependency level
  // inside a task).  A task is a sequence of phases over consecutive row ranges:
  //   level phase: consecutive levels [ph_l0, ph_l0 + ph_nl) of levptr, each level a row
  //                range whose rows are independent; lvl_gf / lvl_gb lanes per row;
  //   dense phase: rows [ph_a, ph_b) solved through the explicit inverse of their unit
  //                lower-triangular diagonal block (row-major at ph_inv in invR,
  //                column-major at ph_inv in invC); ph_g lanes per row for the gathers.
  std::vector<int32_t> task_r0, task_r1, task_ph0, task_ph1;
  std::vector<int32_t> ph_type, ph_a, ph_b, ph_l0, ph_nl, ph_gf, ph_gb;
  std::vector<int64_t> ph_inv;
  std::vector<int32_t> levptr, lvl_gf, lvl_gb;
  std::vector<double> invR, invC;
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
