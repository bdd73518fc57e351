// strom_internal.h -- data shared by the host setup, the C ABI layer and the HIP kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/strom.h"

namespace strom {

constexpr int32_t kSolveThreads = 1024;       // workgroup size of the solve kernels
constexpr int32_t kMaxBlockRows = 192;        // rows of one component (dense diagonal block) of a phase
constexpr int32_t kMaxPhaseBlockRows = 4096;  // rows in components of two or more, per phase
constexpr int32_t kMaxLdsTaskRows = 14336;    // task values kept in LDS up to this many rows
constexpr int32_t kStreamBatch = 8;              // granule of a stream slice (entries per thread); read two at a time
constexpr int kStreamKinds = 5;                  // fg, fi, bg, bi (per phase), push (per task)
constexpr int32_t kLastFlag = int32_t(1) << 30;  // stream index flag: last entry of a row
constexpr int32_t kPartFlag = int32_t(1) << 29;  // forward gather index flag: a pushed partial sum
constexpr int32_t kStartFlag = int32_t(1) << 30; // first-row flag of a stream slice: the row starts there

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
  // Solve tasks: contiguous row ranges of the new order.  A task is a sequence of phases
  // over consecutive row ranges [ph_a, ph_b); the rows of a phase form connected components
  // (contiguous, the first ph_nns rows in components of two or more rows, single rows last).
  // Row i belongs to component [rcs[i], rce[i]) whose inverse diagonal block starts at
  // rio[i] (-1 for a single row), packed lower triangle by rows in invR (row r at r(r+1)/2)
  // and by columns in invC (column c at c*n - c(c-1)/2).  ph_gf / ph_gb: lanes per row of
  // the forward / backward gathers.
  std::vector<int32_t> task_r0, task_r1, task_ph0, task_ph1;
  std::vector<int32_t> ph_a, ph_b, ph_nns, ph_gf, ph_gb;
  std::vector<int32_t> rcs, rce;
  std::vector<int64_t> rio;
  std::vector<double> invR, invC;
  // Forward entries of row i: [Lrp[i], Lin[i]) lie in columns of other (earlier) tasks and
  // arrive as pushed partial sums; [Lin[i], Lend[i]) are the task's own columns of earlier
  // phases, gathered by the row ([Lend[i], Lrp[i+1]) lie in the row's own component).
  // Backward entries of row j: [Ubeg[j], Urp[j+1]) (the prefix inside the component skipped).
  std::vector<int64_t> Lin, Lend, Ubeg;
  // Push segments: segment s is the run [seg_pb[s], seg_pe[s]) of one row's forward entries
  // whose columns belong to one other task; the owner task computes its partial sum right
  // after solving its rows.  Row i sums segments [sptr[i], sptr[i+1]); task t owns the
  // segments tseg[tsptr[t] .. tsptr[t+1]) and pushes them task_sg[t] lanes per segment.
  std::vector<int64_t> sptr, seg_pb, seg_pe;
  std::vector<int32_t> tsptr, tseg, task_sg;
  // The entries of every segment, copied in segment order (what the device reads for the
  // pushes): segment s is [push_off[s], push_off[s+1]) of push_ci / push_v.
  std::vector<int64_t> push_off;
  std::vector<int32_t> push_ci;
  std::vector<double> push_v;
  // Streams (kinds 0 fg, 1 fi, 2 bg, 3 bi per phase, 4 push per task; see setup.cpp): values
  // and indices, and per phase (task) the offset, the entries per thread K, the thread count
  // Tp and, for kSolveThreads + 1 threads, the first row of each slice.
  std::vector<double> sval[kStreamKinds];
  std::vector<int32_t> sidx[kStreamKinds];
  std::vector<int64_t> s_off[kStreamKinds];
  std::vector<int32_t> s_K[kStreamKinds];
  std::vector<int32_t> s_T[kStreamKinds];   // thread stride of the layout
  std::vector<int32_t> s_ra[kStreamKinds];
  // Task-local index space of a task whose values are staged in LDS (task_inl): local index
  // k < nt is row r0 + k; in the forward streams nt + q is the pushed partial sum
  // task_pin[t] + q (the task's rows sum the segments [task_pin[t], task_pin[t + 1])); in the
  // backward streams nt + q is the value of row task_xrow[task_xoff[t] + q] of a later task.
  // Other tasks index rows and partial sums (kPartFlag) globally.
  std::vector<int32_t> task_pin;
  std::vector<int64_t> task_xoff;
  std::vector<int32_t> task_xrow;
  std::vector<char> task_inl;
  int32_t max_task_stage = 0;  // max over LDS tasks of nt + max(partial sums, later-task rows)
  // Launch schedule: task ids grouped by dependency depth.
  std::vector<int32_t> fwd_order, fwd_gptr, bwd_order, bwd_gptr;
  int32_t max_task_rows = 0;
  int32_t max_phase_nns = 0;
  int64_t nnzL = 0;
};

// Validates the CSR, orders, factors and analyses.  Returns STROM_OK or an error with `err`.
// split_mode: task split of the solve schedule (0 none, 1 overweight tasks, 2 every group
// task, -1 the STROM_TASK_SPLIT environment variable if set, else 2).  block_rows: largest
// component of a phase (1..256; 0: the STROM_BLOCK_ROWS environment variable if set, else
// kMaxBlockRows).
strom_status analyze_instance(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
                              const int32_t *col, const double *val, double eps_reg, HostAnalysis &H,
                              std::string &err, int split_mode = -1, int block_rows = 0);

// A device buffer handed to an entry point instead of a per-call allocation.
struct DeviceBuf {
  unsigned char *base = nullptr;
  size_t bytes = 0;
};

// The certificate's dual bound; its temporary device memory comes from `work` (nullptr:
// allocated and freed per call).
strom_status dual_bound_impl(strom_sdp *s, const double *R_beta, double *lb, double *lam_min, const DeviceBuf *work);
int sdp_device(const strom_sdp *s);
strom_status set_error(strom_status st, const std::string &msg);
// Address of the static work buffer on `device` (current), looked up once per device.
strom_status scratch_init(int device);

}  // namespace strom
