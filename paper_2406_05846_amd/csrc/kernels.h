// kernels.h -- device-side types and host launchers of the sGS-ADMM kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "strom_internal.h"

namespace strom {
namespace dev {

// Per-instance scalars that live in device memory, so that the iteration can be enqueued
// without host round trips.
struct DevState {
  double sigma;       // current sigma
  double tau;
  double eta_p, eta_d, eta_g, pobj, dobj;
  double sigma_used;  // sigma of the iteration the residuals belong to
};

// Pointer policies of the argument structs below: plain pointers (host side and kernel
// arguments), or pointers typed as global memory -- the device's view of a struct that merged
// launches read from a table in device memory.  The compiler takes a plain pointer loaded
// from memory as generic and accesses through it with flat instructions; the global view keeps
// global ones.  G(p) gives the plain pointer (an explicit cast for a global one).
template <class T>
using HostPtr = T *;
template <class T>
using GlobPtr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ T *G(T *p) {
  return p;
}
template <class T>
__device__ __forceinline__ T *G(__attribute__((address_space(1))) T *p) {
  return (T *)p;
}

// Device arrays of the triangular solves (see setup.cpp for their meaning).
template <template <class> class Ptr>
struct SolveArgsT {
  Ptr<const int32_t> task_r0, task_r1, task_ph0, task_ph1;
  Ptr<const int32_t> ph_a, ph_nns;  // first row and rows in components of 2+ of every phase
  Ptr<const double> D;
  Ptr<const int32_t> perm;
  // pushes: task t sums its push stream (kind 4) into part[tseg[tsptr[t] + r]], row r
  Ptr<const int32_t> tsptr, tseg;
  Ptr<double> part;
  // streams, kinds 0 forward gather, 1 forward inverse, 2 backward gather, 3 backward inverse
  // (per phase), 4 push (per task): values, indices, per-phase (task) offset, entries per
  // thread, thread stride, first rows of the slices
  Ptr<const double> sval[kStreamKinds];
  Ptr<const int32_t> sidx[kStreamKinds];
  Ptr<const int64_t> s_off[kStreamKinds];
  Ptr<const int32_t> s_K[kStreamKinds];
  Ptr<const int32_t> s_T[kStreamKinds];
  Ptr<const int32_t> s_ra[kStreamKinds];
  // task-local staging (task_inl[t] != 0): the task's rows, then its incoming partial sums
  // part[task_pin[t] ..] (forward) or the later-task rows task_xrow[task_xoff[t] ..]
  // (backward) are staged in LDS and the fg / bg stream indices address that buffer
  Ptr<const int32_t> task_pin, task_inl;
  Ptr<const int64_t> task_xoff;
  Ptr<const int32_t> task_xrow;
  int32_t lds_rows;  // LDS doubles for a staged task (at least every staged task's total)
  int32_t c_cap;     // LDS doubles for the right-hand sides of a phase's components
};
using SolveArgs = SolveArgsT<HostPtr>;
using SolveArgsG = SolveArgsT<GlobPtr>;

// One instance of a merged (batched) launch: what the kernels read of it, and its flags, which
// the host rewrites between rounds (a captured round stays valid for any flags).
template <template <class> class Ptr>
struct BatchInstT {
  int32_t m, nrow_chunks;  // rows of A, and 256-row chunks
  int64_t n;               // svec length
  int32_t ncol_chunks;     // 256-column chunks
  int32_t active;          // 0: retired, every merged launch skips the instance
  int32_t f32;             // projection precision: 1 FP32, 0 FP64
  int32_t warm;            // Q holds eigenvectors to start from
  int32_t sig;             // the sigma rule applies at the end of this round
  Ptr<const int64_t> A_rp, At_rp, boff, qoff;
  Ptr<const int32_t> A_ci, At_ci, pinv, bsz;
  Ptr<const double> A_v, At_v, b, C;
  Ptr<double> X, S, Xb, y, w, part_rows, part_cols, part_cone, Q;
  Ptr<DevState> st;
  double normb, normC;
};
using BatchInst = BatchInstT<HostPtr>;
using BatchInstG = BatchInstT<GlobPtr>;
// The host fills these tables and the device reads them through the global view: both
// compilations must see one layout.
static_assert(sizeof(SolveArgs) == 368 && sizeof(SolveArgsG) == sizeof(SolveArgs), "SolveArgs layout");
static_assert(sizeof(BatchInst) == 232 && sizeof(BatchInstG) == sizeof(BatchInst) &&
                  offsetof(BatchInst, st) == 208 && offsetof(BatchInstG, st) == 208,
              "BatchInst layout");

// A work item of a merged launch: the instance and its local index (row or column chunk, solve
// task, or PSD block).
struct BatchItem {
  int32_t inst, idx;
};

struct SolveSchedule {
  std::vector<int32_t> fwd_gptr, bwd_gptr;    // host: group boundaries
  std::vector<int32_t> fwd_order, bwd_order;  // host: tasks of the groups in launch order
  std::vector<int32_t> fwd_cost, bwd_cost;    // host: stream entries per thread of each task
  const int32_t *fwd_order_dev = nullptr, *bwd_order_dev = nullptr;
};

size_t project_lds_bytes(int n, bool f32, int nthreads);
int project_threads(int n);

hipError_t launch_rhs(hipStream_t s, int32_t m, const int64_t *rp, const int32_t *ci, const double *av,
                      const double *X, const double *S, const double *C, const double *b, const int32_t *pinv,
                      const DevState *st, double *w);
hipError_t launch_solve(hipStream_t s, const SolveSchedule &sch, const SolveArgs &a, double *w, double *y);
hipError_t launch_xb(hipStream_t s, int64_t n, const int64_t *trp, const int32_t *tci, const double *tv,
                     const double *y, const double *X, const double *C, const DevState *st, double *Xb);
// S = (Pi(X_b) - X_b) * scale for the listed blocks; scale <= 0 means 1 / sigma.  Q (nullable)
// holds the eigenvectors of each block at qoff[k]; warm starts from them, and they are
// overwritten with the new ones, re-orthogonalized (one Newton-Schulz step) when reorth.
hipError_t launch_project_admm(hipStream_t s, bool f32, int n, int count, const int32_t *ids, const int64_t *boff,
                               const int32_t *bsz, const double *Xb, double *S, const DevState *st, double scale,
                               double *Q, const int64_t *qoff, bool warm, bool reorth);
// Eigenvalues (ascending, at w + woff[k]) and, with v != nullptr, eigenvectors (columns of an
// n x n block at v + od[k]) of dense column-major blocks; err as for launch_project_dense.
hipError_t launch_eig_dense(hipStream_t s, bool f32, int nblocks, int max_n, const int32_t *nd, const int64_t *od,
                            const void *in, const int64_t *woff, void *w, void *v, int32_t *err);
// Dense n x n column-major double copies of the svec blocks ids[k] (at out + od[k]).
hipError_t launch_unpack_svec(hipStream_t s, int count, const int32_t *ids, const int64_t *boff, const int32_t *bsz,
                              const double *sv, const int64_t *od, double *out);
// Z = C - A^* y (svec), A^* through the CSR of A^T.
hipError_t launch_slack(hipStream_t s, int64_t n, const int64_t *trp, const int32_t *tci, const double *tv,
                        const double *y, const double *C, double *Z);
hipError_t launch_project_dense(hipStream_t s, bool f32, int nblocks, int max_n, const int32_t *nd, const int64_t *od,
                                const void *in, void *out, int32_t *err);
hipError_t launch_xupdate(hipStream_t s, int64_t n, const int64_t *trp, const int32_t *tci, const double *tv,
                          const double *y, const double *S, const double *C, const DevState *st, double *X,
                          double *part, int update);
// Residuals of the termination rule; with do_sigma also the sigma rule, which needs
// cone_diff = Pi(X) - X (svec) for the cone distance of X.
hipError_t launch_kkt(hipStream_t s, int32_t m, int64_t n, const int64_t *rp, const int32_t *ci, const double *av,
                      const double *X, const double *b, const double *y, double *part_rows, const double *part_cols,
                      const double *cone_diff, double *part_cone, double normb, double normC, int do_sigma,
                      DevState *st);

// Merged launches over the instances of a batch (items: one workgroup each; retired
// instances are skipped).  The solve's groups are merged by dependency depth: group g of every
// instance in one launch, lds_bytes at least every instance's need.
// r_s of every running instance: a column pass forms X/sigma + S - C in the X_b buffer, a row
// pass gathers it.
hipError_t launch_rhs_batch(hipStream_t s, int nrows, const BatchItem *rows, int ncols, const BatchItem *cols,
                            const BatchInst *bi);
hipError_t launch_solve_batch(hipStream_t s, const std::vector<int32_t> &fwd_gptr, const BatchItem *fwd,
                              const std::vector<int32_t> &bwd_gptr, const BatchItem *bwd, const SolveArgs *args,
                              const BatchInst *bi, size_t lds_bytes);
hipError_t launch_xb_batch(hipStream_t s, int count, const BatchItem *cols, const BatchInst *bi);
hipError_t launch_xupdate_batch(hipStream_t s, int count, const BatchItem *cols, const BatchInst *bi, int want_part);
// Residuals of every running instance; with do_sigma, the sigma rule too for the instances whose
// sig flag is set.
hipError_t launch_kkt_batch(hipStream_t s, int nrows, const BatchItem *rows, int ncols, const BatchItem *cols,
                            int ninst, const BatchInst *bi, int do_sigma);
// Copies every instance's DevState to out[0 .. ninst).
hipError_t launch_gather_states(hipStream_t s, int ninst, const BatchInst *bi, DevState *out);
// PSD projection of blocks of one size n over a batch, nt threads per workgroup; only the
// instances whose precision flag matches f32 are projected.  cone = 0: S = (Pi(X_b) - X_b) /
// sigma (step 2); cone = 1: X_b = Pi(X) - X (the sigma rule's cone distance), only for the
// instances whose sig flag is set.
hipError_t launch_project_batch(hipStream_t s, bool f32, int n, int nt, int count, const BatchItem *items,
                                const BatchInst *bi, int cone, bool reorth);
// Whether the one-workgroup projection takes blocks of size n (its LDS within lds_cap and a
// worker thread for every 2 x 2 block and eigenvector row): n <= 113 in FP64, <= 122 in FP32.
bool project_fits(int n, bool f32, size_t lds_cap);
// Thread counts the projection kernel accepts for blocks of size n (at most 5, ascending).
int project_thread_options(int n, bool f32, int *out);

// Blocks too large for one workgroup's LDS (big.hip): count blocks padded to np (a multiple of
// 64, at most kBigMaxN).  Block k is block ids[k] of an svec vector (boff, bsz) or, with ids ==
// nullptr, the dense column-major block k (nd[k], od[k]).  work: big_work_doubles(np, count)
// doubles of device memory; err (nullable) is or-ed with 1 when a block size is <= 0 or > np.
constexpr int kBigMaxN = 512;
struct BigArgs {
  int32_t np = 0, count = 0;
  const int32_t *ids = nullptr;
  const int64_t *boff = nullptr;
  const int32_t *bsz = nullptr;
  const int32_t *nd = nullptr;
  const int64_t *od = nullptr;
  double *work = nullptr;
  int32_t *err = nullptr;
};
size_t big_work_doubles(int np, int count);
int big_padded(int n);
// ADMM step 2 for the listed svec blocks, as launch_project_admm (always FP64).
hipError_t launch_project_big_admm(hipStream_t s, const BigArgs &a, const double *X, double *S, const DevState *st,
                                   double scale, double *Q, const int64_t *qoff, bool warm, bool reorth);
// out = Pi(in) for dense column-major FP64 blocks (out may alias in).
hipError_t launch_project_big_dense(hipStream_t s, const BigArgs &a, const double *in, double *out);
// Eigenvalues ascending at w + woff[k]; with v, eigenvectors as the columns of the block at v + od[k].
hipError_t launch_eig_big_dense(hipStream_t s, const BigArgs &a, const double *in, const int64_t *woff, double *w,
                                double *v);

}  // namespace dev
}  // namespace strom
