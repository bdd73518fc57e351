// kernels.h -- device-side types and host launchers of the sGS-ADMM kernels.
#pragma once
#include <hip/hip_runtime.h>

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

// Device arrays of the triangular solves (see setup.cpp for their meaning).
struct SolveArgs {
  const int32_t *task_r0, *task_r1, *task_ph0, *task_ph1;
  const int32_t *ph_a, *ph_nns;  // first row and rows in components of 2+ of every phase
  const double *D;
  const int32_t *perm;
  // pushes: task t sums its push stream (kind 4) into part[tseg[tsptr[t] + r]], row r
  const int32_t *tsptr, *tseg;
  double *part;
  // streams, kinds 0 forward gather, 1 forward inverse, 2 backward gather, 3 backward inverse
  // (per phase), 4 push (per task): values, indices, per-phase (task) offset, entries per
  // thread, thread stride, first rows of the slices
  const double *sval[kStreamKinds];
  const int32_t *sidx[kStreamKinds];
  const int64_t *s_off[kStreamKinds];
  const int32_t *s_K[kStreamKinds];
  const int32_t *s_T[kStreamKinds];
  const int32_t *s_ra[kStreamKinds];
  // task-local staging (task_inl[t] != 0): the task's rows, then its incoming partial sums
  // part[task_pin[t] ..] (forward) or the later-task rows task_xrow[task_xoff[t] ..]
  // (backward) are staged in LDS and the fg / bg stream indices address that buffer
  const int32_t *task_pin, *task_inl;
  const int64_t *task_xoff;
  const int32_t *task_xrow;
  int32_t lds_rows;  // LDS doubles for a staged task (at least every staged task's total)
  int32_t c_cap;     // LDS doubles for the right-hand sides of a phase's components
};

struct SolveSchedule {
  std::vector<int32_t> fwd_gptr, bwd_gptr;  // host: group boundaries
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
// overwritten with the new ones.
hipError_t launch_project_admm(hipStream_t s, bool f32, int n, int count, const int32_t *ids, const int64_t *boff,
                               const int32_t *bsz, const double *Xb, double *S, const DevState *st, double scale,
                               double *Q, const int64_t *qoff, bool warm);
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

}  // namespace dev
}  // namespace strom
