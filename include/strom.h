/*
 * strom.h -- C ABI of the MI355X sGS-ADMM solver for PSD-only multi-block SDPs.
 *
 * The solver runs Algorithm 1 of Kang, Xu, Sarva, Liang, Yang, "Fast and Certifiable
 * Trajectory Optimization" (sGS-ADMM, Sec. "Algorithmic Backbone") on the standard SDP
 *     min <C,X>  s.t.  A(X) = b,  X = (X_1, ..., X_B) with every X_beta PSD
 * (the standard multi-block SDP equation of Sec. "Faster Conversion to Standard SDP") and its
 * dual  max <b,y> s.t. A^*y + S = C, S PSD.  Every step of the iteration runs in HIP
 * kernels on one MI355X (gfx950); the host only does one-time setup (validation, the
 * ordering and the FP64 LDL^T factorization of eps*I + A A^*) and reads results back.
 *
 * Conventions shared by every call:
 *   - X, S and C are stored as the concatenation of the svec of every block in block order:
 *     column-major upper triangle, off-diagonal entries multiplied by sqrt(2), so that
 *     <svec P, svec Q> = tr(PQ) (the svec of the cited SDPT3 convention, Sec. "GPU Speedup").
 *   - A is CSR with m rows over the n_svec svec columns: row i holds svec(A_i), int64 row
 *     pointers, int32 column indices, FP64 values.
 *   - Every call returns a strom_status (0 = OK, < 0 = error) and never aborts or throws;
 *     strom_last_error() returns a thread-local description of the last error.
 *   - Host pointers are read before the call returns; the caller keeps ownership.
 *     Device pointers are caller-owned (for example PyTorch tensors); the library never
 *     frees them.  Device memory the library allocates itself belongs to the ctx / sdp
 *     handle and is released by the matching destroy call.
 *   - Work is enqueued on the HIP stream given to strom_ctx_create (or the stream argument
 *     of strom_project_psd_batched); calls that return host data synchronize that stream.
 *   - A strom_sdp handle must be used by one host thread at a time.
 */
#ifndef STROM_H
#define STROM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STROM_OK = 0,
  STROM_E_INVAL = -1,    /* malformed argument: bad CSR, column >= n_svec, block size <= 0 */
  STROM_E_NOMEM = -2,    /* device allocation failed or the HBM budget is exceeded          */
  STROM_E_HIP = -3,      /* a HIP runtime call failed                                       */
  STROM_E_FACTOR = -4,   /* a non-positive pivot in the LDL^T factor of eps*I + A A^*        */
  STROM_E_AGAIN = -5,    /* result not ready yet (strom_poll)                               */
  STROM_E_NOTFOUND = -6, /* unknown ticket                                                  */
  STROM_E_STATE = -7     /* call not valid in the handle's current state                    */
} strom_status;

typedef enum { STROM_F64 = 0, STROM_F32 = 1 } strom_dtype;

typedef enum {
  STROM_RUNNING = 0,
  STROM_CONVERGED = 1, /* eta <= tol                          */
  STROM_MAXITER = 2,   /* maxiter reached with eta > tol      */
  STROM_DIVERGED = 3   /* NaN or Inf in the KKT residuals     */
} strom_solve_state;

typedef struct strom_ctx strom_ctx; /* one per device: stream, scratch, HBM budget, queue */
typedef struct strom_sdp strom_sdp; /* one per SDP instance: device data, factor, iterates */

/* Solver options.  The paper fixes only tau in (0, 2) and sigma > 0 (Algorithm 1 input) and
 * the stopping rule eta <= tol or maxiter (termination paragraph); the other values are
 * this library's choices.  strom_default_opts fills:
 *   sigma0 = 1, tau = 1.6, eps_reg = 1e-12 (eps = eps_reg * max_i (A A^*)_ii), tol = 1e-6,
 *   maxiter = 100000, kkt_every = 10, proj_dtype = STROM_F64, polish_eta = 1e-5,
 *   sigma_every = 50, task_split = -1, block_rows = 0.  Sigma rule: every sigma_every iterations, with the primal
 *   infeasibility r_P = max(eta_p, eta_K), eta_K = ||X - Pi(X)|| / (1 + ||X||) the distance of
 *   X from the cone, sigma is multiplied by 1.5 when eta_d > 3 r_P and divided by 1.5 when
 *   r_P > 3 eta_d, kept in [1e-4, 1e4]; 0 keeps sigma fixed.  sigma_every must be a multiple
 *   of kkt_every (or 0).  With proj_dtype = STROM_F32 the projection runs in FP32 (FP64
 *   eigenvectors) until eta <= polish_eta or eta has not halved over 500 iterations, then in
 *   FP64 (the switch is taken where the residuals are read: strom_admm_step and the serving
 *   loop); y-solves, iterates and residuals are FP64 throughout. */
typedef struct {
  double sigma0;
  double tau;
  double eps_reg;
  double tol;
  int64_t maxiter;
  int32_t kkt_every;
  strom_dtype proj_dtype; /* precision of the eigensolver / reconstruction in the projection */
  double polish_eta;      /* with proj_dtype = F32: switch the projection to FP64 once eta <= polish_eta */
  int32_t sigma_every;
  /* load balancing of the y-solve's task schedule: 0 no task is split, 1 only tasks far above
   * the median cost, 2 every clique-group task (shortest dependency chain for one instance in
   * flight), -1 (default) the STROM_TASK_SPLIT environment variable if set, else 2.  In a
   * merged batch the instances supply the parallelism and 1 is faster. */
  int32_t task_split;
  /* largest connected component (rows) a phase of the y-solve solves through its explicit
   * inverse, 1..256; 0 (default): the STROM_BLOCK_ROWS environment variable if set, else 192.
   * Larger components mean fewer dependent phases (one instance's latency) but more inverse
   * entries to stream (a batch's throughput prefers 64). */
  int32_t block_rows;
} strom_opts;

typedef struct {
  double eta_p, eta_d, eta_g; /* KKT residuals of the termination rule (FP64) */
  double pobj, dobj;          /* <C,X> and <b,y> */
  double sigma;
  int64_t iters;
  strom_solve_state state;
  double t_queue_s, t_setup_s, t_solve_s;
} strom_info;

/* One SDP instance, host arrays.  The blocks X_beta are given by their sizes; the svec
 * length is sum_beta n_beta (n_beta + 1) / 2.  X0/S0 are the starting point of Algorithm 1
 * (NULL means zero). */
typedef struct {
  int32_t nblocks;
  const int32_t *block_sizes;
  int32_t m;
  int64_t nnz;
  const int64_t *A_rowptr; /* m + 1 */
  const int32_t *A_col;    /* nnz, svec column index of each entry */
  const double *A_val;     /* nnz */
  const double *b;         /* m */
  const double *C_svec;    /* n_svec */
  const double *X0_svec;   /* n_svec or NULL */
  const double *S0_svec;   /* n_svec or NULL */
} strom_problem;

void strom_default_opts(strom_opts *opts);
const char *strom_last_error(void);

/* Create a context on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t; NULL:
 * the context creates its own non-blocking stream, so that work of other threads on the
 * legacy default stream never waits on it).  hbm_budget_bytes bounds the device memory of
 * all instances set up in this ctx (0 = no bound).  Rounds of kkt_every iterations are
 * replayed from HIP graphs captured on a private non-blocking stream; the library's own
 * synchronous copies are serialized with those captures, and a caller must not enqueue work
 * on the legacy default stream from another thread while strom calls are in flight. */
strom_status strom_ctx_create(int device, void *hip_stream, size_t hbm_budget_bytes, strom_ctx **out);
strom_status strom_ctx_destroy(strom_ctx *ctx);

/* Set up one instance: validates the CSR (E_INVAL), orders the rows (clique interiors first,
 * then the rows coupling two cliques by nested dissection over the chain, a consequence of the
 * chain-like sparsity of Def. 1; inside each clique's interior either the given order or a
 * minimum-degree one, whichever gives the shorter modelled y-solve, decided once per sparsity
 * pattern up to 500,000 rows; the STROM_ROW_ORDER environment variable, 0 or 1, forces the
 * given or the minimum-degree order), factors eps*I + A A^* = P L D L^T P^T in FP64 on the host
 * (the paper's Cholesky-with-pre-permutation equation; E_FACTOR on a non-positive pivot),
 * uploads everything and sets the iterate to (X0, 0, S0).  opts may be NULL (defaults).
 * Blocks up to n = 113 are projected by one workgroup each (in FP64, or FP32 before the polish
 * switch); larger ones, up to n = 512 (E_INVAL beyond), by the multi-workgroup block Jacobi,
 * always in FP64, with about 16 n^2 bytes of device memory each. */
strom_status strom_sdp_setup(strom_ctx *ctx, const strom_problem *problem, const strom_opts *opts,
                             strom_sdp **out);
strom_status strom_sdp_destroy(strom_sdp *sdp);

/* Run up to n_iter iterations of Algorithm 1 (steps 1-4) on the device.  The KKT residuals
 * are evaluated every kkt_every iterations and after the last one; the call returns early
 * once eta <= tol (state CONVERGED), or NaN appears (DIVERGED), or maxiter is reached.
 * info (nullable) receives the residuals of the final iterate.  Synchronizes the stream. */
strom_status strom_admm_step(strom_sdp *sdp, int32_t n_iter, strom_info *info);

/* Enqueue exactly n_iter iterations without any host synchronization or convergence check
 * (the residual-balancing sigma rule still runs on the device).  Used for timing. */
strom_status strom_admm_enqueue(strom_sdp *sdp, int32_t n_iter);

/* Mean device time per iteration of each phase, measured with HIP events on the instance's
 * stream over `reps` real iterations (the iterate advances as with strom_admm_enqueue;
 * residuals are evaluated every iteration).  rhs and solve include both right-hand sides /
 * both y-solves of an iteration; project is the PSD projection of every block. */
typedef struct {
  double rhs_ms, solve_ms, xb_ms, project_ms, xupdate_ms, kkt_ms, iteration_ms;
} strom_phase_times;
strom_status strom_profile_iteration(strom_sdp *sdp, int32_t reps, strom_phase_times *out);

/* KKT residuals of the current iterate (termination-rule equation), FP64; synchronizes. */
strom_status strom_kkt_residuals(strom_sdp *sdp, strom_info *out);

/* Copy the current iterate to / from host arrays (X, S: n_svec; y: m).  Any pointer may be
 * NULL to skip that part.  set_iterate also resets the iteration count. */
strom_status strom_get_iterate(strom_sdp *sdp, double *X_svec, double *y, double *S_svec);
strom_status strom_set_iterate(strom_sdp *sdp, const double *X_svec, const double *y,
                               const double *S_svec);
/* Sizes of an instance: n_svec, m and nnz of the L factor. */
strom_status strom_sdp_sizes(strom_sdp *sdp, int64_t *n_svec, int32_t *m, int64_t *nnz_L);

/* Projection onto the PSD cone of nblocks dense symmetric blocks (the parallel PSD cone
 * projection of Sec. "GPU Speedup": eigendecomposition, negative eigenvalues set to zero,
 * reconstruction).  Block k is n_dev[k] x n_dev[k], column-major, starting at element
 * offset_dev[k] of in_dev / out_dev; in and out may alias.  n_dev, offset_dev, in_dev and
 * out_dev are device pointers; max_n (host) bounds every n_dev[k], 1 <= max_n <= 512.  When
 * one block and its eigenvectors fit one workgroup (160 KiB of LDS on gfx950, and a worker thread
 * per 2 x 2 block: max_n <= 113 in F64, <= 122 in F32) every block is projected by one
 * workgroup; beyond that (F64 only,
 * else E_INVAL) by the multi-workgroup block Jacobi, every block padded to max_n's size, with
 * temporary device memory of about 16 max_n^2 bytes per block.  A block with n_dev[k] <= 0 or
 * > max_n makes the call return E_INVAL (other blocks are still written).  dtype selects double
 * or float data.  The one-workgroup path reads only the upper triangle of each input block, the
 * other both; the output is exactly symmetric. */
strom_status strom_project_psd_batched(strom_ctx *ctx, int32_t nblocks, int32_t max_n,
                                       const int32_t *n_dev, const int64_t *offset_dev,
                                       const void *in_dev, void *out_dev, strom_dtype dtype,
                                       void *hip_stream);

/* Eigendecomposition of nblocks dense symmetric blocks (layout, limits and eigensolvers as
 * strom_project_psd_batched).  Eigenvalues of block k, in
 * ascending order (ties in index order), are written at element offset woff_dev[k] of w_dev;
 * with v_dev != NULL the eigenvectors are written as the columns of an n x n column-major block
 * at offset_dev[k] of v_dev (column j for eigenvalue j; v_dev may alias in_dev).  With
 * v_dev == NULL only eigenvalues are computed and the eigenvector work is skipped (the
 * eigenvalues-only mode used by the certificate below).  n_dev, offset_dev, woff_dev, in_dev,
 * w_dev and v_dev are device pointers; dtype selects double or float for in, w and v. */
strom_status strom_eig_batched(strom_ctx *ctx, int32_t nblocks, int32_t max_n, const int32_t *n_dev,
                               const int64_t *offset_dev, const void *in_dev, const int64_t *woff_dev,
                               void *w_dev, void *v_dev, strom_dtype dtype, void *hip_stream);

/* Valid lower bound of the refined certificate of suboptimality (Sec. "Algorithmic Backbone",
 * the valid-lower-bound equation after the rank-one lifting operator): for the current y,
 *     lb = <b, y> + sum_beta R_beta * min(0, lambda_min((C - A^* y)_beta)),
 * a lower bound of the POP optimum whenever R_beta >= trace(X(z)_beta) for every feasible z
 * (the rank-one lifting; App. "Existence of R_beta" gives such bounds from box bounds on the
 * clique variables: they are problem knowledge, so the caller supplies them).  R_beta: host,
 * nblocks values.  lb (host) receives the bound; lam_min (host, nullable, nblocks) the smallest
 * eigenvalue of every block of C - A^* y.  FP64; synchronizes; uses temporary device memory. */
strom_status strom_dual_bound(strom_sdp *sdp, const double *R_beta, double *lb, double *lam_min);

/* strom_dual_bound without any device allocation, for callers that cannot allocate (code
 * around graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and synchronization as strom_dual_bound; its temporary device memory (the dense
 * copies of every block, their eigenvalues and the index lists) lives in a static per-device
 * work buffer of strom_scratch_bytes() bytes (32 MiB, held until the process ends), whose
 * address is taken when the device's first context is created.  E_INVAL (nothing launched)
 * when the instance's blocks need more than that: about 8 * sum n_beta^2 bytes plus the
 * eigenvalues.  Every call on a device shares the buffer: the library serializes its own calls,
 * but calls that overlap on one device from elsewhere race. */
strom_status strom_dual_bound_noalloc(strom_sdp *sdp, const double *R_beta, double *lb, double *lam_min);
size_t strom_scratch_bytes(void);

/* Rank test and extraction from the current X (Sec. "Sparse Moment Relaxation": the rank-one
 * condition of the convergence theorem, and the first two steps of the extraction heuristic).
 * For each listed block: lam[2k], lam[2k+1] = the largest and second largest eigenvalue
 * (lam[2k+1] / lam[2k] small: numerically rank one), and vtop (n_k values per listed block,
 * concatenated) = the eigenvector of the largest eigenvalue scaled so that its first entry is 1
 * (for a moment matrix the entries after it are the degree-one moments z-bar); if that entry is
 * exactly 0 the vector is returned with unit norm and its largest entry positive.  blocks (host,
 * nlist block indices), lam and vtop are host arrays.  FP64; synchronizes; uses temporary
 * device memory.  E_INVAL for an index outside [0, nblocks). */
strom_status strom_extract(strom_sdp *sdp, int32_t nlist, const int32_t *blocks, double *lam, double *vtop);

/* Merged form: Alg. 1 advanced for many independent instances at once.  A batch groups instances
 * of one ctx that were set up with the same kkt_every and sigma_every and whose iteration
 * counts agree modulo kkt_every (a fresh instance, at 0, joins instances that have run whole
 * rounds); while it exists they are iterated only through it (strom_admm_step,
 * strom_admm_enqueue, strom_set_iterate and strom_sdp_destroy on them return E_STATE).  Each
 * step of the iteration is one launch over all instances (a workgroup per row or column chunk,
 * solve task or PSD block of any instance; the solve's dependency groups are merged by depth),
 * and a round of kkt_every iterations is captured as a HIP graph.  Every instance keeps its
 * own arrays, options, sigma, polish switch and state: strom_batch_step advances the running
 * instances by up to n_iter iterations and retires each one, unchanged from then on, at the
 * round where it converges, reaches maxiter or diverges, exactly as strom_admm_step would.
 * instances: host array of count handles (copied).  infos (host, nullable): count entries,
 * filled as strom_admm_step fills its info.  Synchronizes once per round.  Instances with
 * blocks beyond one workgroup's LDS (see strom_sdp_setup) are not batched: E_INVAL. */
typedef struct strom_batch strom_batch;
strom_status strom_batch_create(strom_ctx *ctx, int32_t count, strom_sdp *const *instances, strom_batch **out);
strom_status strom_batch_step(strom_batch *batch, int32_t n_iter, strom_info *infos);
/* Autotuner of the merged projection: for every class of blocks (block size n and default
 * threads per workgroup, which is the instance's own launch configuration) and each precision
 * in use, times reps launches of every thread count the kernel accepts for n on the batch's
 * current iterates and keeps the fastest (the timing launches refresh the kept eigenvectors
 * and overwrite the X_b scratch, as a sigma-rule projection does).  reps = 0 only reports.
 * Needs at least one completed iteration (E_STATE otherwise).  Reports up to cap classes: n,
 * threads per workgroup for FP64 and FP32 (host arrays, nullable), and the class count in
 * nclass (nullable). */
strom_status strom_batch_tune(strom_batch *batch, int32_t reps, int32_t cap, int32_t *n, int32_t *nt_f64,
                              int32_t *nt_f32, int32_t *nclass);
/* Releases the batch (not its instances, which can be stepped on their own again). */
strom_status strom_batch_destroy(strom_batch *batch);

/* Serving.  strom_submit copies a problem and queues it; a solver thread owned by the ctx
 * admits queued problems while their device footprint fits the ctx's HBM budget, keeps their
 * iterates on the device, advances every admitted instance, retires an instance when it
 * converges (or reaches maxiter, or diverges) and admits the next.  strom_poll returns
 * E_AGAIN while the ticket is in flight; once done it fills info (and the optional host
 * arrays) and forgets the ticket.  The loop iterates merged batches: a problem with blocks
 * beyond one workgroup's LDS (see strom_sdp_setup) is refused with E_INVAL. */
strom_status strom_submit(strom_ctx *ctx, const strom_problem *problem, const strom_opts *opts,
                          uint64_t *ticket);
strom_status strom_poll(strom_ctx *ctx, uint64_t ticket, strom_info *out, double *X_svec,
                        double *y, double *S_svec);

#ifdef __cplusplus
}
#endif
#endif
