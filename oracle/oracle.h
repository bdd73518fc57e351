/*
 * oracle.h -- plain FP64 CPU oracle for the sGS-ADMM moment-relaxation solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * library: only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * do.  It shares no code, header, table or helper with the HIP path.
 *
 * It is written to be checked against the paper by eye, not to be fast:
 *   - relax.c / pop.c : polynomial trajectory problems and their sparse second-order moment
 *                       relaxation converted to a PSD-only multi-block SDP
 *                       (Sec. "Sparse Moment Relaxation", Prop. 1 and "Faster Conversion to
 *                       Standard SDP", the four constraint types of the worked example).
 *   - ldl.c           : sparse LDL^T factorization of eps*I + A A^*, up-looking, natural order
 *                       (Sec. "GPU Speedup", hybrid sparse linear system solver equation).
 *   - jacobi.c        : cyclic two-sided Jacobi eigensolver and PSD projection
 *                       (Sec. "GPU Speedup", parallel PSD cone projection: eig, clamp, rebuild).
 *   - admm.c          : Algorithm 1 (sGS-ADMM), the KKT residuals of the termination rule
 *                       and a residual-balancing sigma rule (Sec. "Algorithmic Backbone").
 */
#ifndef STROM_ORACLE_H
#define STROM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem families (the polynomial trajectory problems the relaxation is built from). */
enum {
  ORC_TOY1D = 0,          /* worked example of the paper: xdot = -(1+u)x, |u| <= 1   */
  ORC_PENDULUM = 1,       /* pendulum, explicit Euler + Cayley rotation, 7-var cliques */
  ORC_CARTPOLE = 2,       /* cart-pole, explicit Euler + Cayley rotation, 11-var cliques */
  ORC_PAPER_PENDULUM = 3, /* the paper's variational-integrator pendulum (sizes only)   */
  ORC_CAR = 4,            /* planar car, unicycle-12 / bicycle-13, one obstacle          */
  ORC_FLYING = 5,         /* the paper's flying robot (App. "Flying Robot"), 20-var cliques */
  ORC_LANDING = 6,        /* the paper's vehicle landing (App. "Vehicle Landing"), 18-var cliques */
  ORC_BACKIN = 7,         /* the paper's car back-in (App. "Car Back-in"), 18-var cliques */
  ORC_PAPER_CARTPOLE = 8  /* the paper's cart-pole (App. "Cart-Pole"), 13-var cliques with lookahead */
};

/* Row types, in the order they are generated inside a clique. */
enum { ORC_ROW_NORM = 0, ORC_ROW_MOMENT = 1, ORC_ROW_LOCALIZING = 2, ORC_ROW_EQUALITY = 3,
       ORC_ROW_CONSENSUS = 4 };

/* A PSD-only multi-block SDP  min <C,X>  s.t.  A(X) = b,  X in Omega_+.
 * X is stored as the concatenation of the svec of every block (column-major upper
 * triangle, off-diagonal entries scaled by sqrt(2)).  A is CSR over svec columns. */
typedef struct {
  int32_t nblocks;
  int32_t *bsize;    /* block dimension                                  */
  int32_t *bkind;    /* 0 = moment matrix M_k, 1 = localizing L_{k,i}    */
  int32_t *bclique;  /* clique index                                     */
  int64_t *boff;     /* svec offset of the block                          */
  int64_t nsvec;
  int32_t m;
  int64_t nnz;
  int64_t *rowptr;   /* m + 1 */
  int32_t *col;      /* nnz, ascending inside a row */
  double *val;       /* nnz */
  double *b;         /* m */
  double *C;         /* nsvec */
  int32_t *rowkind;  /* m, ORC_ROW_* */
  int32_t *rowclique;/* m */
  int32_t nclique_vars;  /* variables per clique */
  int32_t dx, du;        /* state / control dimension */
} orc_sdp;

/* Build the relaxation.  params depend on the family:
 *   TOY1D:          [x_init, dt, P_f]
 *   PENDULUM:       [theta0, omega0]
 *   CARTPOLE:       [x0, v0, theta0, omega0]
 *   PAPER_PENDULUM: [theta0, omega0]
 *   CAR:            [variant(0 unicycle-12, 1 bicycle-13), sx, sy, heading0, gx, gy, ox, oy]
 *   FLYING, LANDING: [x0, y0, theta0, vx0, vy0, omega0]
 *   BACKIN:         [x0, y0, theta0]
 *   PAPER_CARTPOLE: [a0, adot0, theta0, thetadot0]  (theta from the hanging position)
 * Returns 0 on success, <0 on a bad argument. */
int orc_relax(int family, int N, const double *params, int nparams, orc_sdp **out);
void orc_sdp_free(orc_sdp *p);

/* Number of lookahead variables of a family (0 for most): clique k of such a family holds
 * (x_k, u_k, x_{k+1}) followed by some components of x_{k+2}, which it shares with clique k+1. */
int orc_lookahead(int family);
/* The same, with the lookahead components (indices into x) written to lmap (up to 21). */
int orc_lookahead_map(int family, int *lmap);

/* Evaluate the POP at a trajectory z (all clique variables in chain order:
 * x_0, u_0, x_1, u_1, ..., x_N, in scaled variables, then for a family with lookahead the
 * lookahead components of x_{N+1}).  Writes the rank-one lifting
 * X(z) in svec form (length nsvec) and returns the POP objective sum_k f_k(z).
 * Used to pin A and C against the POP (A(X(z)) = b, <C,X(z)> = f(z)). */
double orc_lift(int family, int N, const double *params, int nparams, const double *z,
                double *X_svec);
/* Roll out the dynamics from the initial state with the given (scaled) controls
 * u[0..N*du-1]; writes z (length (N+1)*dx + N*du + orc_lookahead(family)) and returns the
 * POP objective. */
double orc_rollout(int family, int N, const double *params, int nparams, const double *u,
                   double *z);

/* Trace bounds R_beta (nblocks values, block order of orc_relax) for the certificate's lower
 * bound: every trace of a block of the rank-one lifting of a feasible point is below them
 * (App. "Existence of R_beta", see relax.c).  Returns -2 if a variable of the family is
 * unbounded (the pendulum's angular rate). */
int orc_trace_bounds(int family, int N, const double *params, int nparams, double *R_beta);

/* ---- sparse LDL^T of eps I + A A^* (ldl.c) ---- */
typedef struct {
  int32_t m;
  double eps;
  int64_t *Lp;     /* m + 1, CSC column pointers of strictly lower L */
  int32_t *Li;
  double *Lx;
  double *D;
  int64_t nnzL;
} orc_ldl;
/* eps_rel <= 0 selects the default 1e-12 * max diag(A A^*). */
int orc_ldl_factor(int32_t m, int64_t nsvec, const int64_t *rowptr, const int32_t *col,
                   const double *val, double eps_rel, orc_ldl **out);
void orc_ldl_solve(const orc_ldl *f, double *x);  /* in place: x <- (eps I + A A^*)^{-1} x */
void orc_ldl_free(orc_ldl *f);

/* ---- projection (jacobi.c) ---- */
/* Symmetric eigendecomposition of the n x n column-major matrix a (overwritten by its
 * eigenvalues on the diagonal); v receives the eigenvectors as columns.  Returns sweeps. */
int orc_jacobi_eig(int n, double *a, double *v, double *w);
/* Pi_{S_+}(a) for one dense n x n column-major block, out may alias a. */
int orc_project_psd(int n, const double *a, double *out);

/* ---- sGS-ADMM (admm.c) ---- */
typedef struct {
  double sigma0;     /* initial sigma                         (default 1)    */
  double tau;        /* dual step length                      (default 1.6)  */
  double tol;        /* stop when eta <= tol                  (default 1e-6) */
  int64_t maxiter;   /*                                       (default 1e5)  */
  int32_t sigma_every;  /* residual-balancing period, 0 = fixed sigma (default 50) */
  double eps_rel;    /* LDL regularization, <= 0 -> 1e-12     */
  int32_t verbose;
} orc_opts;

typedef struct {
  double eta_p, eta_d, eta_g, eta, pobj, dobj, sigma;
  int64_t iters;
  int32_t converged;
  double t_setup_s, t_solve_s;
  int64_t nnzL;
} orc_info;

void orc_default_opts(orc_opts *o);
/* Solve an SDP given in CSR svec form.  X, y, S are in/out (X, S: nsvec; y: m):
 * their values on entry are the starting point (X^0, S^0; y is ignored on entry).
 * hist (nullable, length >= 4*maxiter) receives eta_p, eta_d, eta_g, sigma per iteration. */
int orc_admm_solve(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
                   const int32_t *col, const double *val, const double *b, const double *C,
                   const orc_opts *opts, double *X, double *y, double *S, orc_info *info,
                   double *hist);

/* One projection of every block of an svec vector (used to compare a single
 * projection step block by block). */
void orc_project_svec(int32_t nblocks, const int32_t *bsize, const double *in, double *out);

/* KKT residuals of a given (X, y, S) in the sense of the termination rule. */
void orc_kkt(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
             const int32_t *col, const double *val, const double *b, const double *C,
             const double *X, const double *y, const double *S, orc_info *info);

/* ---- certificate (cert.c) ---- */
/* lb = <b,y> + sum_beta R_beta min(0, lambda_min((C - A^* y)_beta)); lam_min (nullable)
 * receives lambda_min per block.  Returns 0, or < 0 on an allocation failure. */
int orc_dual_bound(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
                   const int32_t *col, const double *val, const double *b, const double *C,
                   const double *y, const double *R_beta, double *lb, double *lam_min);
/* For each listed block of X (svec): lam[2t], lam[2t+1] = largest and second largest eigenvalue;
 * vtop (n per listed block, concatenated) = the top eigenvector divided by its first entry.
 * Returns 0, or < 0 for a block index out of range. */
int orc_extract(int32_t nblocks, const int32_t *bsize, const double *X, int32_t nlist,
                const int32_t *blocks, double *lam, double *vtop);

#ifdef __cplusplus
}
#endif
#endif
