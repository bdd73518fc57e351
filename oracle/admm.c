/*
 * admm.c -- oracle side: sGS-ADMM (Algorithm 1 of the paper) on a PSD-only multi-block SDP,
 * with the KKT residuals of the paper's termination rule.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Shares nothing with the HIP path.
 *
 * Primal  min <C,X> s.t. A(X) = b, X in Omega_+;  dual  max <b,y> s.t. A^*y + S = C, S PSD.
 * One iteration, in the paper's order:
 *   step 1: r = b/sigma - A(X/sigma + S - C),          y_half = (A A^*)^{-1} r
 *   step 2: X_b = X + sigma (A^* y_half - C),          S = (Pi(X_b) - X_b) / sigma
 *   step 3: r = b/sigma - A(X/sigma + S - C),          y = (A A^*)^{-1} r
 *   step 4: X = X + tau sigma (S + A^* y - C)
 * Termination (KKT residual equation): eta = max(eta_p, eta_d, eta_g) <= tol, with
 *   eta_p = ||A(X) - b|| / (1 + ||b||),  eta_d = ||A^*y + S - C|| / (1 + ||C||),
 *   eta_g = |<C,X> - <b,y>| / (1 + |<C,X>| + |<b,y>|),
 * two-norms on R^m and Frobenius norms (= 2-norms of svec) on Omega.
 * (A A^*)^{-1} is applied through the LDL^T factor of eps I + A A^* (ldl.c).
 * The paper fixes neither sigma nor its schedule.  Every `sigma_every` iterations the primal
 * infeasibility r_P = max(eta_p, eta_K), with eta_K = ||X - Pi(X)|| / (1 + ||X||) the distance
 * of X from the cone, is balanced against eta_d: sigma is multiplied by 1.5 when
 * eta_d > 3 r_P and divided by 1.5 when r_P > 3 eta_d, kept in [1e-4, 1e4].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "oracle.h"

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

void orc_default_opts(orc_opts *o) {
  o->sigma0 = 1.0;
  o->tau = 1.6;
  o->tol = 1e-6;
  o->maxiter = 100000;
  o->sigma_every = 50;
  o->eps_rel = 1e-12;
  o->verbose = 0;
}

/* out = A v */
static void spmv(int32_t m, const int64_t *rp, const int32_t *ci, const double *vx, const double *v,
                 double *out) {
  for (int32_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += vx[p] * v[ci[p]];
    out[i] = s;
  }
}

/* out = A^* y  (= sum_i y_i A_i in svec coordinates) */
static void spmv_t(int32_t m, int64_t n, const int64_t *rp, const int32_t *ci, const double *vx,
                   const double *y, double *out) {
  memset(out, 0, sizeof(double) * (size_t)n);
  for (int32_t i = 0; i < m; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) out[ci[p]] += vx[p] * y[i];
}

static double dot(int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

static int64_t svec_len(int32_t nblocks, const int32_t *bsize) {
  int64_t n = 0;
  for (int32_t k = 0; k < nblocks; ++k) n += (int64_t)bsize[k] * (bsize[k] + 1) / 2;
  return n;
}

/* Project every block of an svec vector onto the PSD cone. */
void orc_project_svec(int32_t nblocks, const int32_t *bsize, const double *in, double *out) {
  int64_t off = 0;
  for (int32_t k = 0; k < nblocks; ++k) {
    const int n = bsize[k];
    double *a = (double *)malloc(sizeof(double) * (size_t)n * n);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i <= j; ++i) {
        double v = in[off + (int64_t)j * (j + 1) / 2 + i];
        if (i != j) v *= M_SQRT1_2;
        a[(size_t)j * n + i] = v;
        a[(size_t)i * n + j] = v;
      }
    orc_project_psd(n, a, a);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i <= j; ++i) {
        double v = a[(size_t)j * n + i];
        out[off + (int64_t)j * (j + 1) / 2 + i] = (i == j) ? v : v * M_SQRT2;
      }
    free(a);
    off += (int64_t)n * (n + 1) / 2;
  }
}

void orc_kkt(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rp, const int32_t *ci,
             const double *vx, const double *b, const double *C, const double *X, const double *y,
             const double *S, orc_info *info) {
  const int64_t n = svec_len(nblocks, bsize);
  double *r = (double *)malloc(sizeof(double) * (size_t)m);
  double *d = (double *)malloc(sizeof(double) * (size_t)n);
  spmv(m, rp, ci, vx, X, r);
  for (int32_t i = 0; i < m; ++i) r[i] -= b[i];
  spmv_t(m, n, rp, ci, vx, y, d);
  for (int64_t i = 0; i < n; ++i) d[i] += S[i] - C[i];
  const double pobj = dot(n, C, X), dobj = dot(m, b, y);
  info->eta_p = sqrt(dot(m, r, r)) / (1.0 + sqrt(dot(m, b, b)));
  info->eta_d = sqrt(dot(n, d, d)) / (1.0 + sqrt(dot(n, C, C)));
  info->eta_g = fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
  info->eta = fmax(info->eta_p, fmax(info->eta_d, info->eta_g));
  info->pobj = pobj;
  info->dobj = dobj;
  free(r);
  free(d);
}

int orc_admm_solve(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rp,
                   const int32_t *ci, const double *vx, const double *b, const double *C,
                   const orc_opts *opts, double *X, double *y, double *S, orc_info *info,
                   double *hist) {
  orc_opts o;
  if (opts) o = *opts; else orc_default_opts(&o);
  memset(info, 0, sizeof *info);
  const int64_t n = svec_len(nblocks, bsize);
  const double t0 = now_s();
  orc_ldl *F = NULL;
  int rc = orc_ldl_factor(m, n, rp, ci, vx, o.eps_rel, &F);
  if (rc) return rc;
  info->nnzL = F->nnzL;
  const double t1 = now_s();
  info->t_setup_s = t1 - t0;

  double *v = (double *)malloc(sizeof(double) * (size_t)n);
  double *Aty = (double *)malloc(sizeof(double) * (size_t)n);
  double *Xb = (double *)malloc(sizeof(double) * (size_t)n);
  double *P = (double *)malloc(sizeof(double) * (size_t)n);
  double *r = (double *)malloc(sizeof(double) * (size_t)m);
  const double nb = sqrt(dot(m, b, b)), nC = sqrt(dot(n, C, C));
  double sigma = o.sigma0;
  const double tau = o.tau;

  int64_t it;
  for (it = 0; it < o.maxiter; ++it) {
    /* step 1 */
    for (int64_t i = 0; i < n; ++i) v[i] = X[i] / sigma + S[i] - C[i];
    spmv(m, rp, ci, vx, v, r);
    for (int32_t i = 0; i < m; ++i) y[i] = b[i] / sigma - r[i];
    orc_ldl_solve(F, y);
    /* step 2 */
    spmv_t(m, n, rp, ci, vx, y, Aty);
    for (int64_t i = 0; i < n; ++i) Xb[i] = X[i] + sigma * (Aty[i] - C[i]);
    orc_project_svec(nblocks, bsize, Xb, P);
    for (int64_t i = 0; i < n; ++i) S[i] = (P[i] - Xb[i]) / sigma;
    /* step 3 */
    for (int64_t i = 0; i < n; ++i) v[i] = X[i] / sigma + S[i] - C[i];
    spmv(m, rp, ci, vx, v, r);
    for (int32_t i = 0; i < m; ++i) y[i] = b[i] / sigma - r[i];
    orc_ldl_solve(F, y);
    /* step 4 */
    spmv_t(m, n, rp, ci, vx, y, Aty);
    for (int64_t i = 0; i < n; ++i) X[i] = X[i] + tau * sigma * (S[i] + Aty[i] - C[i]);

    /* KKT residuals of (X, y, S) */
    spmv(m, rp, ci, vx, X, r);
    double rp2 = 0.0;
    for (int32_t i = 0; i < m; ++i) rp2 += (r[i] - b[i]) * (r[i] - b[i]);
    double rd2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double d = Aty[i] + S[i] - C[i];
      rd2 += d * d;
    }
    const double pobj = dot(n, C, X), dobj = dot(m, b, y);
    info->eta_p = sqrt(rp2) / (1.0 + nb);
    info->eta_d = sqrt(rd2) / (1.0 + nC);
    info->eta_g = fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
    info->eta = fmax(info->eta_p, fmax(info->eta_d, info->eta_g));
    info->pobj = pobj;
    info->dobj = dobj;
    info->sigma = sigma;
    if (hist) {
      hist[4 * it + 0] = info->eta_p;
      hist[4 * it + 1] = info->eta_d;
      hist[4 * it + 2] = info->eta_g;
      hist[4 * it + 3] = sigma;
    }
    if (!(info->eta == info->eta)) break; /* NaN: diverged */
    if (info->eta <= o.tol) { info->converged = 1; it++; break; }
    if (o.sigma_every > 0 && (it + 1) % o.sigma_every == 0) {
      /* primal infeasibility including the cone: eta_K = ||X - Pi(X)|| / (1 + ||X||) */
      orc_project_svec(nblocks, bsize, X, P);
      double dk = 0.0, nx = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        const double d = P[i] - X[i];
        dk += d * d;
        nx += X[i] * X[i];
      }
      const double eta_k = sqrt(dk) / (1.0 + sqrt(nx));
      const double rp = fmax(info->eta_p, eta_k);
      if (info->eta_d > 3.0 * rp) sigma = fmin(sigma * 1.5, 1e4);
      else if (rp > 3.0 * info->eta_d) sigma = fmax(sigma / 1.5, 1e-4);
    }
  }
  info->iters = it;
  info->sigma = sigma;
  info->t_solve_s = now_s() - t1;
  free(v); free(Aty); free(Xb); free(P); free(r);
  orc_ldl_free(F);
  return 0;
}
