/*
 * ldl.c -- oracle side: sparse LDL^T factorization of  eps*I + A A^*  and its solve.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Shares nothing with the HIP path.
 *
 * The paper (Sec. "GPU Speedup", hybrid sparse linear system solver) factors
 * eps*I + A A^* = P L D L^T P^T once and then solves with it in both y-updates of
 * Algorithm 1.  The oracle uses the natural row order (P = I) -- any order gives the same
 * solution up to rounding -- and the textbook up-looking method: row k of L solves a sparse
 * lower-triangular system whose nonzero pattern is the set of elimination-tree paths
 * starting at the nonzeros of column k of the upper triangle.
 *
 * eps = eps_rel * max_i (A A^*)_ii with eps_rel = 1e-12 unless given.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

int orc_ldl_factor(int32_t m, int64_t nsvec, const int64_t *rowptr, const int32_t *col,
                   const double *val, double eps_rel, orc_ldl **out) {
  *out = NULL;
  if (m <= 0) return -1;
  if (eps_rel <= 0) eps_rel = 1e-12;

  /* A^T in CSR (rows of A^T = columns of A) */
  int64_t nnz = rowptr[m];
  int64_t *tp = (int64_t *)calloc((size_t)nsvec + 1, sizeof(int64_t));
  int32_t *ti = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
  double *tx = (double *)malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
  for (int64_t p = 0; p < nnz; ++p) tp[col[p] + 1]++;
  for (int64_t c = 0; c < nsvec; ++c) tp[c + 1] += tp[c];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nsvec + 1));
  memcpy(fill, tp, sizeof(int64_t) * (size_t)(nsvec + 1));
  for (int32_t i = 0; i < m; ++i)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int64_t q = fill[col[p]]++;
      ti[q] = i;
      tx[q] = val[p];
    }
  free(fill);

  /* K = A A^*: column k of the upper triangle, K(i,k) = sum_c A(k,c) A(i,c), i <= k */
  double *w = (double *)calloc((size_t)m, sizeof(double));
  int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  int32_t *lst = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  for (int32_t i = 0; i < m; ++i) mark[i] = -1;
  int64_t kcap = nnz * 4 + m, knz = 0;
  int64_t *Kp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
  int32_t *Ki = (int32_t *)malloc(sizeof(int32_t) * (size_t)kcap);
  double *Kx = (double *)malloc(sizeof(double) * (size_t)kcap);
  double maxdiag = 0.0;
  for (int32_t k = 0; k < m; ++k) {
    int nl = 0;
    for (int64_t p = rowptr[k]; p < rowptr[k + 1]; ++p) {
      int32_t c = col[p];
      for (int64_t q = tp[c]; q < tp[c + 1]; ++q) {
        int32_t i = ti[q];
        if (i > k) continue;
        if (mark[i] != k) { mark[i] = k; lst[nl++] = i; w[i] = 0.0; }
        w[i] += val[p] * tx[q];
      }
    }
    if (mark[k] != k) { mark[k] = k; lst[nl++] = k; w[k] = 0.0; }
    if (knz + nl > kcap) {
      kcap = 2 * (knz + nl);
      Ki = (int32_t *)realloc(Ki, sizeof(int32_t) * (size_t)kcap);
      Kx = (double *)realloc(Kx, sizeof(double) * (size_t)kcap);
    }
    Kp[k] = knz;
    for (int t = 0; t < nl; ++t) { Ki[knz] = lst[t]; Kx[knz] = w[lst[t]]; knz++; }
    if (w[k] > maxdiag) maxdiag = w[k];
  }
  Kp[m] = knz;
  free(tp); free(ti); free(tx);
  const double eps = eps_rel * (maxdiag > 0 ? maxdiag : 1.0);
  for (int32_t k = 0; k < m; ++k)
    for (int64_t p = Kp[k]; p < Kp[k + 1]; ++p)
      if (Ki[p] == k) Kx[p] += eps;

  /* symbolic: elimination tree and column counts of L */
  int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  int64_t *Lnz = (int64_t *)calloc((size_t)m, sizeof(int64_t));
  int32_t *flag = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  for (int32_t k = 0; k < m; ++k) {
    parent[k] = -1;
    flag[k] = k;
    for (int64_t p = Kp[k]; p < Kp[k + 1]; ++p) {
      int32_t i = Ki[p];
      if (i >= k) continue;
      for (; flag[i] != k; i = parent[i]) {
        if (parent[i] == -1) parent[i] = k;
        Lnz[i]++;
        flag[i] = k;
      }
    }
  }
  orc_ldl *F = (orc_ldl *)calloc(1, sizeof(orc_ldl));
  F->m = m;
  F->eps = eps;
  F->Lp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
  F->Lp[0] = 0;
  for (int32_t k = 0; k < m; ++k) F->Lp[k + 1] = F->Lp[k] + Lnz[k];
  F->nnzL = F->Lp[m];
  F->Li = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F->nnzL ? F->nnzL : 1));
  F->Lx = (double *)malloc(sizeof(double) * (size_t)(F->nnzL ? F->nnzL : 1));
  F->D = (double *)malloc(sizeof(double) * (size_t)m);

  /* numeric: row k of L from a sparse triangular solve on the etree reach */
  int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  int32_t *path = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  double *Y = w;
  memset(Y, 0, sizeof(double) * (size_t)m);
  for (int32_t k = 0; k < m; ++k) { Lnz[k] = 0; flag[k] = -1; }
  int rc = 0;
  for (int32_t k = 0; k < m && !rc; ++k) {
    int32_t top = m;
    flag[k] = k;
    for (int64_t p = Kp[k]; p < Kp[k + 1]; ++p) {
      int32_t i = Ki[p];
      Y[i] += Kx[p];
      if (i >= k) continue;
      int len = 0;
      for (; flag[i] != k; i = parent[i]) { path[len++] = i; flag[i] = k; }
      while (len > 0) stack[--top] = path[--len];
    }
    double dk = Y[k];
    Y[k] = 0.0;
    for (; top < m; ++top) {
      int32_t i = stack[top];
      double yi = Y[i];
      Y[i] = 0.0;
      int64_t p0 = F->Lp[i], p1 = F->Lp[i] + Lnz[i];
      for (int64_t p = p0; p < p1; ++p) Y[F->Li[p]] -= F->Lx[p] * yi;
      double lki = yi / F->D[i];
      dk -= lki * yi;
      F->Li[p1] = k;
      F->Lx[p1] = lki;
      Lnz[i]++;
    }
    if (!(dk > 0.0)) rc = -4;
    F->D[k] = dk;
  }
  free(stack); free(path); free(w); free(mark); free(lst); free(Kp); free(Ki); free(Kx);
  free(parent); free(Lnz); free(flag);
  if (rc) { orc_ldl_free(F); return rc; }
  *out = F;
  return 0;
}

void orc_ldl_solve(const orc_ldl *F, double *x) {
  const int32_t m = F->m;
  for (int32_t j = 0; j < m; ++j) {
    const double xj = x[j];
    for (int64_t p = F->Lp[j]; p < F->Lp[j + 1]; ++p) x[F->Li[p]] -= F->Lx[p] * xj;
  }
  for (int32_t j = 0; j < m; ++j) x[j] /= F->D[j];
  for (int32_t j = m - 1; j >= 0; --j) {
    double s = x[j];
    for (int64_t p = F->Lp[j]; p < F->Lp[j + 1]; ++p) s -= F->Lx[p] * x[F->Li[p]];
    x[j] = s;
  }
}

void orc_ldl_free(orc_ldl *F) {
  if (!F) return;
  free(F->Lp); free(F->Li); free(F->Lx); free(F->D);
  free(F);
}
