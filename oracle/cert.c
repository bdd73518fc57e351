/*
 * cert.c -- oracle side: the certificate pieces computed from an (X, y) pair.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Shares nothing with the HIP path.
 *
 * Valid lower bound of the refined certificate of suboptimality (Sec. "Algorithmic Backbone",
 * the valid-lower-bound equation): for any y and any bounds R_beta on the traces of the blocks
 * of the rank-one lifting of feasible points,
 *     lb(y) = <b, y> + sum_beta R_beta * min(0, lambda_min((C - A^* y)_beta)) <= p*.
 * Rank test and extraction (Sec. "Sparse Moment Relaxation", the convergence theorem's rank-one
 * condition and the extraction heuristic's first two steps): the two largest eigenvalues of a
 * block and the eigenvector of the largest, divided by its first entry.
 * Eigenvalues come from the oracle's cyclic Jacobi method (jacobi.c).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Dense n x n column-major copy of the svec block at sv (off-diagonal svec entries carry sqrt 2). */
static void unpack_block(int n, const double *sv, double *a) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) {
      double v = sv[(int64_t)j * (j + 1) / 2 + i];
      if (i != j) v *= M_SQRT1_2;
      a[(size_t)j * n + i] = v;
      a[(size_t)i * n + j] = v;
    }
}

int orc_dual_bound(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rp, const int32_t *ci,
                   const double *vx, const double *b, const double *C, const double *y, const double *R_beta,
                   double *lb, double *lam_min) {
  int64_t n = 0;
  for (int32_t k = 0; k < nblocks; ++k) n += (int64_t)bsize[k] * (bsize[k] + 1) / 2;
  double *z = (double *)malloc(sizeof(double) * (size_t)n);
  if (!z) return -1;
  /* Z = C - A^* y, with A^* y = sum_i y_i A_i in svec coordinates */
  memcpy(z, C, sizeof(double) * (size_t)n);
  for (int32_t i = 0; i < m; ++i)
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) z[ci[p]] -= vx[p] * y[i];
  double bound = 0.0;
  for (int32_t i = 0; i < m; ++i) bound += b[i] * y[i];
  int64_t off = 0;
  for (int32_t k = 0; k < nblocks; ++k) {
    const int nb = bsize[k];
    double *a = (double *)malloc(sizeof(double) * (size_t)nb * nb);
    double *v = (double *)malloc(sizeof(double) * (size_t)nb * nb);
    double *w = (double *)malloc(sizeof(double) * (size_t)nb);
    unpack_block(nb, z + off, a);
    orc_jacobi_eig(nb, a, v, w);
    double lmin = w[0];
    for (int i = 1; i < nb; ++i) lmin = fmin(lmin, w[i]);
    if (lam_min) lam_min[k] = lmin;
    bound += R_beta[k] * fmin(0.0, lmin);
    free(a);
    free(v);
    free(w);
    off += (int64_t)nb * (nb + 1) / 2;
  }
  *lb = bound;
  free(z);
  return 0;
}

int orc_extract(int32_t nblocks, const int32_t *bsize, const double *X, int32_t nlist, const int32_t *blocks,
                double *lam, double *vtop) {
  int64_t *boff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nblocks > 0 ? nblocks : 1));
  int64_t off = 0;
  for (int32_t k = 0; k < nblocks; ++k) {
    boff[k] = off;
    off += (int64_t)bsize[k] * (bsize[k] + 1) / 2;
  }
  int64_t out = 0;
  for (int32_t t = 0; t < nlist; ++t) {
    const int32_t k = blocks[t];
    if (k < 0 || k >= nblocks) { free(boff); return -1; }
    const int nb = bsize[k];
    double *a = (double *)malloc(sizeof(double) * (size_t)nb * nb);
    double *v = (double *)malloc(sizeof(double) * (size_t)nb * nb);
    double *w = (double *)malloc(sizeof(double) * (size_t)nb);
    unpack_block(nb, X + boff[k], a);
    orc_jacobi_eig(nb, a, v, w);
    int i1 = 0;  /* largest eigenvalue, then the second largest */
    for (int i = 1; i < nb; ++i) if (w[i] > w[i1]) i1 = i;
    int i2 = -1;
    for (int i = 0; i < nb; ++i) if (i != i1 && (i2 < 0 || w[i] > w[i2])) i2 = i;
    lam[2 * t] = w[i1];
    lam[2 * t + 1] = i2 >= 0 ? w[i2] : 0.0;
    double s = v[(size_t)i1 * nb];  /* first entry of the top eigenvector */
    if (s == 0.0) {
      int ia = 0;
      for (int i = 1; i < nb; ++i) if (fabs(v[(size_t)i1 * nb + i]) > fabs(v[(size_t)i1 * nb + ia])) ia = i;
      s = v[(size_t)i1 * nb + ia] < 0 ? -1.0 : 1.0;
    }
    for (int i = 0; i < nb; ++i) vtop[out + i] = v[(size_t)i1 * nb + i] / s;
    out += nb;
    free(a);
    free(v);
    free(w);
  }
  free(boff);
  return 0;
}
