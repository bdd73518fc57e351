/*
 * jacobi.c -- oracle side: symmetric eigendecomposition by the cyclic two-sided Jacobi
 * method and the projection onto the PSD cone.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Shares nothing with the HIP path.
 *
 * The projection follows the paper's parallel PSD cone projection (Sec. "GPU Speedup"):
 * X = Q W Q^T, then Pi(X) = Q max(0, W) Q^T.  The eigendecomposition is the classical
 * cyclic-by-row Jacobi method with the numerically stable choice of the rotation
 * (tangent of the smaller angle, Rutishauser), as in Golub and Van Loan, Sec. 8.5.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define A_(i, j) a[(size_t)(j) * n + (i)]
#define V_(i, j) v[(size_t)(j) * n + (i)]

int orc_jacobi_eig(int n, double *a, double *v, double *w) {
  double fro = 0.0;
  for (size_t t = 0; t < (size_t)n * n; ++t) fro += a[t] * a[t];
  fro = sqrt(fro);
  const double thresh = 1e-18 * fro;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) V_(i, j) = (i == j) ? 1.0 : 0.0;
  int sweep;
  for (sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A_(p, q);
        if (apq == 0.0 || fabs(apq) <= thresh) continue;
        const double theta = (A_(q, q) - A_(p, p)) / (2.0 * apq);
        double t;
        if (fabs(theta) > 1e150) t = 0.5 / theta;
        else t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {
          if (r == p || r == q) continue;
          const double arp = A_(r, p), arq = A_(r, q);
          const double nrp = c * arp - s * arq, nrq = s * arp + c * arq;
          A_(r, p) = nrp; A_(p, r) = nrp;
          A_(r, q) = nrq; A_(q, r) = nrq;
        }
        A_(p, p) -= t * apq;
        A_(q, q) += t * apq;
        A_(p, q) = 0.0;
        A_(q, p) = 0.0;
        for (int r = 0; r < n; ++r) {
          const double vrp = V_(r, p), vrq = V_(r, q);
          V_(r, p) = c * vrp - s * vrq;
          V_(r, q) = s * vrp + c * vrq;
        }
        rotated++;
      }
    if (!rotated) break;
  }
  for (int i = 0; i < n; ++i) w[i] = A_(i, i);
  return sweep;
}

int orc_project_psd(int n, const double *a_in, double *out) {
  double *a = (double *)malloc(sizeof(double) * (size_t)n * n);
  double *v = (double *)malloc(sizeof(double) * (size_t)n * n);
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  memcpy(a, a_in, sizeof(double) * (size_t)n * n);
  int sweeps = orc_jacobi_eig(n, a, v, w);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) {
      double s = 0.0;
      for (int k = 0; k < n; ++k)
        if (w[k] > 0.0) s += w[k] * V_(i, k) * V_(j, k);
      out[(size_t)j * n + i] = s;
      out[(size_t)i * n + j] = s;
    }
  free(a); free(v); free(w);
  return sweeps;
}
