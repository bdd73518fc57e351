// kernels.hip -- gfx950 kernels of one sGS-ADMM iteration (Algorithm 1 of the paper), except
// the PSD projection (project.hip).
//
// Iteration (sigma, tau read from device memory so that the host never synchronizes):
//   step 1  k_rhs        r = b/sigma - A(X/sigma + S - C), written in the factor's row order
//           k_solve_fwd  L z = r      (tasks of one dependency depth per launch)
//           k_solve_bwd  L^T x = D^{-1} z, y = P x
//   step 2  k_xb         X_b = X + sigma (A^* y - C)
//           k_project    S = (Pi(X_b) - X_b) / sigma, one workgroup per PSD block
//   step 3  k_rhs, k_solve_fwd, k_solve_bwd  (with the new S)
//   step 4  k_xupdate    X += tau sigma (S + A^* y - C), with the dual-residual partial sums
//   KKT     k_kkt_rows + k_kkt_final  (termination-rule residuals, sigma balancing)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace strom {
namespace dev {

// ------------------------------------------------------------------ reductions
template <int NT>
__device__ inline double block_sum(double v, double *red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ step 1 / 3: right-hand side
__global__ void __launch_bounds__(256) k_rhs(int32_t m, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                             const double *__restrict__ av, const double *__restrict__ X,
                                             const double *__restrict__ S, const double *__restrict__ C,
                                             const double *__restrict__ b, const int32_t *__restrict__ pinv,
                                             const DevState *__restrict__ st, double *__restrict__ w) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double sig = st->sigma;
  double acc = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
    const int32_t c = ci[p];
    acc += av[p] * (X[c] / sig + S[c] - C[c]);
  }
  w[pinv[i]] = b[i] / sig - acc;
}

// ------------------------------------------------------------------ triangular solves
// One workgroup per task.  Level tasks walk their rows level by level with a barrier in
// between; dense tasks gather the contributions of earlier tasks and multiply by the
// explicit inverse of their diagonal block.
__global__ void __launch_bounds__(256) k_solve_fwd(const int32_t *__restrict__ tasks, SolveArgs a, double *__restrict__ w) {
  extern __shared__ double sh[];
  const int32_t t = tasks[blockIdx.x];
  const int32_t r0 = a.task_r0[t], r1 = a.task_r1[t];
  if (a.task_type[t] == 0) {
    const int32_t l0 = a.task_flev0[t], nl = a.task_fnlev[t];
    for (int32_t l = 0; l < nl; ++l) {
      const int32_t k0 = a.flevptr[l0 + l], k1 = a.flevptr[l0 + l + 1];
      for (int32_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
        const int32_t i = a.frows[k];
        double s = w[i];
        for (int64_t p = a.Lrp[i]; p < a.Lrp[i + 1]; ++p) s -= a.Lv[p] * w[a.Lci[p]];
        w[i] = s;
      }
      __threadfence_block();
      __syncthreads();
    }
  } else {
    const int32_t nt = r1 - r0;
    double *c = sh;
    for (int32_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
      double s = w[i];
      for (int64_t p = a.Lrp[i]; p < a.Lrp[i + 1]; ++p) {
        const int32_t j = a.Lci[p];
        if (j >= r0) break;  // columns ascending: the rest lies in the diagonal block
        s -= a.Lv[p] * w[j];
      }
      c[i - r0] = s;
    }
    __syncthreads();
    const double *inv = a.inv + a.task_inv[t];
    for (int32_t i = threadIdx.x; i < nt; i += blockDim.x) {
      double x = 0.0;
      for (int32_t j = 0; j <= i; ++j) x += inv[i + (int64_t)j * nt] * c[j];
      w[r0 + i] = x;
    }
  }
}

__global__ void __launch_bounds__(256) k_solve_bwd(const int32_t *__restrict__ tasks, SolveArgs a, double *__restrict__ w,
                                                   double *__restrict__ y) {
  extern __shared__ double sh[];
  const int32_t t = tasks[blockIdx.x];
  const int32_t r0 = a.task_r0[t], r1 = a.task_r1[t];
  if (a.task_type[t] == 0) {
    const int32_t l0 = a.task_blev0[t], nl = a.task_bnlev[t];
    for (int32_t l = 0; l < nl; ++l) {
      const int32_t k0 = a.blevptr[l0 + l], k1 = a.blevptr[l0 + l + 1];
      for (int32_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
        const int32_t j = a.brows[k];
        double s = w[j] / a.D[j];
        for (int64_t p = a.Urp[j]; p < a.Urp[j + 1]; ++p) s -= a.Uv[p] * w[a.Uci[p]];
        w[j] = s;
        y[a.perm[j]] = s;
      }
      __threadfence_block();
      __syncthreads();
    }
  } else {
    const int32_t nt = r1 - r0;
    double *c = sh;
    for (int32_t j = r0 + threadIdx.x; j < r1; j += blockDim.x) {
      double s = w[j] / a.D[j];
      for (int64_t p = a.Urp[j]; p < a.Urp[j + 1]; ++p) {
        const int32_t i = a.Uci[p];
        if (i < r1) continue;  // inside the diagonal block
        s -= a.Uv[p] * w[i];
      }
      c[j - r0] = s;
    }
    __syncthreads();
    const double *invT = a.invT + a.task_inv[t];
    for (int32_t j = threadIdx.x; j < nt; j += blockDim.x) {
      double x = 0.0;
      for (int32_t i = j; i < nt; ++i) x += invT[(int64_t)i * nt + j] * c[i];
      w[r0 + j] = x;
      y[a.perm[r0 + j]] = x;
    }
  }
}

// ------------------------------------------------------------------ step 2: X_b
__global__ void __launch_bounds__(256) k_xb(int64_t n, const int64_t *__restrict__ trp, const int32_t *__restrict__ tci,
                                            const double *__restrict__ tv, const double *__restrict__ y,
                                            const double *__restrict__ X, const double *__restrict__ C,
                                            const DevState *__restrict__ st, double *__restrict__ Xb) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double aty = 0.0;
  for (int64_t p = trp[c]; p < trp[c + 1]; ++p) aty += tv[p] * y[tci[p]];
  Xb[c] = X[c] + st->sigma * (aty - C[c]);
}

// ------------------------------------------------------------------ step 4: X update + dual residual
__global__ void __launch_bounds__(256) k_xupdate(int64_t n, const int64_t *__restrict__ trp, const int32_t *__restrict__ tci,
                                                 const double *__restrict__ tv, const double *__restrict__ y,
                                                 const double *__restrict__ S, const double *__restrict__ C,
                                                 const DevState *__restrict__ st, double *__restrict__ X,
                                                 double *__restrict__ part, int32_t update) {
  __shared__ double red[256];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d2 = 0.0, cx = 0.0;
  if (c < n) {
    double aty = 0.0;
    for (int64_t p = trp[c]; p < trp[c + 1]; ++p) aty += tv[p] * y[tci[p]];
    const double d = S[c] + aty - C[c];
    double xn = X[c];
    if (update) {
      xn += st->tau * st->sigma * d;
      X[c] = xn;
    }
    d2 = d * d;
    cx = C[c] * xn;
  }
  if (part) {
    d2 = block_sum<256>(d2, red);
    cx = block_sum<256>(cx, red);
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x] = d2;
      part[2 * blockIdx.x + 1] = cx;
    }
  }
}

// ------------------------------------------------------------------ KKT
__global__ void __launch_bounds__(256) k_kkt_rows(int32_t m, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                  const double *__restrict__ av, const double *__restrict__ X,
                                                  const double *__restrict__ b, const double *__restrict__ y,
                                                  double *__restrict__ part) {
  __shared__ double red[256];
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  double r2 = 0.0, by = 0.0;
  if (i < m) {
    double ax = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) ax += av[p] * X[ci[p]];
    const double r = ax - b[i];
    r2 = r * r;
    by = b[i] * y[i];
  }
  r2 = block_sum<256>(r2, red);
  by = block_sum<256>(by, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r2;
    part[2 * blockIdx.x + 1] = by;
  }
}

// Per-block partial sums of ||a||^2 and ||b||^2 (a = Pi(X) - X, b = X for the cone distance).
__global__ void __launch_bounds__(256) k_sqnorms(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                                 double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sa = 0.0, sb = 0.0;
  if (c < n) {
    sa = a[c] * a[c];
    sb = b[c] * b[c];
  }
  sa = block_sum<256>(sa, red);
  sb = block_sum<256>(sb, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sa;
    part[2 * blockIdx.x + 1] = sb;
  }
}

// Sums the partials in a fixed order (deterministic), forms the residuals of the
// termination rule and, when asked, balances sigma: with eta_K = ||X - Pi(X)|| / (1 + ||X||)
// and r_P = max(eta_p, eta_K), sigma is multiplied by 1.5 when eta_d > 3 r_P and divided by
// 1.5 when r_P > 3 eta_d, kept in [1e-4, 1e4].
__global__ void k_kkt_final(const double *__restrict__ part_rows, int32_t nrow_parts,
                            const double *__restrict__ part_cols, int32_t ncol_parts,
                            const double *__restrict__ part_cone, double normb, double normC,
                            int32_t do_sigma, DevState *__restrict__ st) {
  __shared__ double red[256];
  double r2 = 0.0, by = 0.0, d2 = 0.0, cx = 0.0, k2 = 0.0, x2 = 0.0;
  for (int32_t k = threadIdx.x; k < nrow_parts; k += blockDim.x) { r2 += part_rows[2 * k]; by += part_rows[2 * k + 1]; }
  for (int32_t k = threadIdx.x; k < ncol_parts; k += blockDim.x) { d2 += part_cols[2 * k]; cx += part_cols[2 * k + 1]; }
  if (do_sigma)
    for (int32_t k = threadIdx.x; k < ncol_parts; k += blockDim.x) { k2 += part_cone[2 * k]; x2 += part_cone[2 * k + 1]; }
  r2 = block_sum<256>(r2, red);
  by = block_sum<256>(by, red);
  d2 = block_sum<256>(d2, red);
  cx = block_sum<256>(cx, red);
  k2 = block_sum<256>(k2, red);
  x2 = block_sum<256>(x2, red);
  if (threadIdx.x == 0) {
    const double ep = sqrt(r2) / (1.0 + normb);
    const double ed = sqrt(d2) / (1.0 + normC);
    const double eg = fabs(cx - by) / (1.0 + fabs(cx) + fabs(by));
    st->eta_p = ep;
    st->eta_d = ed;
    st->eta_g = eg;
    st->pobj = cx;
    st->dobj = by;
    st->sigma_used = st->sigma;
    if (do_sigma) {
      const double ek = sqrt(k2) / (1.0 + sqrt(x2));
      const double rp = fmax(ep, ek);
      if (ed > 3.0 * rp) st->sigma = fmin(st->sigma * 1.5, 1e4);
      else if (rp > 3.0 * ed) st->sigma = fmax(st->sigma / 1.5, 1e-4);
    }
  }
}

// ------------------------------------------------------------------ host launchers
hipError_t launch_rhs(hipStream_t s, int32_t m, const int64_t *rp, const int32_t *ci, const double *av,
                      const double *X, const double *S, const double *C, const double *b, const int32_t *pinv,
                      const DevState *st, double *w) {
  hipLaunchKernelGGL(k_rhs, dim3((m + 255) / 256), dim3(256), 0, s, m, rp, ci, av, X, S, C, b, pinv, st, w);
  return hipGetLastError();
}

hipError_t launch_solve(hipStream_t s, const SolveSchedule &sch, const SolveArgs &a, double *w, double *y) {
  const size_t lds = sizeof(double) * (size_t)(sch.max_dense_rows > 0 ? sch.max_dense_rows : 1);
  for (int g = 0; g + 1 < (int)sch.fwd_gptr.size(); ++g) {
    const int cnt = sch.fwd_gptr[g + 1] - sch.fwd_gptr[g];
    if (cnt <= 0) continue;
    hipLaunchKernelGGL(k_solve_fwd, dim3(cnt), dim3(256), lds, s, sch.fwd_order_dev + sch.fwd_gptr[g], a, w);
  }
  for (int g = 0; g + 1 < (int)sch.bwd_gptr.size(); ++g) {
    const int cnt = sch.bwd_gptr[g + 1] - sch.bwd_gptr[g];
    if (cnt <= 0) continue;
    hipLaunchKernelGGL(k_solve_bwd, dim3(cnt), dim3(256), lds, s, sch.bwd_order_dev + sch.bwd_gptr[g], a, w, y);
  }
  return hipGetLastError();
}

hipError_t launch_xb(hipStream_t s, int64_t n, const int64_t *trp, const int32_t *tci, const double *tv,
                     const double *y, const double *X, const double *C, const DevState *st, double *Xb) {
  hipLaunchKernelGGL(k_xb, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, trp, tci, tv, y, X, C, st, Xb);
  return hipGetLastError();
}

hipError_t launch_xupdate(hipStream_t s, int64_t n, const int64_t *trp, const int32_t *tci, const double *tv,
                          const double *y, const double *S, const double *C, const DevState *st, double *X,
                          double *part, int update) {
  hipLaunchKernelGGL(k_xupdate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, trp, tci, tv, y, S, C, st, X,
                     part, update);
  return hipGetLastError();
}

hipError_t launch_kkt(hipStream_t s, int32_t m, int64_t n, const int64_t *rp, const int32_t *ci, const double *av,
                      const double *X, const double *b, const double *y, double *part_rows, const double *part_cols,
                      const double *cone_diff, double *part_cone, double normb, double normC, int do_sigma,
                      DevState *st) {
  const int nrb = (m + 255) / 256;
  const int ncb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_kkt_rows, dim3(nrb), dim3(256), 0, s, m, rp, ci, av, X, b, y, part_rows);
  if (do_sigma) hipLaunchKernelGGL(k_sqnorms, dim3(ncb), dim3(256), 0, s, n, cone_diff, X, part_cone);
  hipLaunchKernelGGL(k_kkt_final, dim3(1), dim3(256), 0, s, part_rows, nrb, part_cols, ncb, part_cone, normb, normC,
                     do_sigma, st);
  return hipGetLastError();
}

}  // namespace dev
}  // namespace strom
