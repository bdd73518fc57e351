// project.hip -- projection of dense symmetric blocks onto the PSD cone (the parallel PSD cone
// projection of the paper's Sec. "GPU Speedup": eigendecomposition, negative eigenvalues set
// to zero, reconstruction), one workgroup per block with the block resident in LDS.
//
// Eigensolver: cyclic Jacobi in the round-robin parallel ordering.  In one round the n/2
// disjoint pairs are rotated together, A <- J^T A J; the new value of every 2x2 block
// (pair P1 x pair P2) depends only on its own four old entries, so the 2x2 blocks of the
// packed upper triangle are updated in parallel with no barrier inside the round.  Rotation
// parameters are computed in double for both storage types; the matrix is held in T (double,
// or float for the reduced-precision form); eigenvectors, norms and the reconstruction are
// double.
//
// Warm start (ADMM step): the eigenvectors of the previous call on the same block are kept
// in HBM; the sweeps start from A = Q^T X_b Q and V = Q, which is nearly diagonal once the
// iteration settles, so one to three sweeps replace the eight to ten of a cold start.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace strom {
namespace dev {

__device__ inline int pidx(int i, int j) {  // packed upper triangle, by columns
  if (i > j) { const int t = i; i = j; j = t; }
  return j * (j + 1) / 2 + i;
}

__device__ inline void tri_ij(int k, int &i, int &j) {  // k -> (i <= j) of the packed index
  j = (int)((sqrtf(8.0f * k + 1.0f) - 1.0f) * 0.5f);
  while (j * (j + 1) / 2 > k) --j;
  while ((j + 1) * (j + 2) / 2 <= k) ++j;
  i = k - j * (j + 1) / 2;
}

// Pair k of round r of the circle schedule over nn (even) slots, mm = nn - 1.
__device__ inline void rr_pair(int r, int k, int mm, int &p, int &q) {
  if (k == 0) { p = r; q = mm; }
  else {
    p = r + k;
    if (p >= mm) p -= mm;
    q = r - k;
    if (q < 0) q += mm;
  }
  if (p > q) { const int t = p; p = q; q = t; }
}

template <typename T>
struct JacobiTol;
template <>
struct JacobiTol<double> {
  static constexpr double off_rel = 1e-13;   // stop when off(A) <= off_rel * ||A||_F
  static constexpr double skip_rel = 1e-18;  // no rotation for |a_pq| <= skip_rel * ||A||_F
};
template <>
struct JacobiTol<float> {
  static constexpr double off_rel = 1e-6;
  static constexpr double skip_rel = 1e-9;
};

// LDS: V (n*n doubles, column-major) | red (nthreads doubles) | rotd (two buffers of 2 doubles
//      per pair: c, s) | A (packed upper triangle, T) | rot (two buffers of 4 T per pair: c, s,
//      new a_pp, new a_qq) | sel (n + 4 ints), every region 32-byte aligned.
struct Layout {
  size_t red, rotd, A, rot, sel, total;
};

__host__ __device__ inline size_t align32(size_t x) { return (x + 31) & ~(size_t)31; }

__host__ __device__ inline Layout lds_layout(int n, int nthreads, size_t tsize) {
  const size_t np2 = (size_t)(n + 1) / 2, npk = (size_t)n * (n + 1) / 2;
  Layout L;
  L.red = align32(8 * (size_t)n * n);
  L.rotd = align32(L.red + 8 * (size_t)nthreads);
  L.A = align32(L.rotd + 2 * 16 * np2);
  L.rot = align32(L.A + tsize * npk);
  L.sel = align32(L.rot + 2 * 4 * tsize * np2);
  L.total = align32(L.sel + 4 * ((size_t)n + 4));
  return L;
}

template <typename T>
inline size_t lds_bytes_t(int n, int nthreads) {
  return lds_layout(n, nthreads, sizeof(T)).total;
}

struct Smem {
  double *V, *red, *rotd;
  void *A, *rot;
  int *sel;
};

template <typename T>
__device__ inline Smem carve(unsigned char *base, int n) {
  const Layout L = lds_layout(n, blockDim.x, sizeof(T));
  Smem s;
  s.V = reinterpret_cast<double *>(base);
  s.red = reinterpret_cast<double *>(base + L.red);
  s.rotd = reinterpret_cast<double *>(base + L.rotd);
  s.A = base + L.A;
  s.rot = base + L.rot;
  s.sel = reinterpret_cast<int *>(base + L.sel);
  return s;
}

__device__ inline double wg_sum(double v, double *red) {
  const int tid = threadIdx.x, nth = blockDim.x;
  red[tid] = v;
  __syncthreads();
  for (int s = nth / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// A <- Q^T X Q (packed upper triangle) with Q = V (LDS) and X the svec block at xs (global).
// Each thread forms 4 entries of a column of W = X Q at a time from X staged through A, then
// A is overwritten column block by column block once W is complete: W is kept in the block's
// slot wq of the eigenvector buffer (n*n doubles, free until the eigenvectors are written back).
template <typename T>
__device__ __forceinline__ void rotate_into_basis(int n, const double *xs, const double *V, double *wq, T *A) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const double rs2 = 0.70710678118654752440;
  const int npk = n * (n + 1) / 2;
  for (int k = tid; k < npk; k += nth) {  // A <- X (packed, unscaled off-diagonal)
    int i, j;
    tri_ij(k, i, j);
    const double v = xs[k];
    A[k] = (T)(i == j ? v : v * rs2);
  }
  __syncthreads();
  const int nc4 = (n + 3) / 4;
  for (int e = tid; e < n * nc4; e += nth) {  // W(i, 4c .. 4c+3) = sum_k X(i,k) Q(k, 4c ..)
    const int i = e % n, c0 = 4 * (e / n);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int c1 = min(c0 + 1, n - 1), c2 = min(c0 + 2, n - 1), c3 = min(c0 + 3, n - 1);
    for (int k = 0; k < n; ++k) {
      const double x = (double)A[pidx(i, k)];
      s0 += x * V[c0 * n + k];
      s1 += x * V[c1 * n + k];
      s2 += x * V[c2 * n + k];
      s3 += x * V[c3 * n + k];
    }
    wq[c0 * n + i] = s0;
    if (c0 + 1 < n) wq[(c0 + 1) * n + i] = s1;
    if (c0 + 2 < n) wq[(c0 + 2) * n + i] = s2;
    if (c0 + 3 < n) wq[(c0 + 3) * n + i] = s3;
  }
  __threadfence_block();
  __syncthreads();
  for (int e = tid; e < npk; e += nth) {  // A(i, j) = sum_k Q(k, i) W(k, j), i <= j
    int i, j;
    tri_ij(e, i, j);
    const double *q = V + i * n;
    const double *w = wq + j * n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += q[k] * w[k];
    A[e] = (T)s;
  }
  __syncthreads();
}

template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
  typedef double4 type;
};
template <>
struct Vec4<float> {
  typedef float4 type;
};

// New value of the 2x2 block (pair I) x (pair J), I <= J, of round r.
template <typename T>
__device__ __forceinline__ void rotate_block(int r, int I, int J, int n, int mm, T *A, const T *rot) {
  typedef typename Vec4<T>::type V4;
  int p1, q1;
  rr_pair(r, I, mm, p1, q1);
  const V4 ri = reinterpret_cast<const V4 *>(rot)[I];
  if (I == J) {
    if (q1 < n) {
      A[pidx(p1, p1)] = ri.z;
      A[pidx(q1, q1)] = ri.w;
      A[pidx(p1, q1)] = T(0);
    }
    return;
  }
  int p2, q2;
  rr_pair(r, J, mm, p2, q2);
  const V4 rj = reinterpret_cast<const V4 *>(rot)[J];
  const T c1 = ri.x, s1 = ri.y, c2 = rj.x, s2 = rj.y;
  const bool hq1 = q1 < n, hq2 = q2 < n;
  const T a = A[pidx(p1, p2)];
  const T bq = hq2 ? A[pidx(p1, q2)] : T(0);
  const T cq = hq1 ? A[pidx(q1, p2)] : T(0);
  const T d = (hq1 && hq2) ? A[pidx(q1, q2)] : T(0);
  const T ra = c1 * a - s1 * cq, rb = c1 * bq - s1 * d;  // rows p1, q1 rotated
  const T rc = s1 * a + c1 * cq, rd = s1 * bq + c1 * d;
  A[pidx(p1, p2)] = c2 * ra - s2 * rb;  // then columns p2, q2
  if (hq2) A[pidx(p1, q2)] = s2 * ra + c2 * rb;
  if (hq1) A[pidx(q1, p2)] = c2 * rc - s2 * rd;
  if (hq1 && hq2) A[pidx(q1, q2)] = s2 * rc + c2 * rd;
}

// Rotation parameters of every pair of round r from A (threads t0, t0 + stride, ...).
template <typename T>
__device__ __forceinline__ void round_rotations(int r, int n, int np2, int mm, double skip, const T *A, T *rot, double *rotd,
                                       int t0, int stride) {
  for (int k = t0; k < np2; k += stride) {
    int p, q;
    rr_pair(r, k, mm, p, q);
    double c = 1.0, s = 0.0, dp = 0.0, dq = 0.0;
    if (q < n) {
      const double apq = (double)A[pidx(p, q)], app = (double)A[pidx(p, p)], aqq = (double)A[pidx(q, q)];
      dp = app;
      dq = aqq;
      if (fabs(apq) > skip) {
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        c = 1.0 / sqrt(t * t + 1.0);
        s = t * c;
        dp = app - t * apq;
        dq = aqq + t * apq;
      }
    }
    typedef typename Vec4<T>::type V4;
    V4 rv;
    rv.x = (T)c;
    rv.y = (T)s;
    rv.z = (T)dp;
    rv.w = (T)dq;
    reinterpret_cast<V4 *>(rot)[k] = rv;
    reinterpret_cast<double2 *>(rotd)[k] = make_double2(c, s);
  }
}

// V <- V J for the rotations rotd of round r: this thread's eigenvector row vrow, pairs
// vk0, vk0 + vks, ...
__device__ __forceinline__ void rotate_vectors(int r, int n, int np2, int mm, const double *rotd, double *V, int vrow, int vk0,
                                      int vks) {
  for (int k = vk0; k < np2; k += vks) {
    int p, q;
    rr_pair(r, k, mm, p, q);
    if (q >= n) continue;
    const double2 cs = reinterpret_cast<const double2 *>(rotd)[k];
    const double c = cs.x, s = cs.y;
    const double vp = V[vrow + p * n], vq = V[vrow + q * n];
    V[vrow + p * n] = c * vp - s * vq;
    V[vrow + q * n] = s * vp + c * vq;
  }
}

// Cyclic Jacobi, two barriers per round.  With enough threads (split), the first wave
// computes the rotations of round r while the other waves apply those of round r - 1 to the
// eigenvectors (rot / rotd double-buffered); then all threads rotate the 2x2 blocks of A.
template <typename T>
__device__ __forceinline__ void jacobi_eig(int n, T *A, double *V, T *rot, double *rotd, double *red, bool v_ready) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int np2 = (n + 1) / 2, nn = 2 * np2, mm = nn - 1;
  const int npk = n * (n + 1) / 2;
  const int nblk = np2 * (np2 + 1) / 2;  // at most 2 * nth (checked at launch)
  int I0 = -1, J0 = -1, I1 = -1, J1 = -1;  // this thread's 2x2 blocks, fixed over the rounds
  if (tid < nblk) tri_ij(tid, I0, J0);
  if (tid + nth < nblk) tri_ij(tid + nth, I1, J1);
  // eigenvector rows: thread -> (row, first pair, pair stride), fixed over the rounds; in
  // split mode the first wave takes no rows
  const bool split = nth - 64 >= n;
  const int vt = split ? tid - 64 : tid, nv = split ? nth - 64 : nth;
  const int vks = nv / n, vrow = vt >= 0 ? vt % n : 0, vk0 = (vt >= 0 && vks > 0 && vt < vks * n) ? vt / n : np2;
  if (!v_ready)
    for (int k = tid; k < n * n; k += nth) V[k] = (k % (n + 1) == 0) ? 1.0 : 0.0;
  double f2 = 0.0;
  for (int k = tid; k < npk; k += nth) {
    int i, j;
    tri_ij(k, i, j);
    const double a = (double)A[k];
    f2 += (i == j ? 1.0 : 2.0) * a * a;
  }
  const double fro2 = wg_sum(f2, red);
  const double skip = JacobiTol<T>::skip_rel * sqrt(fro2);
  const double offtol2 = JacobiTol<T>::off_rel * JacobiTol<T>::off_rel * fro2;
  int g = 0;         // rounds done; round g uses buffer g & 1
  int pending = -1;  // split mode: round whose eigenvector update is still to do
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0;  // off-diagonal mass at the start of the sweep
    for (int k = tid; k < npk; k += nth) {
      int i, j;
      tri_ij(k, i, j);
      const double a = (double)A[k];
      if (i != j) off += 2.0 * a * a;
    }
    if (wg_sum(off, red) <= offtol2) break;
    for (int r = 0; r < mm; ++r, ++g) {
      T *rc = rot + (g & 1) * 4 * np2;
      double *rdc = rotd + (g & 1) * 2 * np2;
      if (split) {
        if (tid < 64) round_rotations<T>(r, n, np2, mm, skip, A, rc, rdc, tid, 64);
        else if (pending >= 0) rotate_vectors(pending, n, np2, mm, rotd + ((g + 1) & 1) * 2 * np2, V, vrow, vk0, vks);
      } else {
        round_rotations<T>(r, n, np2, mm, skip, A, rc, rdc, tid, nth);
      }
      __syncthreads();
      if (I0 >= 0) rotate_block<T>(r, I0, J0, n, mm, A, rc);
      if (I1 >= 0) rotate_block<T>(r, I1, J1, n, mm, A, rc);
      if (split) pending = r;
      else rotate_vectors(r, n, np2, mm, rdc, V, vrow, vk0, vks);
      __syncthreads();
    }
  }
  if (pending >= 0) {  // the last round's eigenvector update
    if (tid >= 64) rotate_vectors(pending, n, np2, mm, rotd + ((g + 1) & 1) * 2 * np2, V, vrow, vk0, vks);
    __syncthreads();
  }
}

// Eigen-indices of the cheaper side: the positive eigenvalues when they are at most as many
// as the negative ones (Pi = sum_{lam > 0} lam v v^T), else the negative ones
// (Pi = X - sum_{lam < 0} lam v v^T).  sel[n] = 1 for the positive side, sel[n+1] = count.
// The first wave counts and compacts with ballots.
template <typename T>
__device__ __forceinline__ void select_side(int n, const T *A, int *sel) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    int np = 0, nneg = 0;
    for (int b = 0; b < n; b += 64) {
      const int i = b + tid;
      const T l = i < n ? A[pidx(i, i)] : T(0);
      np += __popcll(__ballot(l > T(0)));
      nneg += __popcll(__ballot(l < T(0)));
    }
    const int pos = np <= nneg;
    const unsigned long long below = (tid == 0) ? 0ull : (~0ull >> (64 - tid));
    int c = 0;
    for (int b = 0; b < n; b += 64) {
      const int i = b + tid;
      const T l = i < n ? A[pidx(i, i)] : T(0);
      const bool f = i < n && (pos ? (l > T(0)) : (l < T(0)));
      const unsigned long long m = __ballot(f);
      if (f) sel[c + __popcll(m & below)] = i;
      c += __popcll(m);
    }
    if (tid == 0) {
      sel[n] = pos;
      sel[n + 1] = c;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ inline double rebuild(int i, int j, int n, const T *A, const double *V, const int *sel, int cnt) {
  double acc = 0.0;
  for (int t = 0; t < cnt; ++t) {
    const int e = sel[t];
    acc += (double)A[pidx(e, e)] * V[i + e * n] * V[j + e * n];
  }
  return acc;
}

// ADMM step 2: S = (Pi(X_b) - X_b) * scale for the listed blocks (svec in and out), scale <= 0
// meaning 1 / sigma.  With Q != nullptr the eigenvectors of block k live at Q + qoff[k]; warm
// selects a start from them (else a cold start) and they are written back after the sweeps.
template <typename T>
__global__ void __launch_bounds__(1024) k_project_admm(const int32_t *__restrict__ blk_ids, const int64_t *__restrict__ boff,
                                                       const int32_t *__restrict__ bsz, const double *__restrict__ Xb,
                                                       double *__restrict__ S, const DevState *__restrict__ st,
                                                       double scale, double *__restrict__ Q,
                                                       const int64_t *__restrict__ qoff, int32_t warm) {
  extern __shared__ __align__(32) unsigned char smem[];
  const int32_t bk = blk_ids[blockIdx.x];
  const int n = bsz[bk];
  const int64_t off = boff[bk];
  const int nth = blockDim.x, tid = threadIdx.x;
  const int npk = n * (n + 1) / 2;
  Smem sm = carve<T>(smem, n);
  T *A = reinterpret_cast<T *>(sm.A);
  const double rs2 = 0.70710678118654752440, s2 = 1.41421356237309504880;
  double *q = Q ? Q + qoff[bk] : nullptr;
  const bool use_q = q && warm;
  if (use_q) {
    for (int k = tid; k < n * n; k += nth) sm.V[k] = q[k];
    __syncthreads();
    rotate_into_basis<T>(n, Xb + off, sm.V, q, A);
  } else {
    for (int k = tid; k < npk; k += nth) {  // svec is the packed upper triangle with sqrt(2) off-diagonal
      int i, j;
      tri_ij(k, i, j);
      const double v = Xb[off + k];
      A[k] = (T)(i == j ? v : v * rs2);
    }
    __syncthreads();
  }
  jacobi_eig<T>(n, A, sm.V, reinterpret_cast<T *>(sm.rot), sm.rotd, sm.red, use_q);
  select_side<T>(n, A, sm.sel);
  if (q)
    for (int k = tid; k < n * n; k += nth) q[k] = sm.V[k];
  const int pos = sm.sel[n], cnt = sm.sel[n + 1];
  const double mul = scale > 0.0 ? scale : 1.0 / st->sigma;
  for (int k = tid; k < npk; k += nth) {
    int i, j;
    tri_ij(k, i, j);
    const double acc = rebuild<T>(i, j, n, A, sm.V, sm.sel, cnt) * (i == j ? 1.0 : s2);
    S[off + k] = pos ? (acc - Xb[off + k]) * mul   // (Pi - X_b) * mul
                     : -acc * mul;                  // -Pi_-(X_b) * mul
  }
}

// strom_project_psd_batched: column-major blocks in T, at element offsets.
template <typename T>
__global__ void __launch_bounds__(1024) k_project_dense(int32_t nblocks, const int32_t *__restrict__ nd,
                                                        const int64_t *__restrict__ od, const T *__restrict__ in,
                                                        T *__restrict__ out, int32_t max_n, int32_t *__restrict__ err) {
  extern __shared__ __align__(32) unsigned char smem[];
  const int32_t bk = blockIdx.x;
  const int n = nd[bk];
  const int64_t off = od[bk];
  if (n <= 0 || n > max_n) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  const int nth = blockDim.x, tid = threadIdx.x;
  const int npk = n * (n + 1) / 2;
  Smem sm = carve<T>(smem, n);
  T *A = reinterpret_cast<T *>(sm.A);
  for (int k = tid; k < npk; k += nth) {
    int i, j;
    tri_ij(k, i, j);
    A[k] = in[off + i + (int64_t)j * n];
  }
  __syncthreads();
  jacobi_eig<T>(n, A, sm.V, reinterpret_cast<T *>(sm.rot), sm.rotd, sm.red, false);
  select_side<T>(n, A, sm.sel);
  const int pos = sm.sel[n], cnt = sm.sel[n + 1];
  // every thread reads only the upper entries it writes, so out may alias in
  for (int k = tid; k < npk; k += nth) {
    int i, j;
    tri_ij(k, i, j);
    const double acc = rebuild<T>(i, j, n, A, sm.V, sm.sel, cnt);
    const double x = (double)in[off + i + (int64_t)j * n];
    const T pv = (T)(pos ? acc : x - acc);
    out[off + i + (int64_t)j * n] = pv;
    if (i != j) out[off + j + (int64_t)i * n] = pv;
  }
}

size_t project_lds_bytes(int n, bool f32, int nthreads) {
  return f32 ? lds_bytes_t<float>(n, nthreads) : lds_bytes_t<double>(n, nthreads);
}

// Threads per block: 16 waves for the large blocks (latency hiding of the LDS traffic), and
// for small blocks one thread per 2x2 block and eigenvector row pair where possible.  Always
// at least 2n, so that every eigenvector row has its own threads.
int project_threads(int n) {
  if (n > 32) return 1024;
  const int np2 = (n + 1) / 2;
  const int need = np2 * (np2 + 1) / 2 > n * np2 ? np2 * (np2 + 1) / 2 : n * np2;
  int nt = 64;
  while (nt < 1024 && (nt < need / 2 || nt < 2 * n)) nt *= 2;
  return nt;
}

static bool threads_ok(int n, int nt) {
  const int np2 = (n + 1) / 2;
  return nt >= n && np2 * (np2 + 1) / 2 <= 2 * nt;
}

hipError_t launch_project_admm(hipStream_t s, bool f32, int n, int count, const int32_t *ids, const int64_t *boff,
                               const int32_t *bsz, const double *Xb, double *S, const DevState *st, double scale,
                               double *Q, const int64_t *qoff, bool warm) {
  if (count <= 0) return hipSuccess;
  const int nt = project_threads(n);
  if (!threads_ok(n, nt)) return hipErrorInvalidValue;
  const size_t lds = project_lds_bytes(n, f32, nt);
  if (f32) {
    (void)hipFuncSetAttribute((const void *)k_project_admm<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_project_admm<float>, dim3(count), dim3(nt), lds, s, ids, boff, bsz, Xb, S, st, scale, Q, qoff,
                       warm ? 1 : 0);
  } else {
    (void)hipFuncSetAttribute((const void *)k_project_admm<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_project_admm<double>, dim3(count), dim3(nt), lds, s, ids, boff, bsz, Xb, S, st, scale, Q, qoff,
                       warm ? 1 : 0);
  }
  return hipGetLastError();
}

hipError_t launch_project_dense(hipStream_t s, bool f32, int nblocks, int max_n, const int32_t *nd, const int64_t *od,
                                const void *in, void *out, int32_t *err) {
  const int nt = project_threads(max_n);
  if (!threads_ok(max_n, nt)) return hipErrorInvalidValue;
  const size_t lds = project_lds_bytes(max_n, f32, nt);
  if (f32) {
    (void)hipFuncSetAttribute((const void *)k_project_dense<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_project_dense<float>, dim3(nblocks), dim3(nt), lds, s, nblocks, nd, od, (const float *)in,
                       (float *)out, max_n, err);
  } else {
    (void)hipFuncSetAttribute((const void *)k_project_dense<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_project_dense<double>, dim3(nblocks), dim3(nt), lds, s, nblocks, nd, od, (const double *)in,
                       (double *)out, max_n, err);
  }
  return hipGetLastError();
}

}  // namespace dev
}  // namespace strom
