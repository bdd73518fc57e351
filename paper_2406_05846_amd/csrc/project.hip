// project.hip -- projection of dense symmetric blocks onto the PSD cone (the parallel PSD cone
// projection of the paper's Sec. "GPU Speedup": eigendecomposition, negative eigenvalues set
// to zero, reconstruction), one workgroup per block with the block resident in LDS.
//
// The eigensolver is the LDS-resident cyclic Jacobi of jacobi_lds.h.
//
// Warm start (ADMM step): the eigenvectors of the previous call on the same block are kept
// in HBM; the sweeps start from A = Q^T X_b Q and V = Q, which is nearly diagonal once the
// iteration settles, so a few sweeps replace the eight to ten of a cold start.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"
#include "jacobi_lds.h"

namespace strom {
namespace dev {

// A <- Q^T X Q in the block arrays Ab (position order of round 0), with Q = V (n x nn, LDS)
// and X the svec block at xs (global), as two products on the matrix cores in T: X is staged
// (packed upper triangle, unscaled off-diagonal) in the first buffer; W = X Q (n x nn) goes to
// wq, row-major, in the global eigenvector slot of the block (free until the eigenvectors are
// written back; its rows are read back coalesced); then the upper tiles of A = Q^T W are stored
// in position order, every unordered entry once.  A wave computes whole 16 x 16 tiles.
template <typename T>
__device__ __forceinline__ void rotate_into_basis(int n, const double *xs, const T *V, double *wq, T *Ab,
                                                  int nblk) {
  typedef Mfma<T> M;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;
  const int nn = n + (n & 1), np2 = nn / 2, mm = nn - 1;
  const double rs2 = 0.70710678118654752440;
  const int npk = n * (n + 1) / 2;
  T *Xs = Ab;
  for (int k = tid; k < npk; k += nth) {
    int i, j;
    tri_ij(k, i, j);
    const double v = xs[k];
    Xs[k] = (T)(i == j ? v : v * rs2);
  }
  __syncthreads();
  const int rt = (n + 15) >> 4, ct = (nn + 15) >> 4, ks = (n + 3) >> 2;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < rt * ct; t += nwaves) {  // W = X Q, tile (I, J)
    const int I = t / ct, J = t % ct;
    const int i = 16 * I + li, j = 16 * J + li;
    typename M::acc_t acc = {0, 0, 0, 0};
    for (int s = 0; s < ks; ++s) {
      const int k = 4 * s + lk;
      const T a = (i < n && k < n) ? Xs[pidx(i, k)] : T(0);
      const T b = (k < n && j < nn) ? V[j * n + k] : T(0);
      acc = M::step(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = 16 * I + M::row(lane, r);
      if (ii < n && j < nn) wq[ii * nn + j] = (double)acc[r];
    }
  }
  __threadfence_block();
  __syncthreads();
  for (int t = wave; t < ct * (ct + 1) / 2; t += nwaves) {  // A = Q^T W, upper tile (I <= J)
    int I, J;
    tri_ij(t, I, J);
    const int i = 16 * I + li, j = 16 * J + li;
    typename M::acc_t acc = {0, 0, 0, 0};
    for (int s = 0; s < ks; ++s) {
      const int k = 4 * s + lk;
      const T a = (k < n && i < nn) ? V[i * n + k] : T(0);
      const T b = (k < n && j < nn) ? (T)wq[k * nn + j] : T(0);
      acc = M::step(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = 16 * I + M::row(lane, r);
      if (ii <= j && j < nn) store_entry<T>(Ab, nblk, position0(ii, np2, mm), position0(j, np2, mm), (T)acc[r]);
    }
  }
  __syncthreads();
}

// Eigenpairs of the cheaper side: the positive eigenvalues when they are at most as many as
// the negative ones (Pi = sum_{lam > 0} lam v v^T), else the negative ones
// (Pi = X - sum_{lam < 0} lam v v^T).  Entry t: eigenvector column sel[t], eigenvalue lam[t];
// sel[nn] = 1 for the positive side, sel[nn+1] = count.  A is in the position order of round
// rfin.  The first wave counts and compacts with ballots.
template <typename T>
__device__ __forceinline__ void select_side(int nn, int nblk, const T *A, int rfin, int *sel, double *lam) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    int np = 0, nneg = 0;
    for (int b = 0; b < nn; b += 64) {
      const int x = b + tid;
      const T l = x < nn ? diag_entry(A, nblk, x) : T(0);
      np += __popcll(__ballot(l > T(0)));
      nneg += __popcll(__ballot(l < T(0)));
    }
    const int pos = np <= nneg;
    const unsigned long long below = (tid == 0) ? 0ull : (~0ull >> (64 - tid));
    int c = 0;
    for (int b = 0; b < nn; b += 64) {
      const int x = b + tid;
      const T l = x < nn ? diag_entry(A, nblk, x) : T(0);
      const bool f = x < nn && (pos ? (l > T(0)) : (l < T(0)));
      const unsigned long long m = __ballot(f);
      if (f) {
        const int t = c + __popcll(m & below);
        sel[t] = logical_index(x, rfin, nn - 1);
        lam[t] = (double)l;
      }
      c += __popcll(m);
    }
    if (tid == 0) {
      sel[nn] = pos;
      sel[nn + 1] = c;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ inline double rebuild(int i, int j, int n, const double *lam, const T *V, const int *sel, int cnt) {
  double acc = 0.0;
  for (int t = 0; t < cnt; ++t) {
    const int c = sel[t];
    acc += lam[t] * (double)V[i + c * n] * (double)V[j + c * n];
  }
  return acc;
}

// Eigenvectors V (n x nn, T) written back to q in double after one Newton-Schulz step towards
// orthogonality, q = V - V (V^T V - I) / 2.  Eigenvectors carried from one projection to the
// next drift away from orthogonal by a rounding error per iteration (float: ~1e-7 each; a
// float-era Q also reaches the double projection when the polish switches precision), and the
// warm start's Q^T X_b Q assumes Q orthogonal; one step maps a defect d to about d^2.  G - I =
// V^T V - I (upper tiles, packed) goes to Gp, the block arrays, free once the eigenvalues are
// selected; both products on the matrix cores in T, the update in double.  The dummy column of
// an odd block is zero and stays zero.
template <typename T>
__device__ __forceinline__ void store_reorthogonalized(int n, const T *V, T *Gp, double *q) {
  typedef Mfma<T> M;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6, li = lane & 15, lk = lane >> 4;
  const int nn = n + (n & 1), ct = (nn + 15) >> 4, rt = (n + 15) >> 4;
  for (int t = wave; t < ct * (ct + 1) / 2; t += nwaves) {
    int I, J;
    tri_ij(t, I, J);
    const int i = 16 * I + li, j = 16 * J + li;
    typename M::acc_t acc = {0, 0, 0, 0};
    for (int s = 0; s < (n + 3) >> 2; ++s) {
      const int k = 4 * s + lk;
      const T a = (k < n && i < nn) ? V[i * n + k] : T(0);
      const T b = (k < n && j < nn) ? V[j * n + k] : T(0);
      acc = M::step(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = 16 * I + M::row(lane, r);
      if (ii <= j && j < nn) Gp[pidx(ii, j)] = acc[r] - (ii == j ? T(1) : T(0));
    }
  }
  __syncthreads();
  for (int t = wave; t < rt * ct; t += nwaves) {
    const int I = t / ct, J = t % ct;
    const int i = 16 * I + li, j = 16 * J + li;
    typename M::acc_t acc = {0, 0, 0, 0};
    for (int s = 0; s < (nn + 3) >> 2; ++s) {
      const int k = 4 * s + lk;
      const T a = (i < n && k < nn) ? V[k * n + i] : T(0);
      const T b = (k < nn && j < nn) ? Gp[pidx(k, j)] : T(0);
      acc = M::step(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = 16 * I + M::row(lane, r);
      if (ii < n && j < nn) q[j * n + ii] = (double)V[j * n + ii] - 0.5 * (double)acc[r];
    }
  }
}

// ADMM step 2: S = (Pi(X_b) - X_b) * scale for the listed blocks (svec in and out), scale <= 0
// meaning 1 / sigma.  With Q != nullptr the eigenvectors of block k (n x nn, position order)
// live at Q + qoff[k]; bit 0 of warm selects a start from them (else a cold start), and they
// are written back after the sweeps, re-orthogonalized when bit 1 is set (the host sets it on
// the first projection of every round and on the cone projections of the sigma rule, so the
// drift of the kept eigenvectors stays at that of a round).  lds_cap: the dynamic LDS of the
// launch.
template <typename T, bool BIG>
__device__ __forceinline__ void project_block(int32_t bk, const int64_t *__restrict__ boff, const int32_t *__restrict__ bsz,
                                              const double *__restrict__ Xb, double *__restrict__ S,
                                              const DevState *__restrict__ st, double scale, double *__restrict__ Q,
                                              const int64_t *__restrict__ qoff, int32_t warm, uint32_t lds_cap,
                                              unsigned char *smem) {
  const int n = bsz[bk];
  const int nn = n + (n & 1), np2 = nn / 2, nblk = np2 * (np2 + 1) / 2;
  const int64_t off = boff[bk];
  const int nth = blockDim.x, tid = threadIdx.x;
  const int npk = n * (n + 1) / 2;
  Smem sm = carve<T>(smem, n, lds_cap);
  T *Ab = reinterpret_cast<T *>(sm.A);
  const double rs2 = 0.70710678118654752440, s2 = 1.41421356237309504880;
  double *q = Q ? Q + qoff[bk] : nullptr;
  const bool use_q = q && (warm & 1);
  T *Vt = reinterpret_cast<T *>(sm.V);
  if (use_q) {
    for (int k = tid; k < n * nn; k += nth) Vt[k] = (T)q[k];
    __syncthreads();
    rotate_into_basis<T>(n, Xb + off, Vt, q, Ab, nblk);
  } else {
    for (int e = tid; e < nn * (nn + 1) / 2; e += nth) {  // svec: packed upper triangle, sqrt(2) off-diagonal
      int x, y;
      tri_ij(e, x, y);
      const int i = logical_index(x, 0, nn - 1), j = logical_index(y, 0, nn - 1);
      const double v = (i < n && j < n) ? Xb[off + pidx(i, j)] : 0.0;
      store_entry<T>(Ab, nblk, x, y, (T)(i == j ? v : v * rs2));
    }
    __syncthreads();
  }
  int rfin = 0;
  const int cur = jacobi_eig<T, BIG>(n, Ab, sm.nbuf, Vt, reinterpret_cast<T *>(sm.rot), sm.rotd, sm.red, use_q, rfin);
  select_side<T>(nn, nblk, Ab + (size_t)cur * 4 * nblk, rfin, sm.sel, sm.lam);
  if (q) {
    if (warm & 2) store_reorthogonalized<T>(n, Vt, Ab, q);
    else
      for (int k = tid; k < n * nn; k += nth) q[k] = (double)Vt[k];
  }
  const int pos = sm.sel[nn], cnt = sm.sel[nn + 1];
  const double mul = scale > 0.0 ? scale : 1.0 / st->sigma;
  // P = U diag(lam) U^T over the selected eigenpairs (U = the columns sel of V) on the matrix
  // cores in T, upper tiles; entry (i <= j) goes to svec place j (j + 1) / 2 + i
  typedef Mfma<T> M;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6, li = lane & 15, lk = lane >> 4;
  const int rt = (n + 15) >> 4, ks = (cnt + 3) >> 2;
  for (int t = wave; t < rt * (rt + 1) / 2; t += nwaves) {
    int I, J;
    tri_ij(t, I, J);
    const int i = 16 * I + li, j = 16 * J + li;
    typename M::acc_t acc = {0, 0, 0, 0};
    for (int s = 0; s < ks; ++s) {
      const int e = 4 * s + lk;
      const int c = e < cnt ? sm.sel[e] : 0;
      const T a = (e < cnt && i < n) ? (T)(sm.lam[e] * (double)Vt[c * n + i]) : T(0);
      const T b = (e < cnt && j < n) ? Vt[c * n + j] : T(0);
      acc = M::step(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = 16 * I + M::row(lane, r);
      if (ii <= j && j < n) {
        const int64_t k = off + (int64_t)j * (j + 1) / 2 + ii;
        const double p = (double)acc[r] * (ii == j ? 1.0 : s2);
        S[k] = pos ? (p - Xb[k]) * mul   // (Pi - X_b) * mul
                   : -p * mul;           // -Pi_-(X_b) * mul
      }
    }
  }
}

template <typename T, bool BIG>
__global__ void __launch_bounds__(1024) k_project_admm(const int32_t *__restrict__ blk_ids, const int64_t *__restrict__ boff,
                                                       const int32_t *__restrict__ bsz, const double *__restrict__ Xb,
                                                       double *__restrict__ S, const DevState *__restrict__ st,
                                                       double scale, double *__restrict__ Q,
                                                       const int64_t *__restrict__ qoff, int32_t warm, uint32_t lds_cap) {
  extern __shared__ __align__(32) unsigned char smem[];
  project_block<T, BIG>(blk_ids[blockIdx.x], boff, bsz, Xb, S, st, scale, Q, qoff, warm, lds_cap, smem);
}

// The same over a batch: item = (instance, block); instances that are retired or whose
// projection precision is not T are skipped.  cone = 0: X_b -> S with 1 / sigma; cone = 1:
// X -> X_b with scale 1, for the instances that apply the sigma rule this round.
template <typename T, bool BIG>
__global__ void __launch_bounds__(1024) k_project_batch(const BatchItem *__restrict__ items,
                                                        const BatchInst *__restrict__ bi, int32_t cone,
                                                        int32_t reorth, uint32_t lds_cap) {
  extern __shared__ __align__(32) unsigned char smem[];
  const BatchItem it = items[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active || I.f32 != (sizeof(T) == sizeof(float) ? 1 : 0) || (cone && !I.sig)) return;
  const double *in = G(cone ? I.X : I.Xb);
  double *out = G(cone ? I.Xb : I.S);
  project_block<T, BIG>(it.idx, G(I.boff), G(I.bsz), in, out, G(I.st), cone ? 1.0 : 0.0, G(I.Q), G(I.qoff),
                        (I.warm ? 1 : 0) | (cone || reorth ? 2 : 0), lds_cap, smem);
}

// strom_project_psd_batched: column-major blocks in T, at element offsets.
template <typename T, bool BIG>
__global__ void __launch_bounds__(1024) k_project_dense(int32_t nblocks, const int32_t *__restrict__ nd,
                                                        const int64_t *__restrict__ od, const T *__restrict__ in,
                                                        T *__restrict__ out, int32_t max_n, int32_t *__restrict__ err,
                                                        uint32_t lds_cap) {
  extern __shared__ __align__(32) unsigned char smem[];
  const int32_t bk = blockIdx.x;
  const int n = nd[bk];
  const int64_t off = od[bk];
  if (n <= 0 || n > max_n) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  const int nn = n + (n & 1), np2 = nn / 2, nblk = np2 * (np2 + 1) / 2;
  const int nth = blockDim.x, tid = threadIdx.x;
  const int npk = n * (n + 1) / 2;
  Smem sm = carve<T>(smem, n, lds_cap);
  T *Ab = reinterpret_cast<T *>(sm.A);
  for (int e = tid; e < nn * (nn + 1) / 2; e += nth) {
    int x, y;
    tri_ij(e, x, y);
    const int i = logical_index(x, 0, nn - 1), j = logical_index(y, 0, nn - 1);
    store_entry<T>(Ab, nblk, x, y, (i < n && j < n) ? in[off + i + (int64_t)j * n] : T(0));
  }
  __syncthreads();
  int rfin = 0;
  T *Vt = reinterpret_cast<T *>(sm.V);
  const int cur = jacobi_eig<T, BIG>(n, Ab, sm.nbuf, Vt, reinterpret_cast<T *>(sm.rot), sm.rotd, sm.red, false, rfin);
  select_side<T>(nn, nblk, Ab + (size_t)cur * 4 * nblk, rfin, sm.sel, sm.lam);
  const int pos = sm.sel[nn], cnt = sm.sel[nn + 1];
  // every thread reads only the upper entries it writes, so out may alias in
  for (int k = tid; k < npk; k += nth) {
    int i, j;
    tri_ij(k, i, j);
    const double acc = rebuild<T>(i, j, n, sm.lam, Vt, sm.sel, cnt);
    const double x = (double)in[off + i + (int64_t)j * n];
    const T pv = (T)(pos ? acc : x - acc);
    out[off + i + (int64_t)j * n] = pv;
    if (i != j) out[off + j + (int64_t)i * n] = pv;
  }
}

// strom_eig_batched: eigenvalues of every block in ascending order (ties by index) at
// w + woff[k], and with WANT_V the eigenvectors as the columns of an n x n column-major block at
// v + od[k] (column j for eigenvalue j).  Without WANT_V the eigenvector work is skipped.
template <typename T, bool BIG, bool WANT_V>
__global__ void __launch_bounds__(1024) k_eig_dense(int32_t nblocks, const int32_t *__restrict__ nd,
                                                    const int64_t *__restrict__ od, const T *__restrict__ in,
                                                    const int64_t *__restrict__ woff, T *__restrict__ w,
                                                    T *__restrict__ v, int32_t max_n, int32_t *__restrict__ err,
                                                    uint32_t lds_cap) {
  extern __shared__ __align__(32) unsigned char smem[];
  const int32_t bk = blockIdx.x;
  const int n = nd[bk];
  const int64_t off = od[bk];
  if (n <= 0 || n > max_n) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  const int nn = n + (n & 1), np2 = nn / 2, nblk = np2 * (np2 + 1) / 2, mm = nn - 1;
  const int nth = blockDim.x, tid = threadIdx.x;
  Smem sm = carve<T>(smem, n, lds_cap);
  T *Ab = reinterpret_cast<T *>(sm.A);
  for (int e = tid; e < nn * (nn + 1) / 2; e += nth) {
    int x, y;
    tri_ij(e, x, y);
    const int i = logical_index(x, 0, mm), j = logical_index(y, 0, mm);
    store_entry<T>(Ab, nblk, x, y, (i < n && j < n) ? in[off + i + (int64_t)j * n] : T(0));
  }
  __syncthreads();
  int rfin = 0;
  T *Vt = reinterpret_cast<T *>(sm.V);
  const int cur = jacobi_eig<T, BIG, WANT_V>(n, Ab, sm.nbuf, Vt, reinterpret_cast<T *>(sm.rot), sm.rotd, sm.red,
                                             false, rfin);
  const T *A = Ab + (size_t)cur * 4 * nblk;
  for (int x = tid; x < nn; x += nth) sm.lam[logical_index(x, rfin, mm)] = (double)diag_entry(A, nblk, x);
  __syncthreads();
  for (int i = tid; i < n; i += nth) {  // the rank of eigenvalue i among the n real ones
    const double li = sm.lam[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = sm.lam[j];
      rank += (lj < li || (lj == li && j < i)) ? 1 : 0;
    }
    w[woff[bk] + rank] = (T)li;
    sm.sel[i] = rank;
  }
  if constexpr (WANT_V) {
    __syncthreads();
    for (int e = tid; e < n * n; e += nth) {
      const int r = e % n, i = e / n;
      v[off + r + (int64_t)sm.sel[i] * n] = Vt[i * n + r];
    }
  }
}

// Dense n x n column-major copies (both triangles) of listed svec blocks: block ids[k] of the
// svec vector at boff, into out + od[k].
__global__ void __launch_bounds__(256) k_unpack_svec(const int32_t *__restrict__ ids, const int64_t *__restrict__ boff,
                                                     const int32_t *__restrict__ bsz, const double *__restrict__ sv,
                                                     const int64_t *__restrict__ od, double *__restrict__ out) {
  const int32_t bk = ids[blockIdx.x];
  const int n = bsz[bk];
  const double rs2 = 0.70710678118654752440;
  const double *src = sv + boff[bk];
  double *dst = out + od[blockIdx.x];
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;
    const double x = src[pidx(i, j)];
    dst[e] = i == j ? x : x * rs2;
  }
}

size_t project_lds_bytes(int n, bool f32, int nthreads) {
  (void)nthreads;
  return lds_bytes_for(n, f32 ? sizeof(float) : sizeof(double));
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

// The kernels assume: every 2x2 block has a worker thread (at most two per thread), every
// eigenvector row has one and no worker holds more than big_vs eigenvector slots; then the
// same holds for every smaller block of a merged launch.  big: the launch needs the variant
// with two blocks and big_vs slots per thread.
static bool threads_ok(int n, int nt, bool f32, bool &big) {
  const int nn = n + (n & 1), np2 = nn / 2, nblk = np2 * (np2 + 1) / 2;
  const int nw = nt - 64 >= n ? nt - 64 : nt;  // block workers (the first wave computes parameters)
  if (nw < n || nblk > 2 * nw) return false;
  const int vks = nw / n, slots = (np2 + vks - 1) / vks;
  big = nblk > nw || slots > kSmallVs;
  return slots <= big_vs(f32);
}

template <typename T, bool BIG>
static void launch_admm_t(hipStream_t s, int count, int nt, size_t lds, const int32_t *ids, const int64_t *boff,
                          const int32_t *bsz, const double *Xb, double *S, const DevState *st, double scale, double *Q,
                          const int64_t *qoff, bool warm, bool reorth) {
  (void)hipFuncSetAttribute((const void *)k_project_admm<T, BIG>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_project_admm<T, BIG>), dim3(count), dim3(nt), lds, s, ids, boff, bsz, Xb, S, st, scale, Q, qoff,
                     (warm ? 1 : 0) | (reorth ? 2 : 0), (uint32_t)lds);
}

hipError_t launch_project_admm(hipStream_t s, bool f32, int n, int count, const int32_t *ids, const int64_t *boff,
                               const int32_t *bsz, const double *Xb, double *S, const DevState *st, double scale,
                               double *Q, const int64_t *qoff, bool warm, bool reorth) {
  if (count <= 0) return hipSuccess;
  const int nt = project_threads(n);
  const size_t lds = project_lds_bytes(n, f32, nt);
  bool big = false;
  if (!threads_ok(n, nt, f32, big) || lds > kLdsCap) return hipErrorInvalidValue;
  if (f32) {
    if (big) launch_admm_t<float, true>(s, count, nt, lds, ids, boff, bsz, Xb, S, st, scale, Q, qoff, warm, reorth);
    else launch_admm_t<float, false>(s, count, nt, lds, ids, boff, bsz, Xb, S, st, scale, Q, qoff, warm, reorth);
  } else {
    if (big) launch_admm_t<double, true>(s, count, nt, lds, ids, boff, bsz, Xb, S, st, scale, Q, qoff, warm, reorth);
    else launch_admm_t<double, false>(s, count, nt, lds, ids, boff, bsz, Xb, S, st, scale, Q, qoff, warm, reorth);
  }
  return hipGetLastError();
}

template <typename T, bool BIG>
static void launch_batch_t(hipStream_t s, int count, int nt, size_t lds, const BatchItem *items, const BatchInst *bi,
                           int cone, int reorth) {
  (void)hipFuncSetAttribute((const void *)k_project_batch<T, BIG>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_project_batch<T, BIG>), dim3(count), dim3(nt), lds, s, items, bi, cone, reorth, (uint32_t)lds);
}

hipError_t launch_project_batch(hipStream_t s, bool f32, int n, int nt, int count, const BatchItem *items,
                                const BatchInst *bi, int cone, bool reorth) {
  if (count <= 0) return hipSuccess;
  const size_t lds = project_lds_bytes(n, f32, nt);
  bool big = false;
  if (!threads_ok(n, nt, f32, big) || lds > kLdsCap) return hipErrorInvalidValue;
  if (f32) {
    if (big) launch_batch_t<float, true>(s, count, nt, lds, items, bi, cone, reorth ? 1 : 0);
    else launch_batch_t<float, false>(s, count, nt, lds, items, bi, cone, reorth ? 1 : 0);
  } else {
    if (big) launch_batch_t<double, true>(s, count, nt, lds, items, bi, cone, reorth ? 1 : 0);
    else launch_batch_t<double, false>(s, count, nt, lds, items, bi, cone, reorth ? 1 : 0);
  }
  return hipGetLastError();
}

bool project_fits(int n, bool f32, size_t lds_cap) {
  if (n <= 0) return false;
  const int nt = project_threads(n);
  bool big = false;
  const size_t lds = project_lds_bytes(n, f32, nt);
  return threads_ok(n, nt, f32, big) && lds <= kLdsCap && lds <= lds_cap;
}

int project_thread_options(int n, bool f32, int *out) {
  int k = 0;
  for (int nt = 64; nt <= 1024; nt *= 2) {
    bool big = false;
    if (threads_ok(n, nt, f32, big)) out[k++] = nt;
  }
  return k;
}

template <typename T, bool BIG>
static void launch_dense_t(hipStream_t s, int nblocks, int nt, size_t lds, int max_n, const int32_t *nd,
                           const int64_t *od, const void *in, void *out, int32_t *err) {
  (void)hipFuncSetAttribute((const void *)k_project_dense<T, BIG>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_project_dense<T, BIG>), dim3(nblocks), dim3(nt), lds, s, nblocks, nd, od, (const T *)in,
                     (T *)out, max_n, err, (uint32_t)lds);
}

hipError_t launch_project_dense(hipStream_t s, bool f32, int nblocks, int max_n, const int32_t *nd, const int64_t *od,
                                const void *in, void *out, int32_t *err) {
  const int nt = project_threads(max_n);
  const size_t lds = project_lds_bytes(max_n, f32, nt);
  bool big = false;
  if (!threads_ok(max_n, nt, f32, big) || lds > kLdsCap) return hipErrorInvalidValue;
  if (f32) {
    if (big) launch_dense_t<float, true>(s, nblocks, nt, lds, max_n, nd, od, in, out, err);
    else launch_dense_t<float, false>(s, nblocks, nt, lds, max_n, nd, od, in, out, err);
  } else {
    if (big) launch_dense_t<double, true>(s, nblocks, nt, lds, max_n, nd, od, in, out, err);
    else launch_dense_t<double, false>(s, nblocks, nt, lds, max_n, nd, od, in, out, err);
  }
  return hipGetLastError();
}

template <typename T, bool BIG, bool WANT_V>
static void launch_eig_t(hipStream_t s, int nblocks, int nt, size_t lds, int max_n, const int32_t *nd,
                         const int64_t *od, const void *in, const int64_t *woff, void *w, void *v, int32_t *err) {
  (void)hipFuncSetAttribute((const void *)k_eig_dense<T, BIG, WANT_V>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL((k_eig_dense<T, BIG, WANT_V>), dim3(nblocks), dim3(nt), lds, s, nblocks, nd, od, (const T *)in,
                     woff, (T *)w, (T *)v, max_n, err, (uint32_t)lds);
}

template <typename T>
static void launch_eig_v(bool big, bool want_v, hipStream_t s, int nblocks, int nt, size_t lds, int max_n,
                         const int32_t *nd, const int64_t *od, const void *in, const int64_t *woff, void *w, void *v,
                         int32_t *err) {
  if (big) {
    if (want_v) launch_eig_t<T, true, true>(s, nblocks, nt, lds, max_n, nd, od, in, woff, w, v, err);
    else launch_eig_t<T, true, false>(s, nblocks, nt, lds, max_n, nd, od, in, woff, w, v, err);
  } else {
    if (want_v) launch_eig_t<T, false, true>(s, nblocks, nt, lds, max_n, nd, od, in, woff, w, v, err);
    else launch_eig_t<T, false, false>(s, nblocks, nt, lds, max_n, nd, od, in, woff, w, v, err);
  }
}

hipError_t launch_eig_dense(hipStream_t s, bool f32, int nblocks, int max_n, const int32_t *nd, const int64_t *od,
                            const void *in, const int64_t *woff, void *w, void *v, int32_t *err) {
  const int nt = project_threads(max_n);
  const size_t lds = project_lds_bytes(max_n, f32, nt);
  bool big = false;
  if (!threads_ok(max_n, nt, f32, big) || lds > kLdsCap) return hipErrorInvalidValue;
  if (f32) launch_eig_v<float>(big, v != nullptr, s, nblocks, nt, lds, max_n, nd, od, in, woff, w, v, err);
  else launch_eig_v<double>(big, v != nullptr, s, nblocks, nt, lds, max_n, nd, od, in, woff, w, v, err);
  return hipGetLastError();
}

hipError_t launch_unpack_svec(hipStream_t s, int count, const int32_t *ids, const int64_t *boff, const int32_t *bsz,
                              const double *sv, const int64_t *od, double *out) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_svec, dim3(count), dim3(256), 0, s, ids, boff, bsz, sv, od, out);
  return hipGetLastError();
}

}  // namespace dev
}  // namespace strom
