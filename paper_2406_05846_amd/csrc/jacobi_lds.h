// jacobi_lds.h -- the one-workgroup eigensolver shared by the projection kernels: cyclic Jacobi
// on a symmetric block held in LDS, with the LDS layout, reductions and matrix-core step it uses.
//
// Eigensolver: cyclic Jacobi in the round-robin (circle) parallel ordering.  A block of size n
// is padded to an even size nn with a zero dummy index when n is odd (its rotations are the
// identity, so it stays zero and its eigenvalue is 0).  The matrix is kept in *position*
// order: in every round the rotations pair positions (2k, 2k + 1) -- slot k -- and after the
// round the data moves by the circle permutation pos_next, which is the same in every round.
// So a thread rotates the same 2x2 block (slot I x slot J) at the same LDS addresses in every
// round and writes its four results to fixed, precomputed places: there is no index
// arithmetic per round.  The 2x2 blocks of the upper triangle are stored as four arrays (entry
// (p,p), (p,q), (q,p), (q,q) of every block), so the loads of a wave are contiguous.  The
// eigenvectors stay in logical order (column i belongs to index i; position x holds index
// logical_index(x, r) in round r), rotated in place one round late while the first wave
// computes the next rotation parameters.  Rotation
// parameters are computed in double for both storage types; the matrix and the eigenvectors
// are held in T (double, or float for the reduced-precision form), norms in double; the
// products (warm start, reconstruction) run on the matrix cores in T.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

namespace strom {
namespace dev {

constexpr size_t kLdsCap = 160 * 1024;  // LDS of one workgroup on gfx950
// Eigenvector slots per worker thread (their column offsets stay in registers): at most
// kSmallVs in the one-block-per-thread variant, big_vs in the other (checked at launch).
constexpr int kSmallVs = 5;
__host__ __device__ constexpr int big_vs(bool f32) { return f32 ? 10 : 8; }

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

// Position of the data at position x after one round of the circle ordering over np2 slots:
// the first halves of the slots move down one slot, the second halves up one slot, with the
// turns at both ends; the second half of slot 0 stays.
__host__ __device__ inline int pos_next(int x, int np2) {
  if (np2 == 1) return x;
  const int k = x >> 1;
  if ((x & 1) == 0) return k >= 1 ? x - 2 : 3;
  if (k == 0) return 1;
  return k < np2 - 1 ? x + 2 : x - 1;
}

// The inverse: the position whose data moves to position x in one round.
__device__ inline int pos_prev(int x, int np2) {
  if (np2 == 1) return x;
  const int k = x >> 1;
  if ((x & 1) == 0) return k < np2 - 1 ? x + 2 : x + 1;
  if (k == 0) return 1;
  return k >= 2 ? x - 2 : 0;
}

__device__ inline int bidx(int I, int J) { return J * (J + 1) / 2 + I; }  // block (I <= J)

// Index held by position x in round r (0 <= r < mm = nn - 1) of the circle ordering: slot k
// pairs indices (r + k, r - k) mod mm, slot 0 pairs (r, mm).  In round 0, position x holds
// index logical_index(x, 0); the dummy index of an odd block (mm) stays at position 1.
__device__ inline int logical_index(int x, int r, int mm) {
  const int k = x >> 1;
  if ((x & 1) == 0) {
    const int i = r + k;
    return i >= mm ? i - mm : i;
  }
  if (k == 0) return mm;
  const int i = r - k;
  return i < 0 ? i + mm : i;
}

template <typename T>
struct JacobiTol;
template <>
struct JacobiTol<double> {
  static constexpr double off_rel = 1e-11;   // stop when off(A) <= off_rel * ||A||_F
  static constexpr double skip_rel = 1e-18;  // no rotation for |a_pq| <= skip_rel * ||A||_F
};
template <>
struct JacobiTol<float> {
  static constexpr double off_rel = 1e-6;
  static constexpr double skip_rel = 1e-9;
};

// One 16 x 16 x 4 matrix-core step, acc += A B, per element type: FP64 operands with FP64
// accumulation, FP32 operands with FP32 accumulation.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; it receives column l % 16 of the 16 x 16 result, register r holding row
// row(l, r) (the two instructions order their result rows differently).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef mfma_d4 acc_t;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Mfma<float> {
  typedef mfma_f4 acc_t;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Position of logical index i in round 0 of the circle ordering (inverse of logical_index(., 0)):
// indices below np2 sit at the even positions, index mm at position 1, the others at odd ones.
__device__ inline int position0(int i, int np2, int mm) {
  if (i < np2) return 2 * i;
  if (i == mm) return 1;
  return 2 * (mm - i) + 1;
}

// LDS: V (n x nn of T, column-major, column = index) | red (16 doubles) | rotd (two
//      buffers of (c, s) doubles per slot) | A (nbuf buffers of four arrays of nblk T) | rot
//      (two buffers of (c, s, new a_pp, new a_qq) T per slot) | lam (nn doubles) | sel (nn + 4 ints), every
//      region 32-byte aligned.  nbuf = 2 (a round writes the other buffer) when that fits,
//      else 1 (one more barrier per round).
struct Layout {
  size_t red, rotd, A, rot, lam, sel, total;
};

__host__ __device__ inline size_t align32(size_t x) { return (x + 31) & ~(size_t)31; }

__host__ __device__ inline Layout lds_layout(int n, size_t tsize, int nbuf) {
  const size_t nn = (size_t)n + (n & 1), np2 = nn / 2, nblk = np2 * (np2 + 1) / 2;
  Layout L;
  L.red = align32(tsize * (size_t)n * nn);
  L.rotd = align32(L.red + 8 * 16);
  L.A = align32(L.rotd + 2 * 16 * np2);
  L.rot = align32(L.A + (size_t)nbuf * 4 * tsize * nblk);
  L.lam = align32(L.rot + 2 * 4 * tsize * np2);
  L.sel = align32(L.lam + 8 * nn);
  L.total = align32(L.sel + 4 * (nn + 4));
  return L;
}

// LDS of a launch whose largest block has size n: double-buffered if that fits.
inline size_t lds_bytes_for(int n, size_t tsize) {
  const size_t two = lds_layout(n, tsize, 2).total;
  return two <= kLdsCap ? two : lds_layout(n, tsize, 1).total;
}

struct Smem {
  void *V;  // n x nn of the launch's element type
  double *red, *rotd, *lam;
  void *A, *rot;
  int *sel;
  int nbuf;
};

template <typename T>
__device__ inline Smem carve(unsigned char *base, int n, size_t lds_cap) {
  const int nbuf = lds_layout(n, sizeof(T), 2).total <= lds_cap ? 2 : 1;
  const Layout L = lds_layout(n, sizeof(T), nbuf);
  Smem s;
  s.V = base;
  s.red = reinterpret_cast<double *>(base + L.red);
  s.rotd = reinterpret_cast<double *>(base + L.rotd);
  s.A = base + L.A;
  s.rot = base + L.rot;
  s.lam = reinterpret_cast<double *>(base + L.lam);
  s.sel = reinterpret_cast<int *>(base + L.sel);
  s.nbuf = nbuf;
  return s;
}

// Sum over the workgroup in a fixed order (wave sums, then the waves in turn).
__device__ inline double wg_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int nw = blockDim.x >> 6;
  __syncthreads();  // red may still be read by the previous call
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nw; ++w) r += red[w];
  return r;
}

// Entry (x, y) of the position-ordered matrix into the block arrays Ab (nblk blocks each).
template <typename T>
__device__ inline void store_entry(T *Ab, int nblk, int x, int y, T v) {
  if (x > y) { const int t = x; x = y; y = t; }
  const int b = bidx(x >> 1, y >> 1);
  Ab[(((x & 1) << 1) | (y & 1)) * nblk + b] = v;
  if ((x >> 1) == (y >> 1) && x != y) Ab[2 * nblk + b] = v;  // (q,p) of a diagonal block
}

template <typename T>
__device__ inline T diag_entry(const T *Ab, int nblk, int x) {
  const int k = x >> 1;
  return Ab[((x & 1) ? 3 : 0) * nblk + bidx(k, k)];
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

// Places of the entries of block (I, J) after one round: index into the block arrays
// (array * nblk + block) of entry h = (p,p), (p,q), (q,p), (q,q), and bit h of *twice when the
// entry lands off the diagonal of a diagonal block, where it is stored twice: as (p,q) at d[h]
// and as (q,p) at d[h] + nblk.  A diagonal block carries its (p,q) entry once: its (q,p)
// entry gets no place (-1).
__device__ inline void block_dests(int I, int J, int np2, int nblk, int *d, int *twice) {
  *twice = 0;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    d[h] = -1;
    if (I < 0 || (I == J && h == 2)) continue;
    int x = pos_next(2 * I + (h >> 1), np2), y = pos_next(2 * J + (h & 1), np2);
    if (x > y) { const int t = x; x = y; y = t; }
    const int b = bidx(x >> 1, y >> 1);
    d[h] = (((x & 1) << 1) | (y & 1)) * nblk + b;
    if ((x >> 1) == (y >> 1) && x != y) *twice |= 1 << h;
  }
}

// J_I^T [a b; c d] J_J for the rotations (c1, s1) of slot I and (c2, s2) of slot J.  The block
// rotations and the look-ahead of the next rotation parameters both use this, so they agree
// to the bit.
template <typename T>
__device__ __forceinline__ void rotate_entries(T a, T bq, T cq, T d, T c1, T s1, T c2, T s2, T *o) {
  const T ra = c1 * a - s1 * cq, rb = c1 * bq - s1 * d;  // rows p1, q1 rotated
  const T rc = s1 * a + c1 * cq, rd = s1 * bq + c1 * d;
  o[0] = c2 * ra - s2 * rb;  // then columns p2, q2
  o[1] = s2 * ra + c2 * rb;
  o[2] = c2 * rc - s2 * rd;
  o[3] = s2 * rc + c2 * rd;
}

// New entries of block b = (I, J) for the rotations of the current round: rot (c, s, new a_pp,
// new a_qq in T per slot) and rotd (c, s in double per slot).  In double, (c, s) are read from
// rotd: 16-byte records at consecutive slots, where the 32-byte records of rot would make every
// wide LDS read of a wave a two-way bank conflict.  In float, rot's records are 16 bytes.
template <typename T>
__device__ __forceinline__ void rotate_block(int b, int I, int J, int nblk, const T *A, const T *rot,
                                             const double *rotd, T *o) {
  typedef typename Vec4<T>::type V4;
  if (I == J) {
    const V4 ri = reinterpret_cast<const V4 *>(rot)[I];
    o[0] = ri.z;
    o[1] = T(0);
    o[2] = T(0);
    o[3] = ri.w;
    return;
  }
  T c1, s1, c2, s2;
  if constexpr (sizeof(T) == sizeof(double)) {
    const double2 ri = reinterpret_cast<const double2 *>(rotd)[I], rj = reinterpret_cast<const double2 *>(rotd)[J];
    c1 = ri.x; s1 = ri.y; c2 = rj.x; s2 = rj.y;
  } else {
    const V4 ri = reinterpret_cast<const V4 *>(rot)[I], rj = reinterpret_cast<const V4 *>(rot)[J];
    c1 = ri.x; s1 = ri.y; c2 = rj.x; s2 = rj.y;
  }
  rotate_entries<T>(A[b], A[nblk + b], A[2 * nblk + b], A[3 * nblk + b], c1, s1, c2, s2, o);
}

template <typename T>
__device__ __forceinline__ void store_block(T *An, int nblk, const int *d, int twice, const T *o) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    if (d[h] >= 0) An[d[h]] = o[h];
    if (twice & (1 << h)) An[d[h] + nblk] = o[h];
  }
}

// Rotation of one slot that annihilates apq of the 2x2 block [app apq; apq aqq]: (c, s) and the
// new diagonal, written to rot (T) and rotd (double).
template <typename T>
__device__ __forceinline__ void slot_rotation(int k, double app, double aqq, double apq, double skip, T *rot,
                                              double *rotd) {
  double c = 1.0, s = 0.0, dp = app, dq = aqq;
  if (fabs(apq) > skip) {
    const double theta = (aqq - app) / (2.0 * apq);
    const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    c = 1.0 / sqrt(t * t + 1.0);
    s = t * c;
    dp = app - t * apq;
    dq = aqq + t * apq;
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

// Rotation parameters of every slot from the diagonal blocks of A (threads t0, t0 + stride, ...).
template <typename T>
__device__ __forceinline__ void round_rotations(int np2, int nblk, double skip, const T *A, T *rot, double *rotd,
                                                int t0, int stride) {
  for (int k = t0; k < np2; k += stride) {
    const int bd = bidx(k, k);
    slot_rotation<T>(k, (double)A[bd], (double)A[3 * nblk + bd], (double)A[nblk + bd], skip, rot, rotd);
  }
}

// Look-ahead: the rotation parameters of the next round, from A and the rotations rc of the
// current round, without waiting for the block rotations.  In the next round slot k holds the
// data of positions x = pos_prev(2k) and y = pos_prev(2k + 1) of this round; its diagonal
// entries are new diagonal entries of this round's slots (rc .z / .w) and its off-diagonal
// entry is one entry of the rotated block (slot(x), slot(y)).
template <typename T>
__device__ __forceinline__ void next_rotations(int np2, int nblk, double skip, const T *A, const T *rc, T *rn,
                                               double *rdn, int t0, int stride) {
  typedef typename Vec4<T>::type V4;
  for (int k = t0; k < np2; k += stride) {
    const int x = pos_prev(2 * k, np2), y = pos_prev(2 * k + 1, np2);
    const int sx = x >> 1, sy = y >> 1;
    const V4 px = reinterpret_cast<const V4 *>(rc)[sx], py = reinterpret_cast<const V4 *>(rc)[sy];
    const double app = (double)((x & 1) ? px.w : px.z), aqq = (double)((y & 1) ? py.w : py.z);
    double apq = 0.0;  // x, y in one slot: the entry the rotation of this round annihilates
    if (sx != sy) {
      const bool tr = sx > sy;
      const int I = tr ? sy : sx, J = tr ? sx : sy;
      const int h = tr ? (((y & 1) << 1) | (x & 1)) : (((x & 1) << 1) | (y & 1));
      const int b = bidx(I, J);
      const V4 ri = tr ? py : px, rj = tr ? px : py;
      T o[4];
      rotate_entries<T>(A[b], A[nblk + b], A[2 * nblk + b], A[3 * nblk + b], ri.x, ri.y, rj.x, rj.y, o);
      apq = (double)o[h];
    }
    slot_rotation<T>(k, app, aqq, apq, skip, rn, rdn);
  }
}

// Off-diagonal mass (and with the diagonal: squared Frobenius norm) of block b = (I, J).
template <typename T>
__device__ inline double block_mass(const T *A, int nblk, int b, int I, int J, bool with_diag) {
  const double a = (double)A[b], bq = (double)A[nblk + b], cq = (double)A[2 * nblk + b], d = (double)A[3 * nblk + b];
  if (I == J) return 2.0 * bq * bq + (with_diag ? a * a + d * d : 0.0);
  return 2.0 * (a * a + bq * bq + cq * cq + d * d);
}

// Cyclic Jacobi on the block arrays (buffer 0 on entry, position order of round 0).  Returns
// the buffer holding the final matrix; rfin = the round (mod mm) whose position order it is in,
// *rounds (when given) = the rounds run, 0 when the block was already diagonal to Tol.  At most
// max_sweeps sweeps.
// A round is one phase and one barrier: the first wave computes the next round's rotation
// parameters (look-ahead) while the other threads rotate the eigenvector pairs in place and the
// 2x2 blocks, storing them to their permuted places (in the other buffer; single-buffered, the
// stores wait for one more barrier).  With few threads (no split) every thread does all three.
template <typename T, bool BIG, bool WANT_V = true, class Tol = JacobiTol<T>>
__device__ __forceinline__ int jacobi_eig(int n, T *Ab, int nbuf, T *V, T *rot, double *rotd, double *red,
                                          bool v_ready, int &rfin, int *rounds = nullptr, int max_sweeps = 40) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nn = n + (n & 1), np2 = nn / 2, mm = nn - 1;
  const int nblk = np2 * (np2 + 1) / 2;
  const bool split = nth - 64 >= n;
  const int wt = split ? tid - 64 : tid, nw = split ? nth - 64 : nth;  // block and eigenvector workers
  // this thread's 2x2 blocks (at most nw, or 2 nw when BIG: checked at launch) and their places
  // after a round, fixed over the rounds
  int I0 = -1, J0 = -1, I1 = -1, J1 = -1;
  if (wt >= 0 && wt < nblk) tri_ij(wt, I0, J0);
  if (BIG && wt >= 0 && wt + nw < nblk) tri_ij(wt + nw, I1, J1);
  const int b0 = wt, b1 = wt + nw;
  int d0[4], d1[4], tw0 = 0, tw1 = 0;
  block_dests(I0, J0, np2, nblk, d0, &tw0);
  if constexpr (BIG) block_dests(I1, J1, np2, nblk, d1, &tw1);
  // eigenvector slots: worker -> (row, first slot, slot stride); the offsets of the two
  // columns of each slot (index * n) advance by one column per round, wrapping at mm, except
  // the fixed second index of slot 0
  constexpr int kMaxVs = BIG ? big_vs(sizeof(T) == 4) : kSmallVs;
  const int vks = nw / n, vrow = wt >= 0 ? wt % n : 0;
  const int vk0 = (wt >= 0 && vks > 0 && wt < vks * n) ? wt / n : np2;
  const int vwrap = mm * n;
  int vcp[kMaxVs], vcq[kMaxVs];
#pragma unroll
  for (int j = 0; j < kMaxVs; ++j) {
    const int k = vk0 + j * vks;
    vcp[j] = k < np2 ? logical_index(2 * k, 0, mm) * n : 0;
    vcq[j] = k < np2 ? logical_index(2 * k + 1, 0, mm) * n : 0;
  }
  if (WANT_V && !v_ready)
    for (int k = tid; k < n * nn; k += nth) V[k] = (k % (n + 1) == 0 && k / n < n) ? T(1) : T(0);
  double f2 = 0.0;
  if (I0 >= 0) f2 += block_mass<T>(Ab, nblk, b0, I0, J0, true);
  if (BIG && I1 >= 0) f2 += block_mass<T>(Ab, nblk, b1, I1, J1, true);
  const double fro2 = wg_sum(f2, red);
  const double skip = Tol::skip_rel * sqrt(fro2);
  const double offtol2 = Tol::off_rel * Tol::off_rel * fro2;
  // parameters of the first round; then round g uses buffer g & 1 and writes (g + 1) & 1
  round_rotations<T>(np2, nblk, skip, Ab, rot, rotd, tid, nth);
  int cur = 0, g = 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    const T *Ac = Ab + (size_t)cur * 4 * nblk;
    double off = 0.0;  // off-diagonal mass at the start of the sweep
    if (I0 >= 0) off += block_mass<T>(Ac, nblk, b0, I0, J0, false);
    if (BIG && I1 >= 0) off += block_mass<T>(Ac, nblk, b1, I1, J1, false);
    if (wg_sum(off, red) <= offtol2) break;  // (the barriers inside also publish the parameters)
    for (int r = 0; r < mm; ++r, ++g) {
      T *A = Ab + (size_t)cur * 4 * nblk;
      T *An = nbuf == 2 ? Ab + (size_t)(cur ^ 1) * 4 * nblk : A;
      const T *rc = rot + (g & 1) * 4 * np2;
      const double *rdc = rotd + (g & 1) * 2 * np2;
      if (!split || tid < 64)
        next_rotations<T>(np2, nblk, skip, A, rc, rot + ((g + 1) & 1) * 4 * np2, rotd + ((g + 1) & 1) * 2 * np2, tid,
                          split ? 64 : nth);
      if (WANT_V && wt >= 0) {
#pragma unroll
        for (int j = 0; j < kMaxVs; ++j) {  // eigenvector columns of slot k, in place
          const int k = vk0 + j * vks;
          if (k < np2) {
            T c, sn;  // (c, s) of slot k: from the double records, or the T records in float
            if constexpr (sizeof(T) == sizeof(double)) {
              const double2 cs = reinterpret_cast<const double2 *>(rdc)[k];
              c = cs.x; sn = cs.y;
            } else {
              const typename Vec4<T>::type cs = reinterpret_cast<const typename Vec4<T>::type *>(rc)[k];
              c = cs.x; sn = cs.y;
            }
            T *vp = V + vcp[j] + vrow;
            T *vq = V + vcq[j] + vrow;
            const T va = *vp, vb = *vq;
            *vp = c * va - sn * vb;
            *vq = sn * va + c * vb;
            vcp[j] = vcp[j] + n >= vwrap ? vcp[j] + n - vwrap : vcp[j] + n;
            if (k > 0) vcq[j] = vcq[j] + n >= vwrap ? vcq[j] + n - vwrap : vcq[j] + n;
          }
        }
      }
      T o0[4], o1[4];
      if (I0 >= 0) rotate_block<T>(b0, I0, J0, nblk, A, rc, rdc, o0);
      if (BIG && I1 >= 0) rotate_block<T>(b1, I1, J1, nblk, A, rc, rdc, o1);
      if (nbuf == 1) __syncthreads();
      if (I0 >= 0) store_block<T>(An, nblk, d0, tw0, o0);
      if (BIG && I1 >= 0) store_block<T>(An, nblk, d1, tw1, o1);
      if (nbuf == 2) cur ^= 1;
      __syncthreads();
    }
  }
  rfin = g % mm;
  if (rounds) *rounds = g;
  return cur;
}

}  // namespace dev
}  // namespace strom
