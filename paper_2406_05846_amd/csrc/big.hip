// big.hip -- PSD projection and eigendecomposition of blocks too large for the LDS of one
// workgroup (the paper's 190 x 190 and 231 x 231 moment blocks in FP64, Table 1), spread over
// many workgroups.  Same operation as project.hip (the parallel PSD cone projection of Sec.
// "GPU Speedup"), different eigensolver.
//
// Two-sided block Jacobi.  A block of size n is padded with zero rows and columns to np, a
// multiple of 64, and cut into nb = np / 32 column blocks of 32.  A sweep is nb - 1 rounds of
// the round-robin tournament over the column blocks.  In a round the nb / 2 pairs (I, J) are
// disjoint; for each pair one workgroup diagonalizes the 64 x 64 subproblem
// [W_II W_IJ; W_JI W_JJ] with the LDS Jacobi of jacobi_lds.h (to a tighter tolerance than the
// outer one), giving an orthogonal G_p.  Then all of them are applied at once, W <- P^T W P and
// U <- U P with P block diagonal (after a permutation) in the G's: the 64 x 64 tile of W between
// pairs X <= Y becomes G_X^T W_XY G_Y (and its transpose goes to W_YX), and a 64-row tile of
// U's pair-Y columns becomes U_RY G_Y -- dense products on the FP64 matrix cores, one
// workgroup per tile.  Zero padding stays exactly zero (a rotation against a zero row is
// skipped), so the padded indices keep eigenvalue 0 and unit eigenvectors and drop out of
// the reconstruction.  The sweeps stop once off(W) <= 1e-11 ||W||_F: the pair launch of every
// round 0 measures it over the whole W, and every later launch on a converged block returns
// at once (the host enqueues a fixed number of sweeps, so the sequence can be captured).
//
// W, U (np x np, column-major), the pair rotations, the eigenvalue selection and the flags
// of every block live in a caller-provided work area (big_work_doubles).  The ADMM form warm-
// starts like the one-workgroup kernel: W = Q^T X_b Q and U = Q from the kept eigenvectors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"
#include "jacobi_lds.h"

namespace strom {
namespace dev {

namespace {

constexpr int kTile = 64;  // product tile, and the size of a pair subproblem
constexpr int kHalf = 32;  // column block of the block Jacobi
constexpr int kKc = 32;    // k-chunk of a product staged in LDS
constexpr int kLd = 68;    // LDS row stride of a staged chunk (doubles)
constexpr int kGemmThreads = 256;
constexpr double kOuterTol = 1e-11;  // stop when off(W) <= kOuterTol ||W||_F

struct SubTol {  // the pair subproblems: tighter than the outer tolerance
  static constexpr double off_rel = 1e-13;
  static constexpr double skip_rel = 1e-18;
};

// Work area of block k (doubles, every region 256-byte aligned): W | U | G (pairs x 64 x 64) |
// lam (np) | sel (np + 2 ints: selected indices, then side and count) | flag (pairs + 2 ints:
// active, sweeps run, then one per pair: its rotation is not the identity).
struct BigBlock {
  double *W, *U, *G, *lam;
  int32_t *sel, *flag;
};

__host__ __device__ inline size_t round32(size_t x) { return (x + 31) & ~size_t(31); }

__host__ __device__ inline size_t block_doubles(int np) {
  const size_t P = size_t(np) / kTile, nps = size_t(np) * np;
  return round32(nps) * 2 + round32(P * kTile * kTile) + round32(size_t(np)) + round32((size_t(np) + 2 + P + 2 + 1) / 2);
}

__device__ inline BigBlock big_block(const BigArgs &a, int k) {
  const size_t P = size_t(a.np) / kTile, nps = size_t(a.np) * a.np;
  double *base = a.work + size_t(k) * block_doubles(a.np);
  BigBlock b;
  b.W = base;
  b.U = b.W + round32(nps);
  b.G = b.U + round32(nps);
  b.lam = b.G + round32(P * kTile * kTile);
  b.sel = reinterpret_cast<int32_t *>(b.lam + round32(size_t(a.np)));
  b.flag = b.sel + a.np + 2;
  return b;
}

// Size of block k; 0 (and the error flag) when it is out of range.
__device__ inline int big_n(const BigArgs &a, int k) {
  const int n = a.ids ? a.bsz[a.ids[k]] : a.nd[k];
  if (n <= 0 || n > a.np) {
    if (a.err && threadIdx.x == 0) atomicOr(a.err, 1);
    return 0;
  }
  return n;
}

// Entry (i, j) of input block k: svec (sqrt(2) on the off-diagonal) or dense column-major.
__device__ inline double big_x(const BigArgs &a, const double *in, int k, int n, int i, int j) {
  if (a.ids) {
    const double v = in[a.boff[a.ids[k]] + pidx(i, j)];
    return i == j ? v : v * 0.70710678118654752440;
  }
  return in[a.od[k] + i + (int64_t)j * n];
}

// The kept eigenvectors of an ADMM block (n x nn at Q + qoff, column = index), padded to np with
// unit vectors.
__device__ inline double q_pad(const double *q, int n, int i, int j) {
  if (i < n && j < n) return q[(int64_t)j * n + i];
  return (i == j && i >= n) ? 1.0 : 0.0;
}

// Pair p of round r of the circle tournament over nb column blocks: block nb - 1 stays put.
__device__ inline void pair_of(int r, int p, int nb, int &I, int &J) {
  const int m = nb - 1;
  if (p == 0) {
    I = r;
    J = m;
  } else {
    I = (r + p) % m;
    J = (r - p + m) % m;
  }
}

// Global index of local index l (0..63) of the pair (I, J).
__device__ inline int pair_glob(int I, int J, int l) { return l < kHalf ? kHalf * I + l : kHalf * J + l - kHalf; }

// acc[c] = the 16 x 64 band (rows 16 wave ..) of A B for K = k_end, chunk by chunk: stage_a(k0)
// fills As[kk * kLd + i] (i < 64) with A(k0 + kk, i)^T, zero past k_end, and stage_b(k0) returns
// the chunk of B, row kk at [kk * kLd] (staged in LDS, or already there).  Lane l of a wave
// receives column 16 c + l % 16, rows 16 wave + 4 r + l / 16.
template <class SA, class SB>
__device__ __forceinline__ void tile_gemm(int k_end, double *As, SA stage_a, SB stage_b, mfma_d4 *acc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < k_end; k0 += kKc) {
    stage_a(k0);
    const double *Bc = stage_b(k0);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kKc / 4; ++s) {
      const int kk = 4 * s + lk;
      const double av = As[kk * kLd + 16 * wave + li];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bc[kk * kLd + 16 * c + li], acc[c], 0, 0, 0);
    }
    __syncthreads();
  }
}

// Staging helpers: fill a 32 x 64 chunk (kk, i) from f(k, i), zero past k_end; "k fast" walks k
// first (coalesced when consecutive k are consecutive in memory), else i first.
template <class F>
__device__ __forceinline__ void stage_kfast(double *D, int k0, int k_end, F f) {
  for (int e = threadIdx.x; e < kKc * kTile; e += blockDim.x) {
    const int kk = e % kKc, i = e / kKc, k = k0 + kk;
    D[kk * kLd + i] = k < k_end ? f(k, i) : 0.0;
  }
}
template <class F>
__device__ __forceinline__ void stage_ifast(double *D, int k0, int k_end, F f) {
  for (int e = threadIdx.x; e < kKc * kTile; e += blockDim.x) {
    const int i = e % kTile, kk = e / kTile, k = k0 + kk;
    D[kk * kLd + i] = k < k_end ? f(k, i) : 0.0;
  }
}

__device__ __forceinline__ int acc_row(int r) { return 16 * (threadIdx.x >> 6) + 4 * r + ((threadIdx.x & 63) >> 4); }
__device__ __forceinline__ int acc_col(int c) { return 16 * c + (threadIdx.x & 15); }

}  // namespace

size_t big_work_doubles(int np, int count) { return block_doubles(np) * size_t(count); }

int big_padded(int n) { return (n + kTile - 1) / kTile * kTile; }


namespace {

// Outer sweeps enqueued from a cold start (a random block of 190-300 needs 8-9) and from the kept
// eigenvectors (about 3 for a perturbation of 1e-4 of the block); every pair subproblem is solved
// to its tolerance.  (One Jacobi sweep per subproblem and round needs as many outer sweeps on
// random spectra in a model of the method on the CPU, but fell short of the outer tolerance
// within 16 sweeps on clustered ones.)
constexpr int kColdSweeps = 24;
constexpr int kWarmSweeps = 10;
constexpr int kPairSweeps = 40;

// ------------------------------------------------------------------------------ start

// Cold start: W = the padded block, U = I.  Tiles (R <= C) of 64 x 64; grid (tiles, blocks).
__global__ void __launch_bounds__(kGemmThreads) k_big_init(BigArgs a, const double *__restrict__ in) {
  const int k = blockIdx.y, np = a.np;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  int R, C;
  tri_ij(blockIdx.x, R, C);
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int i = kTile * R + e % kTile, j = kTile * C + e / kTile;
    const double v = (i < n && j < n) ? big_x(a, in, k, n, i, j) : 0.0;
    b.W[i + (int64_t)j * np] = v;
    b.U[i + (int64_t)j * np] = i == j ? 1.0 : 0.0;
    if (R != C) {
      b.W[j + (int64_t)i * np] = v;
      b.U[j + (int64_t)i * np] = 0.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) b.flag[1] = 0;
}

// Warm start, first product: U <- X Q, the padded block times the padded eigenvectors (all
// tiles; only k < n contributes).
__global__ void __launch_bounds__(kGemmThreads) k_big_xq(BigArgs a, const double *__restrict__ X,
                                                         const double *__restrict__ Q, const int64_t *__restrict__ qoff) {
  __shared__ double As[kKc * kLd], Bs[kKc * kLd];
  const int k = blockIdx.y, np = a.np, Pt = np / kTile;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  const int R = blockIdx.x / Pt, C = blockIdx.x % Pt;
  const double *q = Q + qoff[a.ids[k]];
  mfma_d4 acc[4];
  tile_gemm(
      n, As,
      [&](int k0) {
        stage_ifast(As, k0, n, [&](int kk, int i) {
          const int ii = kTile * R + i;
          return ii < n ? big_x(a, X, k, n, ii, kk) : 0.0;
        });
      },
      [&](int k0) -> const double * {
        stage_kfast(Bs, k0, n, [&](int kk, int j) { return q_pad(q, n, kk, kTile * C + j); });
        return Bs;
      },
      acc);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) b.U[(kTile * R + acc_row(r)) + (int64_t)(kTile * C + acc_col(c)) * np] = acc[c][r];
  if (blockIdx.x == 0 && threadIdx.x == 0) b.flag[1] = 0;
}

// Warm start, second product: W <- Q^T U (upper tiles, mirrored: W is exactly symmetric).
__global__ void __launch_bounds__(kGemmThreads) k_big_qtxq(BigArgs a, const double *__restrict__ Q,
                                                           const int64_t *__restrict__ qoff) {
  __shared__ double As[kKc * kLd], Bs[kKc * kLd];
  const int k = blockIdx.y, np = a.np;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  int R, C;
  tri_ij(blockIdx.x, R, C);
  const double *q = Q + qoff[a.ids[k]];
  mfma_d4 acc[4];
  tile_gemm(
      n, As,
      [&](int k0) { stage_kfast(As, k0, n, [&](int kk, int i) { return q_pad(q, n, kk, kTile * R + i); }); },
      [&](int k0) -> const double * {
        stage_kfast(Bs, k0, n, [&](int kk, int j) { return b.U[kk + (int64_t)(kTile * C + j) * np]; });
        return Bs;
      },
      acc);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = acc_row(r), j = acc_col(c);
      if (R == C && i > j) continue;
      const int gi = kTile * R + i, gj = kTile * C + j;
      b.W[gi + (int64_t)gj * np] = acc[c][r];
      b.W[gj + (int64_t)gi * np] = acc[c][r];
    }
}

// Warm start, last step: U <- Q, padded (all tiles).
__global__ void __launch_bounds__(kGemmThreads) k_big_copyq(BigArgs a, const double *__restrict__ Q,
                                                            const int64_t *__restrict__ qoff) {
  const int k = blockIdx.y, np = a.np, Pt = np / kTile;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  const int R = blockIdx.x / Pt, C = blockIdx.x % Pt;
  const double *q = Q + qoff[a.ids[k]];
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int i = kTile * R + e % kTile, j = kTile * C + e / kTile;
    b.U[i + (int64_t)j * np] = q_pad(q, n, i, j);
  }
}

// ------------------------------------------------------------------------------ sweeps

// Round r, pair blockIdx.x of block blockIdx.y: the subproblem's rotation G_p.  On round 0 of a
// sweep every pair workgroup of the block measures off(W) over the whole block (the same sums
// in the same order, so all reach the same decision) and sets the block's active flag.
__global__ void __launch_bounds__(1024) k_big_pair(BigArgs a, int32_t r, uint32_t lds_cap) {
  extern __shared__ __align__(32) unsigned char smem[];
  const int k = blockIdx.y, p = blockIdx.x, np = a.np, nb = np / kHalf;
  const BigBlock b = big_block(a, k);
  Smem sm = carve<double>(smem, kTile, lds_cap);
  if (r == 0) {
    double off = 0.0, fro = 0.0;
    for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
      const double v = b.W[e];
      fro += v * v;
      if (e % np != e / np) off += v * v;
    }
    off = wg_sum(off, sm.red);
    fro = wg_sum(fro, sm.red);
    const int active = off > kOuterTol * kOuterTol * fro ? 1 : 0;
    if (threadIdx.x == 0) {
      b.flag[0] = active;
      if (p == 0 && active) b.flag[1] += 1;
    }
    if (!active) return;
  } else if (!b.flag[0]) {
    return;
  }
  int I, J;
  pair_of(r, p, nb, I, J);
  const int nn = kTile, np2 = nn / 2, nblk = np2 * (np2 + 1) / 2;
  double *Ab = reinterpret_cast<double *>(sm.A);
  for (int e = threadIdx.x; e < nn * (nn + 1) / 2; e += blockDim.x) {
    int x, y;
    tri_ij(e, x, y);
    const int i = pair_glob(I, J, logical_index(x, 0, nn - 1)), j = pair_glob(I, J, logical_index(y, 0, nn - 1));
    store_entry<double>(Ab, nblk, x, y, b.W[i + (int64_t)j * np]);
  }
  __syncthreads();
  int rfin = 0, rounds = 0;
  double *V = reinterpret_cast<double *>(sm.V);
  jacobi_eig<double, false, true, SubTol>(kTile, Ab, sm.nbuf, V, reinterpret_cast<double *>(sm.rot), sm.rotd, sm.red,
                                          false, rfin, &rounds, kPairSweeps);
  double *G = b.G + (size_t)p * kTile * kTile;
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) G[e] = V[e];  // column c = local index c
  if (threadIdx.x == 0) b.flag[2 + p] = rounds > 0 ? 1 : 0;
}

// Round r: W <- P^T W P and U <- U P.  Workgroups [0, Pt(Pt+1)/2) take the W tiles between
// pairs X <= Y; the next Pt * Pt take the U tiles (64-row tile R, pair Y).  Every workgroup
// reads and writes only its own tiles (the pairs partition the indices), so the update is in
// place.
__global__ void __launch_bounds__(kGemmThreads) k_big_apply(BigArgs a, int32_t r) {
  __shared__ double As[kKc * kLd], BT[kTile * kLd];  // BT: B chunks, then T = W_XY G_Y
  const int k = blockIdx.y, np = a.np, nb = np / kHalf, P = nb / 2;
  const BigBlock b = big_block(a, k);
  if (!b.flag[0]) return;
  const int ntw = P * (P + 1) / 2;
  mfma_d4 acc[4];
  auto stage_g = [&](const double *Gp) {
    return [&, Gp](int k0) -> const double * {
      stage_kfast(BT, k0, kTile, [&](int kk, int j) { return Gp[kk + kTile * j]; });
      return BT;
    };
  };
  if ((int)blockIdx.x < ntw) {
    int X, Y;
    tri_ij(blockIdx.x, X, Y);
    if (!b.flag[2 + X] && !b.flag[2 + Y]) return;  // both rotations are the identity
    int IX, JX, IY, JY;
    pair_of(r, X, nb, IX, JX);
    pair_of(r, Y, nb, IY, JY);
    const double *GX = b.G + (size_t)X * kTile * kTile, *GY = b.G + (size_t)Y * kTile * kTile;
    tile_gemm(
        kTile, As,
        [&](int k0) {
          stage_ifast(As, k0, kTile, [&](int kk, int i) {
            return b.W[pair_glob(IX, JX, i) + (int64_t)pair_glob(IY, JY, kk) * np];
          });
        },
        stage_g(GY), acc);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) BT[acc_row(rr) * kLd + acc_col(c)] = acc[c][rr];
    __syncthreads();
    tile_gemm(
        kTile, As, [&](int k0) { stage_kfast(As, k0, kTile, [&](int kk, int i) { return GX[kk + kTile * i]; }); },
        [&](int k0) -> const double * { return BT + k0 * kLd; }, acc);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int i = acc_row(rr), j = acc_col(c);
        if (X == Y && i > j) continue;
        const int gi = pair_glob(IX, JX, i), gj = pair_glob(IY, JY, j);
        b.W[gi + (int64_t)gj * np] = acc[c][rr];
        b.W[gj + (int64_t)gi * np] = acc[c][rr];
      }
  } else {
    const int u = blockIdx.x - ntw, R = u / P, Y = u % P;
    if (!b.flag[2 + Y]) return;
    int IY, JY;
    pair_of(r, Y, nb, IY, JY);
    const double *GY = b.G + (size_t)Y * kTile * kTile;
    tile_gemm(
        kTile, As,
        [&](int k0) {
          stage_ifast(As, k0, kTile, [&](int kk, int i) {
            return b.U[(kTile * R + i) + (int64_t)pair_glob(IY, JY, kk) * np];
          });
        },
        stage_g(GY), acc);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        b.U[(kTile * R + acc_row(rr)) + (int64_t)pair_glob(IY, JY, acc_col(c)) * np] = acc[c][rr];
  }
}

// ------------------------------------------------------------------------------ finish

// The cheaper side of the spectrum (as select_side of the one-workgroup kernel): the positive
// eigenvalues when they are at most as many as the negative ones, else the negative ones, in
// index order; sel[np] = 1 for the positive side, sel[np + 1] = count.  One wave per block.
__global__ void __launch_bounds__(64) k_big_select(BigArgs a) {
  const int k = blockIdx.x, np = a.np, lane = threadIdx.x;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  int npos = 0, nneg = 0;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    const double l = i < n ? b.W[i + (int64_t)i * np] : 0.0;
    npos += __popcll(__ballot(l > 0.0));
    nneg += __popcll(__ballot(l < 0.0));
  }
  const int pos = npos <= nneg;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int c = 0;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    const double l = i < n ? b.W[i + (int64_t)i * np] : 0.0;
    const bool f = i < n && (pos ? l > 0.0 : l < 0.0);
    const unsigned long long m = __ballot(f);
    if (f) {
      const int t = c + __popcll(m & below);
      b.sel[t] = i;
      b.lam[t] = l;
    }
    c += __popcll(m);
  }
  if (lane == 0) {
    b.sel[np] = pos;
    b.sel[np + 1] = c;
  }
}

// P = U_s diag(lam_s) U_s^T over the selected pairs, upper tiles (R <= C) within n.  DENSE:
// out = Pi(in) (positive side: P; negative side: in - P), both triangles of the column-major
// block (out may alias in: each entry of in is read only by the thread that writes it).  Else
// ADMM: S = (Pi(X) - X) * mul in svec (positive side: P - X; negative: -P), mul = scale, or
// 1 / sigma when scale <= 0.
template <bool DENSE>
__global__ void __launch_bounds__(kGemmThreads) k_big_recon(BigArgs a, const double *in, double *out,
                                                            const DevState *__restrict__ st, double scale) {
  __shared__ double As[kKc * kLd], Bs[kKc * kLd];
  const int k = blockIdx.y, np = a.np;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  int R, C;
  tri_ij(blockIdx.x, R, C);
  if (kTile * C >= n) return;  // R <= C: the tile lies outside the block
  const int pos = b.sel[np], cnt = b.sel[np + 1];
  mfma_d4 acc[4];
  tile_gemm(
      cnt, As,
      [&](int k0) {
        stage_ifast(As, k0, cnt, [&](int t, int i) {
          const int ii = kTile * R + i;
          return ii < n ? b.lam[t] * b.U[ii + (int64_t)b.sel[t] * np] : 0.0;
        });
      },
      [&](int k0) -> const double * {
        stage_ifast(Bs, k0, cnt, [&](int t, int j) {
          const int jj = kTile * C + j;
          return jj < n ? b.U[jj + (int64_t)b.sel[t] * np] : 0.0;
        });
        return Bs;
      },
      acc);
  const double mul = DENSE ? 1.0 : (scale > 0.0 ? scale : 1.0 / st->sigma);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int ii = kTile * R + acc_row(rr), jj = kTile * C + acc_col(c);
      if (ii > jj || jj >= n) continue;
      const double p = acc[c][rr];
      if constexpr (DENSE) {
        const int64_t o = a.od[k];
        const double v = pos ? p : in[o + ii + (int64_t)jj * n] - p;
        out[o + ii + (int64_t)jj * n] = v;
        out[o + jj + (int64_t)ii * n] = v;
      } else {
        const int64_t o = a.boff[a.ids[k]] + (int64_t)jj * (jj + 1) / 2 + ii;
        const double ps = ii == jj ? p : p * 1.41421356237309504880;
        out[o] = pos ? (ps - in[o]) * mul : -ps * mul;
      }
    }
}

// Re-orthogonalization of the eigenvectors before they are kept (one Newton-Schulz step,
// q = U - U (U^T U - I) / 2, as in the one-workgroup kernel).  First W <- U^T U - I (upper
// tiles, mirrored; W is free once the eigenvalues are selected) ...
__global__ void __launch_bounds__(kGemmThreads) k_big_gram(BigArgs a) {
  __shared__ double As[kKc * kLd], Bs[kKc * kLd];
  const int k = blockIdx.y, np = a.np;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  int R, C;
  tri_ij(blockIdx.x, R, C);
  if (kTile * C >= n) return;
  mfma_d4 acc[4];
  tile_gemm(
      n, As, [&](int k0) { stage_kfast(As, k0, n, [&](int kk, int i) { return b.U[kk + (int64_t)(kTile * R + i) * np]; }); },
      [&](int k0) -> const double * {
        stage_kfast(Bs, k0, n, [&](int kk, int j) { return b.U[kk + (int64_t)(kTile * C + j) * np]; });
        return Bs;
      },
      acc);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int i = acc_row(rr), j = acc_col(c);
      if (R == C && i > j) continue;
      const int gi = kTile * R + i, gj = kTile * C + j;
      const double v = acc[c][rr] - (gi == gj ? 1.0 : 0.0);
      b.W[gi + (int64_t)gj * np] = v;
      b.W[gj + (int64_t)gi * np] = v;
    }
}

// ... then q = U - U W / 2 for the n x n part (tiles (R, C) within n); the dummy column of an
// odd block is zero.  REORTH = false: q = U.
template <bool REORTH>
__global__ void __launch_bounds__(kGemmThreads) k_big_storeq(BigArgs a, double *__restrict__ Q,
                                                             const int64_t *__restrict__ qoff) {
  __shared__ double As[kKc * kLd], Bs[kKc * kLd];
  const int k = blockIdx.y, np = a.np, Pt = np / kTile;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  const int R = blockIdx.x / Pt, C = blockIdx.x % Pt;
  const int nn = n + (n & 1);
  if (kTile * R >= n || kTile * C >= nn) return;
  double *q = Q + qoff[a.ids[k]];
  mfma_d4 acc[4];
  if constexpr (REORTH) {
    tile_gemm(
        n, As,
        [&](int k0) { stage_ifast(As, k0, n, [&](int kk, int i) { return b.U[(kTile * R + i) + (int64_t)kk * np]; }); },
        [&](int k0) -> const double * {
          stage_kfast(Bs, k0, n, [&](int kk, int j) { return b.W[kk + (int64_t)(kTile * C + j) * np]; });
          return Bs;
        },
        acc);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int ii = kTile * R + acc_row(rr), jj = kTile * C + acc_col(c);
      if (ii >= n || jj >= nn) continue;
      q[(int64_t)jj * n + ii] = jj < n ? b.U[ii + (int64_t)jj * np] - 0.5 * acc[c][rr] : 0.0;
    }
}

// Eigenvalues in ascending order (ties by index) at w + woff[k] and, with v, the eigenvectors as
// the columns of an n x n column-major block at v + od[k].
__global__ void __launch_bounds__(kGemmThreads) k_big_eigout(BigArgs a, const int64_t *__restrict__ woff,
                                                             double *__restrict__ w, double *__restrict__ v) {
  const int k = blockIdx.x, np = a.np;
  const int n = big_n(a, k);
  const BigBlock b = big_block(a, k);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double li = b.W[i + (int64_t)i * np];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = b.W[j + (int64_t)j * np];
      rank += (lj < li || (lj == li && j < i)) ? 1 : 0;
    }
    w[woff[k] + rank] = li;
    b.sel[i] = rank;
  }
  if (!v) return;
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e % n, i = e / n;
    v[a.od[k] + r + (int64_t)b.sel[i] * n] = b.U[r + (int64_t)i * np];
  }
}

hipError_t enqueue_sweeps(hipStream_t s, const BigArgs &a, int sweeps) {
  const int nb = a.np / kHalf, Pt = a.np / kTile;
  const size_t lds = lds_bytes_for(kTile, sizeof(double));
  hipError_t e = hipFuncSetAttribute((const void *)k_big_pair, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int napply = Pt * (Pt + 1) / 2 + Pt * Pt;
  for (int sw = 0; sw < sweeps; ++sw)
    for (int r = 0; r < nb - 1; ++r) {
      hipLaunchKernelGGL(k_big_pair, dim3(Pt, a.count), dim3(1024), lds, s, a, r, (uint32_t)lds);
      hipLaunchKernelGGL(k_big_apply, dim3(napply, a.count), dim3(kGemmThreads), 0, s, a, r);
    }
  return hipGetLastError();
}

bool args_ok(const BigArgs &a) { return a.np >= kTile && a.np % kTile == 0 && a.np <= kBigMaxN && a.work; }

}  // namespace

hipError_t launch_project_big_admm(hipStream_t s, const BigArgs &a, const double *X, double *S, const DevState *st,
                                   double scale, double *Q, const int64_t *qoff, bool warm, bool reorth) {
  if (a.count <= 0) return hipSuccess;
  if (!args_ok(a) || !a.ids) return hipErrorInvalidValue;
  const int Pt = a.np / kTile, tri = Pt * (Pt + 1) / 2;
  const dim3 blk(kGemmThreads);
  if (warm && Q) {
    hipLaunchKernelGGL(k_big_xq, dim3(Pt * Pt, a.count), blk, 0, s, a, X, Q, qoff);
    hipLaunchKernelGGL(k_big_qtxq, dim3(tri, a.count), blk, 0, s, a, Q, qoff);
    hipLaunchKernelGGL(k_big_copyq, dim3(Pt * Pt, a.count), blk, 0, s, a, Q, qoff);
  } else {
    hipLaunchKernelGGL(k_big_init, dim3(tri, a.count), blk, 0, s, a, X);
  }
  hipError_t e = enqueue_sweeps(s, a, warm && Q ? kWarmSweeps : kColdSweeps);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_select, dim3(a.count), dim3(64), 0, s, a);
  if (Q) {
    if (reorth) {
      hipLaunchKernelGGL(k_big_gram, dim3(tri, a.count), blk, 0, s, a);
      hipLaunchKernelGGL(k_big_storeq<true>, dim3(Pt * Pt, a.count), blk, 0, s, a, Q, qoff);
    } else {
      hipLaunchKernelGGL(k_big_storeq<false>, dim3(Pt * Pt, a.count), blk, 0, s, a, Q, qoff);
    }
  }
  hipLaunchKernelGGL(k_big_recon<false>, dim3(tri, a.count), blk, 0, s, a, X, S, st, scale);
  return hipGetLastError();
}

hipError_t launch_project_big_dense(hipStream_t s, const BigArgs &a, const double *in, double *out) {
  if (a.count <= 0) return hipSuccess;
  if (!args_ok(a) || a.ids) return hipErrorInvalidValue;
  const int Pt = a.np / kTile, tri = Pt * (Pt + 1) / 2;
  hipLaunchKernelGGL(k_big_init, dim3(tri, a.count), dim3(kGemmThreads), 0, s, a, in);
  hipError_t e = enqueue_sweeps(s, a, kColdSweeps);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_select, dim3(a.count), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_big_recon<true>, dim3(tri, a.count), dim3(kGemmThreads), 0, s, a, in, out, nullptr, 1.0);
  return hipGetLastError();
}

hipError_t launch_eig_big_dense(hipStream_t s, const BigArgs &a, const double *in, const int64_t *woff, double *w,
                                double *v) {
  if (a.count <= 0) return hipSuccess;
  if (!args_ok(a) || a.ids) return hipErrorInvalidValue;
  const int Pt = a.np / kTile, tri = Pt * (Pt + 1) / 2;
  hipLaunchKernelGGL(k_big_init, dim3(tri, a.count), dim3(kGemmThreads), 0, s, a, in);
  hipError_t e = enqueue_sweeps(s, a, kColdSweeps);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_eigout, dim3(a.count), dim3(kGemmThreads), 0, s, a, woff, w, v);
  return hipGetLastError();
}

}  // namespace dev
}  // namespace strom
