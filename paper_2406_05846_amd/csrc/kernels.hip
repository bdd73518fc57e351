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
#include <type_traits>

#include "kernels.h"
#include "strom_internal.h"

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
__device__ __forceinline__ void rhs_row(int32_t i, int32_t m, const int64_t *__restrict__ rp,
                                        const int32_t *__restrict__ ci, const double *__restrict__ av,
                                        const double *__restrict__ X, const double *__restrict__ S,
                                        const double *__restrict__ C, const double *__restrict__ b,
                                        const int32_t *__restrict__ pinv, const DevState *__restrict__ st,
                                        double *__restrict__ w) {
  if (i >= m) return;
  const double sig = st->sigma;
  double acc = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
    const int32_t c = ci[p];
    acc += av[p] * (X[c] / sig + S[c] - C[c]);
  }
  w[pinv[i]] = b[i] / sig - acc;
}

__global__ void __launch_bounds__(256) k_rhs(int32_t m, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                             const double *__restrict__ av, const double *__restrict__ X,
                                             const double *__restrict__ S, const double *__restrict__ C,
                                             const double *__restrict__ b, const int32_t *__restrict__ pinv,
                                             const DevState *__restrict__ st, double *__restrict__ w) {
  rhs_row(blockIdx.x * blockDim.x + threadIdx.x, m, rp, ci, av, X, S, C, b, pinv, st, w);
}

// The same over a batch, in two passes: every column's term X/sigma + S - C once, into the X_b
// buffer (free at both right-hand sides of an iteration: step 2 recomputes it), then the rows
// gather that one array instead of three (the gathers fetch whole lines, so one array instead
// of three is most of the kernel's traffic).
__global__ void __launch_bounds__(256) k_rhs_term_batch(const BatchItem *__restrict__ items,
                                                        const BatchInst *__restrict__ bi) {
  const BatchItem it = items[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active) return;
  const int64_t c = (int64_t)it.idx * 256 + threadIdx.x;
  if (c >= I.n) return;
  const double sig = G(I.st)->sigma;
  G(I.Xb)[c] = G(I.X)[c] / sig + G(I.S)[c] - G(I.C)[c];
}

__global__ void __launch_bounds__(256) k_rhs_batch(const BatchItem *__restrict__ items,
                                                   const BatchInst *__restrict__ bi) {
  const BatchItem it = items[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active) return;
  const int32_t i = it.idx * 256 + threadIdx.x;
  if (i >= I.m) return;
  const int64_t *rp = G(I.A_rp);
  const int32_t *ci = G(I.A_ci);
  const double *av = G(I.A_v), *T = G(I.Xb);
  double acc = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) acc += av[p] * T[ci[p]];
  G(I.w)[G(I.pinv)[i]] = G(I.b)[i] / G(I.st)->sigma - acc;
}

// ------------------------------------------------------------------ triangular solves
// One workgroup per task; the task's values stay in LDS while its phases run.  Every phase is
// solved from its streams: the forward gather sums, for each row, the contributions of the
// task's earlier phases and the partial sums pushed by other tasks; rows on their own are
// then solved, and every component of two or more rows is solved by a product with the
// explicit inverse of its diagonal block.  Forward contributions to later tasks' rows are not
// gathered by the receiving row: the task owning the columns computes them as partial sums
// ("push segments", its push stream) right after its own rows are solved, so the work of a
// separator row is spread over the tasks below it.
// One phase stream (see setup.cpp): thread t walks its slice of K entries (entry k at
// off + k * Tp + t), W kStreamBatch loads in flight (kStreamBatch for the last granules),
// then their factors get(index) (get never reads what fin writes), then adds them in order;
// fin(row, sum) completes a row.  A row
// that started in an earlier slice is completed after a barrier by the thread holding its
// last entry, adding the pieces of the earlier slices in order (tail_v / tail_r: the open
// row of every slice).  Contains one __syncthreads(): call from all threads.
// Shape of one stream of a phase (or of a task's push stream): its offset, entries per thread
// and thread count, the same for the whole workgroup (kept in scalar registers), and its
// slice starts (kSolveThreads + 1 of them).  Every phase has all four streams and every task a
// push stream, so the heads of a phase's streams are loaded together, ahead of the passes that
// use them; a pass then issues its slice start and its first entries at once.
struct StreamHead {
  int64_t off;
  int32_t K, Tp;
  const int32_t *first;
};

template <class A>
__device__ __forceinline__ StreamHead stream_head(const A &a, int kind, int32_t ph) {
  StreamHead h;
  const int64_t off = G(a.s_off[kind])[ph];
  h.off = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(off >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)off));
  h.K = __builtin_amdgcn_readfirstlane(G(a.s_K[kind])[ph]);
  h.Tp = __builtin_amdgcn_readfirstlane(G(a.s_T[kind])[ph]);
  h.first = G(a.s_ra[kind]) + (int64_t)ph * (kSolveThreads + 1);
  return h;
}

template <int W, class Get, class Fin>
__device__ inline void stream_phase(const double *__restrict__ val, const int32_t *__restrict__ idx,
                                    const StreamHead &h, double *tail_v, int32_t *tail_r, Get get, Fin fin) {
  const int t = threadIdx.x;
  const int64_t off = h.off;
  const int32_t K = h.K, Tp = h.Tp;
  int32_t head_row = -1;
  double head_v = 0.0;
  if (t < Tp) {
    const int32_t f = h.first[t];
    int32_t row = f & (kStartFlag - 1);
    bool own = (f & kStartFlag) != 0;
    const double *vp = val + off + t;
    const int32_t *ip = idx + off + t;
    double acc = 0.0;
    auto batch = [&](auto nb, int32_t k0) {  // nb entries from k0: loads, factors, then sums in order
      constexpr int NB = decltype(nb)::value;
      double v[NB];
      int32_t x[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        v[u] = vp[(int64_t)(k0 + u) * Tp];
        x[u] = ip[(int64_t)(k0 + u) * Tp];
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) v[u] *= get(x[u] & (kLastFlag - 1));
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        acc += v[u];
        if (x[u] & kLastFlag) {
          if (own) fin(row, acc);
          else { head_row = row; head_v = acc; }
          acc = 0.0;
          ++row;
          own = true;
        }
      }
    };
    // W granules' loads in flight where the slice holds them (K is a multiple of kStreamBatch)
    int32_t k0 = 0;
    for (; k0 + W * kStreamBatch <= K; k0 += W * kStreamBatch)
      batch(std::integral_constant<int, W * kStreamBatch>(), k0);
    for (; k0 < K; k0 += kStreamBatch) batch(std::integral_constant<int, kStreamBatch>(), k0);
    tail_v[t] = acc;
    tail_r[t] = own ? row : -1 - row;  // the open row; negative: it started in an earlier slice
  }
  __syncthreads();
  if (head_row >= 0) {
    double s = 0.0;
    int u = t - 1;
    while (u >= 0 && tail_r[u] == -1 - head_row) --u;  // slices lying inside the row
    // u is the slice where the row starts (its open row is head_row, non-negative)
    for (int q = u; q < t; ++q) s += tail_v[q];
    fin(head_row, s + head_v);
  }
}

// Forward solve of task t.  INL: the task is staged in LDS -- its rows, then the partial sums
// pushed to it -- and the stream indices are task-local; else its values are read and written
// in place in w and the indices are global.  A separate instantiation for each case keeps every
// access in one address space (LDS or global).
template <int W, bool INL, class A>
__device__ __forceinline__ void solve_fwd_task(int32_t t, const A &a, double *__restrict__ w, double *sh) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int32_t r0 = G(a.task_r0)[t], r1 = G(a.task_r1)[t], nt = r1 - r0;
  double *tail_v = sh;  // open-row pieces of the stream slices
  int32_t *tail_r = reinterpret_cast<int32_t *>(sh + kSolveThreads);
  double *buf = sh + kSolveThreads + kSolveThreads / 2;
  const int32_t p0 = INL ? G(a.task_pin)[t] : 0, npin = INL ? G(a.task_pin)[t + 1] - p0 : 0;
  double *xs = INL ? buf : (w + r0);          // values of the task rows, index i - r0
  double *c = INL ? buf + nt + npin : buf;    // right-hand sides of the phase's components
  if (INL) {
    for (int i = tid; i < nt; i += nth) xs[i] = w[r0 + i];
    for (int k = tid; k < npin; k += nth) xs[nt + k] = G(a.part)[p0 + k];
  }
  const StreamHead hp = stream_head(a, 4, t);
  __syncthreads();
  for (int32_t ph = G(a.task_ph0)[t]; ph < G(a.task_ph1)[t]; ++ph) {
    const int32_t pa = G(a.ph_a)[ph], nns = G(a.ph_nns)[ph];
    const StreamHead h0 = stream_head(a, 0, ph), h1 = stream_head(a, 1, ph);
    stream_phase<W>(G(a.sval[0]), G(a.sidx[0]), h0, tail_v, tail_r,
                [&](int32_t j) {
                  if constexpr (INL) return xs[j];
                  else return (j & kPartFlag) ? G(a.part)[j & (kPartFlag - 1)] : w[j];
                },
                [&](int32_t r, double acc) {
                  const double v = xs[pa + r - r0] - acc;
                  if (r < nns) c[r] = v;
                  else xs[pa + r - r0] = v;  // a row on its own: solved
                });
    if (nns > 0) {
      __syncthreads();
      stream_phase<W>(G(a.sval[1]), G(a.sidx[1]), h1, tail_v, tail_r, [&](int32_t j) { return c[j]; },
                   [&](int32_t r, double acc) { xs[pa + r - r0] = acc; });
    }
    __syncthreads();
  }
  // push: partial sums of the later rows over this task's columns, one stream row per segment
  if (G(a.tsptr)[t] < G(a.tsptr)[t + 1]) {
    const int32_t s0 = G(a.tsptr)[t];
    stream_phase<W>(G(a.sval[4]), G(a.sidx[4]), hp, tail_v, tail_r,
                 [&](int32_t j) {
                   if constexpr (INL) return xs[j];
                   else return w[j];
                 },
                 [&](int32_t r, double acc) { G(a.part)[G(a.tseg)[s0 + r]] = acc; });
  }
  if (INL)
    for (int i = tid; i < nt; i += nth) w[r0 + i] = xs[i];
}

__global__ void __launch_bounds__(kSolveThreads) k_solve_fwd(const int32_t *__restrict__ tasks, SolveArgs a,
                                                             double *__restrict__ w) {
  extern __shared__ double sh[];
  const int32_t t = tasks[blockIdx.x];
  if (a.task_inl[t]) solve_fwd_task<2, true>(t, a, w, sh);
  else solve_fwd_task<2, false>(t, a, w, sh);
}

__global__ void __launch_bounds__(kSolveThreads) k_solve_fwd_batch(const BatchItem *__restrict__ tasks,
                                                                   const SolveArgs *__restrict__ args,
                                                                   const BatchInst *__restrict__ bi) {
  extern __shared__ double sh[];
  const BatchItem it = tasks[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active) return;
  const SolveArgsG &a = reinterpret_cast<const SolveArgsG *>(args)[it.inst];
  if (G(a.task_inl)[it.idx]) solve_fwd_task<2, true>(it.idx, a, G(I.w), sh);
  else solve_fwd_task<2, false>(it.idx, a, G(I.w), sh);
}

// Backward: L^T x = D^{-1} z over the phases in reverse order (a row only depends here on
// its own component, later phases and later tasks).  INL: the task's rows and the rows of
// later tasks it reads are staged in LDS, stream indices task-local.
template <int W, bool INL, class A>
__device__ __forceinline__ void solve_bwd_task(int32_t t, const A &a, double *__restrict__ w,
                                               double *__restrict__ y, double *sh) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int32_t r0 = G(a.task_r0)[t], r1 = G(a.task_r1)[t], nt = r1 - r0;
  double *tail_v = sh;
  int32_t *tail_r = reinterpret_cast<int32_t *>(sh + kSolveThreads);
  double *buf = sh + kSolveThreads + kSolveThreads / 2;
  const int64_t x0 = INL ? G(a.task_xoff)[t] : 0;
  const int32_t nx = INL ? (int32_t)(G(a.task_xoff)[t + 1] - x0) : 0;
  double *xs = INL ? buf : (w + r0);
  double *c = INL ? buf + nt + nx : buf;
  if (INL) {
    for (int i = tid; i < nt; i += nth) xs[i] = w[r0 + i];
    for (int k = tid; k < nx; k += nth) xs[nt + k] = w[G(a.task_xrow)[x0 + k]];
  }
  __syncthreads();
  for (int32_t ph = G(a.task_ph1)[t] - 1; ph >= G(a.task_ph0)[t]; --ph) {
    const int32_t pa = G(a.ph_a)[ph], nns = G(a.ph_nns)[ph];
    const StreamHead h2 = stream_head(a, 2, ph), h3 = stream_head(a, 3, ph);
    stream_phase<W>(G(a.sval[2]), G(a.sidx[2]), h2, tail_v, tail_r,
                [&](int32_t i) {
                  if constexpr (INL) return xs[i];
                  else return w[i];
                },
                [&](int32_t r, double acc) {
                  const int32_t j = pa + r;
                  const double v = xs[j - r0] / G(a.D)[j] - acc;
                  if (r < nns) c[r] = v;
                  else xs[j - r0] = v;
                });
    if (nns > 0) {
      __syncthreads();
      stream_phase<W>(G(a.sval[3]), G(a.sidx[3]), h3, tail_v, tail_r, [&](int32_t j) { return c[j]; },
                   [&](int32_t r, double acc) { xs[pa + r - r0] = acc; });
    }
    __syncthreads();
  }
  for (int i = tid; i < nt; i += nth) {
    const double v = xs[i];
    if (INL) w[r0 + i] = v;
    y[G(a.perm)[r0 + i]] = v;
  }
}

__global__ void __launch_bounds__(kSolveThreads) k_solve_bwd(const int32_t *__restrict__ tasks, SolveArgs a,
                                                             double *__restrict__ w, double *__restrict__ y) {
  extern __shared__ double sh[];
  const int32_t t = tasks[blockIdx.x];
  if (a.task_inl[t]) solve_bwd_task<2, true>(t, a, w, y, sh);
  else solve_bwd_task<2, false>(t, a, w, y, sh);
}

__global__ void __launch_bounds__(kSolveThreads) k_solve_bwd_batch(const BatchItem *__restrict__ tasks,
                                                                   const SolveArgs *__restrict__ args,
                                                                   const BatchInst *__restrict__ bi) {
  extern __shared__ double sh[];
  const BatchItem it = tasks[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active) return;
  const SolveArgsG &a = reinterpret_cast<const SolveArgsG *>(args)[it.inst];
  if (G(a.task_inl)[it.idx]) solve_bwd_task<2, true>(it.idx, a, G(I.w), G(I.y), sh);
  else solve_bwd_task<2, false>(it.idx, a, G(I.w), G(I.y), sh);
}

// The root task: the last forward group and the first backward group are both this one task,
// so one workgroup solves it forward and then backward (the barrier between makes its rows,
// written back to w by the forward pass, visible to the backward pass of the same group).
__global__ void __launch_bounds__(kSolveThreads) k_solve_root(int32_t t, SolveArgs a, double *__restrict__ w,
                                                              double *__restrict__ y) {
  extern __shared__ double sh[];
  if (a.task_inl[t]) solve_fwd_task<1, true>(t, a, w, sh);
  else solve_fwd_task<1, false>(t, a, w, sh);
  __syncthreads();
  if (a.task_inl[t]) solve_bwd_task<1, true>(t, a, w, y, sh);
  else solve_bwd_task<1, false>(t, a, w, y, sh);
}

// ------------------------------------------------------------------ step 2: X_b
__device__ __forceinline__ void xb_col(int64_t c, int64_t n, const int64_t *__restrict__ trp,
                                       const int32_t *__restrict__ tci, const double *__restrict__ tv,
                                       const double *__restrict__ y, const double *__restrict__ X,
                                       const double *__restrict__ C, const DevState *__restrict__ st,
                                       double *__restrict__ Xb) {
  if (c >= n) return;
  double aty = 0.0;
  for (int64_t p = trp[c]; p < trp[c + 1]; ++p) aty += tv[p] * y[tci[p]];
  Xb[c] = X[c] + st->sigma * (aty - C[c]);
}

__global__ void __launch_bounds__(256) k_xb(int64_t n, const int64_t *__restrict__ trp, const int32_t *__restrict__ tci,
                                            const double *__restrict__ tv, const double *__restrict__ y,
                                            const double *__restrict__ X, const double *__restrict__ C,
                                            const DevState *__restrict__ st, double *__restrict__ Xb) {
  xb_col((int64_t)blockIdx.x * blockDim.x + threadIdx.x, n, trp, tci, tv, y, X, C, st, Xb);
}

__global__ void __launch_bounds__(256) k_xb_batch(const BatchItem *__restrict__ items, const BatchInst *__restrict__ bi) {
  const BatchItem it = items[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active) return;
  xb_col((int64_t)it.idx * 256 + threadIdx.x, I.n, G(I.At_rp), G(I.At_ci), G(I.At_v), G(I.y), G(I.X), G(I.C), G(I.st),
         G(I.Xb));
}

// ------------------------------------------------------------------ step 4: X update + dual residual
// Columns [256 chunk, 256 chunk + 256): X += tau sigma d (update != 0), d = S + A^* y - C, and
// with part the chunk's sums of d^2 and C X at part[2 chunk ..].  Call from all 256 threads.
__device__ __forceinline__ void xupdate_chunk(int32_t chunk, int64_t n, const int64_t *__restrict__ trp,
                                              const int32_t *__restrict__ tci, const double *__restrict__ tv,
                                              const double *__restrict__ y, const double *__restrict__ S,
                                              const double *__restrict__ C, const DevState *__restrict__ st,
                                              double *__restrict__ X, double *__restrict__ part, int32_t update,
                                              double *red) {
  const int64_t c = (int64_t)chunk * 256 + threadIdx.x;
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
      part[2 * chunk] = d2;
      part[2 * chunk + 1] = cx;
    }
  }
}

__global__ void __launch_bounds__(256) k_xupdate(int64_t n, const int64_t *__restrict__ trp, const int32_t *__restrict__ tci,
                                                 const double *__restrict__ tv, const double *__restrict__ y,
                                                 const double *__restrict__ S, const double *__restrict__ C,
                                                 const DevState *__restrict__ st, double *__restrict__ X,
                                                 double *__restrict__ part, int32_t update) {
  __shared__ double red[256];
  xupdate_chunk(blockIdx.x, n, trp, tci, tv, y, S, C, st, X, part, update, red);
}

__global__ void __launch_bounds__(256) k_xupdate_batch(const BatchItem *__restrict__ items,
                                                       const BatchInst *__restrict__ bi, int32_t want_part) {
  __shared__ double red[256];
  const BatchItem it = items[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active) return;
  xupdate_chunk(it.idx, I.n, G(I.At_rp), G(I.At_ci), G(I.At_v), G(I.y), G(I.S), G(I.C), G(I.st), G(I.X),
                want_part ? G(I.part_cols) : nullptr, 1, red);
}

// ------------------------------------------------------------------ KKT
// Rows [256 chunk, 256 chunk + 256): sums of (A X - b)_i^2 and b_i y_i at part[2 chunk ..].
__device__ __forceinline__ void kkt_rows_chunk(int32_t chunk, int32_t m, const int64_t *__restrict__ rp,
                                               const int32_t *__restrict__ ci, const double *__restrict__ av,
                                               const double *__restrict__ X, const double *__restrict__ b,
                                               const double *__restrict__ y, double *__restrict__ part, double *red) {
  const int32_t i = chunk * 256 + threadIdx.x;
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
    part[2 * chunk] = r2;
    part[2 * chunk + 1] = by;
  }
}

__global__ void __launch_bounds__(256) k_kkt_rows(int32_t m, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                  const double *__restrict__ av, const double *__restrict__ X,
                                                  const double *__restrict__ b, const double *__restrict__ y,
                                                  double *__restrict__ part) {
  __shared__ double red[256];
  kkt_rows_chunk(blockIdx.x, m, rp, ci, av, X, b, y, part, red);
}

// Per-block partial sums of ||a||^2 and ||b||^2 (a = Pi(X) - X, b = X for the cone distance).
__device__ __forceinline__ void sqnorms_chunk(int32_t chunk, int64_t n, const double *__restrict__ a,
                                              const double *__restrict__ b, double *__restrict__ part, double *red) {
  const int64_t c = (int64_t)chunk * 256 + threadIdx.x;
  double sa = 0.0, sb = 0.0;
  if (c < n) {
    sa = a[c] * a[c];
    sb = b[c] * b[c];
  }
  sa = block_sum<256>(sa, red);
  sb = block_sum<256>(sb, red);
  if (threadIdx.x == 0) {
    part[2 * chunk] = sa;
    part[2 * chunk + 1] = sb;
  }
}

__global__ void __launch_bounds__(256) k_sqnorms(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                                 double *__restrict__ part) {
  __shared__ double red[256];
  sqnorms_chunk(blockIdx.x, n, a, b, part, red);
}

// Sums the partials in a fixed order (deterministic), forms the residuals of the
// termination rule and, when asked, balances sigma: with eta_K = ||X - Pi(X)|| / (1 + ||X||)
// and r_P = max(eta_p, eta_K), sigma is multiplied by 1.5 when eta_d > 3 r_P and divided by
// 1.5 when r_P > 3 eta_d, kept in [1e-4, 1e4].
__device__ __forceinline__ void kkt_final_body(const double *__restrict__ part_rows, int32_t nrow_parts,
                                               const double *__restrict__ part_cols, int32_t ncol_parts,
                                               const double *__restrict__ part_cone, double normb, double normC,
                                               int32_t do_sigma, DevState *__restrict__ st, double *red) {
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

__global__ void k_kkt_final(const double *__restrict__ part_rows, int32_t nrow_parts,
                            const double *__restrict__ part_cols, int32_t ncol_parts,
                            const double *__restrict__ part_cone, double normb, double normC,
                            int32_t do_sigma, DevState *__restrict__ st) {
  __shared__ double red[256];
  kkt_final_body(part_rows, nrow_parts, part_cols, ncol_parts, part_cone, normb, normC, do_sigma, st, red);
}

// ------------------------------------------------------------------ merged KKT over a batch
__global__ void __launch_bounds__(256) k_kkt_rows_batch(const BatchItem *__restrict__ items,
                                                        const BatchInst *__restrict__ bi) {
  __shared__ double red[256];
  const BatchItem it = items[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active) return;
  kkt_rows_chunk(it.idx, I.m, G(I.A_rp), G(I.A_ci), G(I.A_v), G(I.X), G(I.b), G(I.y), G(I.part_rows), red);
}

__global__ void __launch_bounds__(256) k_sqnorms_batch(const BatchItem *__restrict__ items,
                                                       const BatchInst *__restrict__ bi) {
  __shared__ double red[256];
  const BatchItem it = items[blockIdx.x];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[it.inst];
  if (!I.active || !I.sig) return;
  sqnorms_chunk(it.idx, I.n, G(I.Xb), G(I.X), G(I.part_cone), red);
}

__global__ void __launch_bounds__(256) k_kkt_final_batch(const BatchInst *__restrict__ bi, int32_t do_sigma) {
  __shared__ double red[256];
  const BatchInstG &I = reinterpret_cast<const BatchInstG *>(bi)[blockIdx.x];
  if (!I.active) return;
  kkt_final_body(G(I.part_rows), I.nrow_chunks, G(I.part_cols), I.ncol_chunks, G(I.part_cone), I.normb, I.normC,
                 do_sigma && I.sig, G(I.st), red);
}

__global__ void k_gather_states(int32_t ninst, const BatchInst *__restrict__ bi, DevState *__restrict__ out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) out[i] = *G(reinterpret_cast<const BatchInstG *>(bi)[i].st);
}

// ------------------------------------------------------------------ host launchers
hipError_t launch_rhs(hipStream_t s, int32_t m, const int64_t *rp, const int32_t *ci, const double *av,
                      const double *X, const double *S, const double *C, const double *b, const int32_t *pinv,
                      const DevState *st, double *w) {
  hipLaunchKernelGGL(k_rhs, dim3((m + 255) / 256), dim3(256), 0, s, m, rp, ci, av, X, S, C, b, pinv, st, w);
  return hipGetLastError();
}

hipError_t launch_solve(hipStream_t s, const SolveSchedule &sch, const SolveArgs &a, double *w, double *y) {
  const size_t lds = sizeof(double) * (size_t)(kSolveThreads + kSolveThreads / 2 + a.lds_rows + a.c_cap);
  (void)hipFuncSetAttribute((const void *)k_solve_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute((const void *)k_solve_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute((const void *)k_solve_root, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  const int nf = (int)sch.fwd_gptr.size() - 1, nb = (int)sch.bwd_gptr.size() - 1;
  // one task closes the forward solve and opens the backward one: a single launch for both
  const bool root = nf > 0 && nb > 0 && sch.fwd_gptr[nf] - sch.fwd_gptr[nf - 1] == 1 &&
                    sch.bwd_gptr[1] - sch.bwd_gptr[0] == 1 && !sch.fwd_order.empty() &&
                    sch.fwd_order[size_t(sch.fwd_gptr[nf - 1])] == sch.bwd_order[size_t(sch.bwd_gptr[0])];
  for (int g = 0; g < nf - (root ? 1 : 0); ++g) {
    const int cnt = sch.fwd_gptr[g + 1] - sch.fwd_gptr[g];
    if (cnt <= 0) continue;
    hipLaunchKernelGGL(k_solve_fwd, dim3(cnt), dim3(kSolveThreads), lds, s, sch.fwd_order_dev + sch.fwd_gptr[g], a, w);
  }
  if (root)
    hipLaunchKernelGGL(k_solve_root, dim3(1), dim3(kSolveThreads), lds, s, sch.fwd_order[size_t(sch.fwd_gptr[nf - 1])],
                       a, w, y);
  for (int g = root ? 1 : 0; g < nb; ++g) {
    const int cnt = sch.bwd_gptr[g + 1] - sch.bwd_gptr[g];
    if (cnt <= 0) continue;
    hipLaunchKernelGGL(k_solve_bwd, dim3(cnt), dim3(kSolveThreads), lds, s, sch.bwd_order_dev + sch.bwd_gptr[g], a, w,
                       y);
  }
  return hipGetLastError();
}

hipError_t launch_xb(hipStream_t s, int64_t n, const int64_t *trp, const int32_t *tci, const double *tv,
                     const double *y, const double *X, const double *C, const DevState *st, double *Xb) {
  hipLaunchKernelGGL(k_xb, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, trp, tci, tv, y, X, C, st, Xb);
  return hipGetLastError();
}

// Dual slack of the certificate's lower bound: Z = C - A^* y.
__global__ void __launch_bounds__(256) k_slack(int64_t n, const int64_t *__restrict__ trp, const int32_t *__restrict__ tci,
                                               const double *__restrict__ tv, const double *__restrict__ y,
                                               const double *__restrict__ C, double *__restrict__ Z) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double aty = 0.0;
  for (int64_t p = trp[c]; p < trp[c + 1]; ++p) aty += tv[p] * y[tci[p]];
  Z[c] = C[c] - aty;
}

hipError_t launch_slack(hipStream_t s, int64_t n, const int64_t *trp, const int32_t *tci, const double *tv,
                        const double *y, const double *C, double *Z) {
  hipLaunchKernelGGL(k_slack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, trp, tci, tv, y, C, Z);
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

// ------------------------------------------------------------------ merged launchers
hipError_t launch_rhs_batch(hipStream_t s, int nrows, const BatchItem *rows, int ncols, const BatchItem *cols,
                            const BatchInst *bi) {
  if (ncols > 0) hipLaunchKernelGGL(k_rhs_term_batch, dim3(ncols), dim3(256), 0, s, cols, bi);
  if (nrows > 0) hipLaunchKernelGGL(k_rhs_batch, dim3(nrows), dim3(256), 0, s, rows, bi);
  return hipGetLastError();
}

hipError_t launch_solve_batch(hipStream_t s, const std::vector<int32_t> &fwd_gptr, const BatchItem *fwd,
                              const std::vector<int32_t> &bwd_gptr, const BatchItem *bwd, const SolveArgs *args,
                              const BatchInst *bi, size_t lds_bytes) {
  (void)hipFuncSetAttribute((const void *)k_solve_fwd_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  (void)hipFuncSetAttribute((const void *)k_solve_bwd_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  for (size_t g = 0; g + 1 < fwd_gptr.size(); ++g) {
    const int cnt = fwd_gptr[g + 1] - fwd_gptr[g];
    if (cnt > 0)
      hipLaunchKernelGGL(k_solve_fwd_batch, dim3(cnt), dim3(kSolveThreads), lds_bytes, s, fwd + fwd_gptr[g], args, bi);
  }
  for (size_t g = 0; g + 1 < bwd_gptr.size(); ++g) {
    const int cnt = bwd_gptr[g + 1] - bwd_gptr[g];
    if (cnt > 0)
      hipLaunchKernelGGL(k_solve_bwd_batch, dim3(cnt), dim3(kSolveThreads), lds_bytes, s, bwd + bwd_gptr[g], args, bi);
  }
  return hipGetLastError();
}

hipError_t launch_xb_batch(hipStream_t s, int count, const BatchItem *cols, const BatchInst *bi) {
  if (count > 0) hipLaunchKernelGGL(k_xb_batch, dim3(count), dim3(256), 0, s, cols, bi);
  return hipGetLastError();
}

hipError_t launch_xupdate_batch(hipStream_t s, int count, const BatchItem *cols, const BatchInst *bi, int want_part) {
  if (count > 0) hipLaunchKernelGGL(k_xupdate_batch, dim3(count), dim3(256), 0, s, cols, bi, want_part);
  return hipGetLastError();
}

hipError_t launch_kkt_batch(hipStream_t s, int nrows, const BatchItem *rows, int ncols, const BatchItem *cols,
                            int ninst, const BatchInst *bi, int do_sigma) {
  if (nrows > 0) hipLaunchKernelGGL(k_kkt_rows_batch, dim3(nrows), dim3(256), 0, s, rows, bi);
  if (do_sigma && ncols > 0) hipLaunchKernelGGL(k_sqnorms_batch, dim3(ncols), dim3(256), 0, s, cols, bi);
  if (ninst > 0) hipLaunchKernelGGL(k_kkt_final_batch, dim3(ninst), dim3(256), 0, s, bi, do_sigma);
  return hipGetLastError();
}

hipError_t launch_gather_states(hipStream_t s, int ninst, const BatchInst *bi, DevState *out) {
  if (ninst > 0) hipLaunchKernelGGL(k_gather_states, dim3((ninst + 255) / 256), dim3(256), 0, s, ninst, bi, out);
  return hipGetLastError();
}

}  // namespace dev
}  // namespace strom
