// setup.cpp -- one-time host analysis of an SDP instance for the device solver.
//
//  * validation of the CSR form of A;
//  * row ordering that follows the chain-like sparsity of Def. 1: every row is assigned to
//    the "clique group" of the blocks it touches (a small block joins the largest block it
//    shares a row with); rows inside one group come first, group by group, then the rows
//    that couple two groups, ordered by nested dissection over the chain of groups;
//  * eps*I + A A^* = P L D L^T P^T in FP64 (the paper's pre-permuted sparse factorization,
//    Sec. "GPU Speedup"), eps = eps_reg * max_i (A A^*)_ii, by a left-looking column method
//    with a symbolic pass over the elimination tree;
//  * the schedule of the device triangular solves.  Every group (and every coupling set) is
//    one task, solved by one workgroup.  The dependency levels of a task are cut into
//    phases whose rows form small connected components (chains of the factor); each
//    component is solved at once through the explicit inverse of its unit lower-triangular
//    diagonal block, so a phase costs one gather and one small dense product whatever the
//    number of levels it spans.  Rows are relabeled in (phase, component, level) order (a
//    topological order, so the relabeled L is the factor of the relabeled matrix and
//    nothing is refactored).  Contributions to rows of later tasks are pushed as partial
//    sums by the task owning the columns.  Tasks are launched by dependency depth.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <list>
#include <memory>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "strom_internal.h"

namespace strom {
namespace {

// Nested-dissection post-order of the chain positions [lo, hi]; depth[p] = the level of
// position p in the dissection tree (0 at the root).
void chain_nd(int lo, int hi, std::vector<int> &out, std::vector<int> &depth, int d = 0) {
  if (lo > hi) return;
  const int mid = lo + (hi - lo) / 2;
  chain_nd(lo, mid - 1, out, depth, d + 1);
  chain_nd(mid + 1, hi, out, depth, d + 1);
  out.push_back(mid);
  depth[size_t(mid)] = d;
}

// Levels of the dissection tree (from the root) whose coupling sets form one task, the root
// task.  Their rows come last, in post-order: the schedule loses that many launches per
// direction minus one, and the root task does their work in sequence.  STROM_TOP_LEVELS if set;
// else as many levels as keep the merged rows within kTopRows (measured on MI355X: the pendulum
// N = 10 solve 26% faster with its top three levels merged, 245 rows, and 17% with four, 315;
// cart-pole N = 30 within 2% either way with two, 378 rows, and 4% slower with three, 882).
constexpr int64_t kTopRows = 256;
int top_levels(const std::vector<int64_t> &rows_at_depth) {
  if (const char *ev = std::getenv("STROM_TOP_LEVELS")) return std::max(1, std::atoi(ev));
  int k = 1;
  int64_t rows = rows_at_depth.empty() ? 0 : rows_at_depth[0];
  while (k < int(rows_at_depth.size()) && rows + rows_at_depth[size_t(k)] <= kTopRows) rows += rows_at_depth[size_t(k++)];
  return k;
}

// Minimum-degree order of the rows rows[0..n) of A A^* (rows adjacent when they share a
// column), the other rows that share columns with them counted in every degree but never
// eliminated (they are ordered after these).  Explicit elimination graph: eliminating v joins
// its neighbours into a clique; the next pivot is the row of least degree, ties to the
// earliest in rows[].  rows[] is reordered in place.  `loc` has m entries, all -1 on entry
// and on return.
void min_degree(std::vector<int32_t> &rows, const int64_t *rowptr, const int32_t *col, const HostAnalysis &H,
                std::vector<int32_t> &loc) {
  const int32_t n = int32_t(rows.size());
  if (n < 3) return;
  std::vector<int32_t> glob(rows.begin(), rows.end());  // local index -> row
  for (int32_t v = 0; v < n; ++v) loc[size_t(rows[size_t(v)])] = v;
  std::vector<std::vector<int32_t>> adj(static_cast<size_t>(n));
  for (int32_t v = 0; v < n; ++v) {
    const int32_t i = rows[size_t(v)];
    auto &a = adj[size_t(v)];
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const int32_t c = col[p];
      for (int64_t q = H.Atrp[size_t(c)]; q < H.Atrp[size_t(c) + 1]; ++q) {
        const int32_t j = H.Atci[size_t(q)];
        if (j == i) continue;
        if (loc[size_t(j)] < 0) { loc[size_t(j)] = int32_t(glob.size()); glob.push_back(j); }
        a.push_back(loc[size_t(j)]);
      }
    }
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  std::set<std::pair<int32_t, int32_t>> q;  // (degree, local index) of the rows not yet eliminated
  for (int32_t v = 0; v < n; ++v) q.emplace(int32_t(adj[size_t(v)].size()), v);
  std::vector<int32_t> order, nb, merged;
  order.reserve(size_t(n));
  while (!q.empty()) {
    const int32_t v = q.begin()->second;
    q.erase(q.begin());
    order.push_back(rows[size_t(v)]);
    nb.swap(adj[size_t(v)]);
    adj[size_t(v)].clear();
    for (int32_t a : nb) {
      if (a >= n) continue;  // a later row: its degree is not needed
      auto &aa = adj[size_t(a)];
      q.erase({int32_t(aa.size()), a});
      merged.clear();
      size_t x = 0, y = 0;  // (aa \ {v}) U (nb \ {a}), both sorted
      while (x < aa.size() || y < nb.size()) {
        int32_t t;
        if (y == nb.size() || (x < aa.size() && aa[x] < nb[y])) t = aa[x++];
        else if (x == aa.size() || nb[y] < aa[x]) t = nb[y++];
        else { t = aa[x++]; ++y; }
        if (t != v && t != a) merged.push_back(t);
      }
      aa.swap(merged);
      q.emplace(int32_t(aa.size()), a);
    }
    nb.clear();
  }
  rows.swap(order);
  for (int32_t g : glob) loc[size_t(g)] = -1;
}

// Lanes per row for a gather of up to `len` entries.
int32_t lanes_for(int64_t len) {
  int32_t g = 1;
  while (g < 64 && int64_t(g) * 4 < len) g *= 2;
  return g;
}

// Where every value of an analysis comes from, so that an instance with the same sparsity
// pattern (the same family, variant and horizon: only the initial state and the obstacle
// change the coefficients) reuses the symbolic part and recomputes only the numbers.
struct NumericMaps {
  std::vector<int64_t> at_src;                 // Atv[q] = val[at_src[q]]
  std::vector<int32_t> perm0, pinv0;           // the row order the factor is computed in
  std::vector<int64_t> Cp0;                    // pattern of L in that order, by columns
  std::vector<int32_t> Ci0;
  std::vector<int32_t> tr0, tr1;               // the tasks of that order (parallel factorization)
  std::vector<int64_t> lv_src, uv_src;         // Lv[p] = Cx0[lv_src[p]], Uv[p] = Cx0[uv_src[p]]
  std::vector<int32_t> d_src;                  // D[i] = D0[d_src[i]]
  std::vector<int64_t> push_src;               // push_v[e] = Lv[push_src[e]]
  std::vector<int64_t> s_src[kStreamKinds];    // stream values: code of Lv / Uv / invR / invC, -1: 0, -2: 1
};

// K = P (A A^*) P^T, lower triangle by columns (diagonal first), in the row order perm;
// returns max diag.
double assemble_K(int32_t m, const int64_t *rowptr, const int32_t *col, const double *val,
                  const std::vector<int32_t> &perm, const std::vector<int32_t> &pinv, const HostAnalysis &H,
                  std::vector<int64_t> &Kp, std::vector<int32_t> &Ki, std::vector<double> &Kx) {
  Kp.assign(size_t(m) + 1, 0);
  Ki.clear();
  Kx.clear();
  double maxdiag = 0.0;
  std::vector<double> acc(size_t(m), 0.0);
  std::vector<int32_t> seen(size_t(m), -1), list;
  Ki.reserve(size_t(rowptr[m]) * 6);
  Kx.reserve(size_t(rowptr[m]) * 6);
  for (int32_t j = 0; j < m; ++j) {  // column j of the lower triangle (new order)
    const int32_t oj = perm[size_t(j)];
    list.clear();
    for (int64_t p = rowptr[oj]; p < rowptr[oj + 1]; ++p) {
      const int32_t c = col[p];
      for (int64_t q = H.Atrp[size_t(c)]; q < H.Atrp[size_t(c) + 1]; ++q) {
        const int32_t ni = pinv[size_t(H.Atci[size_t(q)])];
        if (ni < j) continue;
        if (seen[size_t(ni)] != j) { seen[size_t(ni)] = j; acc[size_t(ni)] = 0.0; list.push_back(ni); }
        acc[size_t(ni)] += val[p] * H.Atv[size_t(q)];
      }
    }
    if (seen[size_t(j)] != j) { seen[size_t(j)] = j; acc[size_t(j)] = 0.0; list.push_back(j); }
    std::sort(list.begin(), list.end());
    Kp[size_t(j)] = int64_t(Ki.size());
    for (int32_t ni : list) { Ki.push_back(ni); Kx.push_back(acc[size_t(ni)]); }
    maxdiag = std::max(maxdiag, acc[size_t(j)]);
  }
  Kp[size_t(m)] = int64_t(Ki.size());
  return maxdiag;
}

// Left-looking LDL^T of K on the known pattern (Cp, Ci) of L by columns.  Column j gathers
// the updates of the earlier columns k with L(j, k) != 0 from a list of columns "waiting on
// row j" (a column waits on the row of its next unused entry): the list is last-in first-out,
// so the order of the updates, and with it the rounding, is the order in which the columns
// arrived at row j.
//
// The columns come in tasks (contiguous row ranges: clique groups, then the coupling sets in
// nested-dissection order).  A task depends on the tasks whose columns have entries in its rows;
// tasks of one dependency level run in parallel threads, each with its own work vector.  A
// column arriving at a row of another task is recorded instead of linked; before a task runs,
// the arrivals at its rows are linked in the sequential order (by the task that performed them,
// then in its order) -- every such task is one of its dependencies (if L(j, k) and L(r, k) are
// nonzero for k < j < r, so is L(r, j)) -- so the result is bit for bit the sequential one.
// STROM_SETUP_THREADS sets the thread count (1: the sequential loop).
strom_status numeric_factor(int32_t m, const std::vector<int64_t> &Kp, const std::vector<int32_t> &Ki,
                            const std::vector<double> &Kx, const std::vector<int64_t> &Cp,
                            const std::vector<int32_t> &Ci, const std::vector<int32_t> &tr0,
                            const std::vector<int32_t> &tr1, std::vector<double> &Cx, std::vector<double> &Dn,
                            std::string &err) {
  Cx.assign(size_t(Cp[size_t(m)]), 0.0);
  Dn.assign(size_t(m), 0.0);
  std::vector<int64_t> nxt(size_t(m), 0);                          // next unused entry of column k
  std::vector<int32_t> head(size_t(m), -1), link(size_t(m), -1);  // columns waiting on row j
  struct Arrival { int32_t r, k; };
  // Columns [a, b) with work vector w; arrivals at rows >= b go to out (when given), else linked.
  auto run = [&](int32_t a, int32_t b, std::vector<double> &w, std::vector<Arrival> *out, int32_t &bad) {
    auto arrive = [&](int32_t r, int32_t k) {
      if (out && r >= b) { out->push_back({r, k}); return; }
      link[size_t(k)] = head[size_t(r)];
      head[size_t(r)] = k;
    };
    for (int32_t j = a; j < b; ++j) {
      for (int64_t p = Kp[size_t(j)]; p < Kp[size_t(j) + 1]; ++p) w[size_t(Ki[size_t(p)])] = Kx[size_t(p)];
      int32_t k = head[size_t(j)];
      while (k >= 0) {
        const int32_t knext = link[size_t(k)];
        const int64_t p0 = nxt[size_t(k)], pend = Cp[size_t(k) + 1];
        const double f = Cx[size_t(p0)] * Dn[size_t(k)];  // L(j,k) D(k)
        for (int64_t p = p0; p < pend; ++p) w[size_t(Ci[size_t(p)])] -= Cx[size_t(p)] * f;
        nxt[size_t(k)] = p0 + 1;
        if (p0 + 1 < pend) arrive(Ci[size_t(p0 + 1)], k);
        k = knext;
      }
      const double dj = w[size_t(j)];
      w[size_t(j)] = 0.0;
      if (!(dj > 0.0) || !std::isfinite(dj)) {
        bad = j;
        return;
      }
      Dn[size_t(j)] = dj;
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
        const int32_t i = Ci[size_t(p)];
        Cx[size_t(p)] = w[size_t(i)] / dj;
        w[size_t(i)] = 0.0;
      }
      if (Cp[size_t(j)] < Cp[size_t(j) + 1]) {
        nxt[size_t(j)] = Cp[size_t(j)];
        arrive(Ci[size_t(Cp[size_t(j)])], j);
      }
    }
  };
  auto pivot_error = [&](int32_t j) {
    err = "non-positive pivot in LDL^T of eps*I + A A^* at row " + std::to_string(j);
    return STROM_E_FACTOR;
  };
  int threads = int(std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency())));
  if (const char *ev = std::getenv("STROM_SETUP_THREADS")) threads = std::max(1, std::atoi(ev));
  const int32_t nt = int32_t(tr0.size());
  bool tasks_ok = nt > 1 && threads > 1 && tr0.size() == tr1.size() && tr0[0] == 0 && tr1[size_t(nt) - 1] == m;
  for (int32_t t = 1; tasks_ok && t < nt; ++t) tasks_ok = tr0[size_t(t)] == tr1[size_t(t) - 1];
  std::vector<int32_t> rtask, level;
  if (tasks_ok) {
    rtask.resize(size_t(m));
    for (int32_t t = 0; t < nt; ++t)
      for (int32_t r = tr0[size_t(t)]; r < tr1[size_t(t)]; ++r) rtask[size_t(r)] = t;
    level.assign(size_t(nt), 0);
    for (int32_t t = 0; t < nt && tasks_ok; ++t)  // tasks ascend, so their dependencies come first
      for (int32_t k = tr0[size_t(t)]; k < tr1[size_t(t)]; ++k)
        for (int64_t p = Cp[size_t(k)]; p < Cp[size_t(k) + 1]; ++p) {
          const int32_t u = rtask[size_t(Ci[size_t(p)])];
          if (u < t) { tasks_ok = false; break; }
          if (u > t) level[size_t(u)] = std::max(level[size_t(u)], level[size_t(t)] + 1);
        }
  }
  if (!tasks_ok) {
    std::vector<double> w(size_t(m), 0.0);
    int32_t bad = -1;
    run(0, m, w, nullptr, bad);
    return bad >= 0 ? pivot_error(bad) : STROM_OK;
  }
  const int32_t nlev = *std::max_element(level.begin(), level.end()) + 1;
  std::vector<std::vector<int32_t>> by_level(static_cast<size_t>(nlev));
  for (int32_t t = 0; t < nt; ++t) by_level[size_t(level[size_t(t)])].push_back(t);
  struct Rec { int32_t src; int64_t seq; Arrival a; };
  std::vector<std::vector<Rec>> inbox(static_cast<size_t>(nt));
  std::vector<std::vector<Arrival>> outs(static_cast<size_t>(nt));
  std::vector<int32_t> bad(size_t(nt), -1);
  std::vector<std::vector<double>> works(static_cast<size_t>(threads));
  bool dag_ok = true;
  for (int32_t L = 0; L < nlev && dag_ok; ++L) {
    const std::vector<int32_t> &ts = by_level[size_t(L)];
    std::atomic<size_t> next(0);
    auto worker = [&](int id) {
      std::vector<double> &w = works[size_t(id)];
      if (w.empty()) w.assign(size_t(m), 0.0);
      for (size_t q; (q = next.fetch_add(1)) < ts.size();) {
        const int32_t t = ts[q];
        std::vector<Rec> &in = inbox[size_t(t)];
        std::sort(in.begin(), in.end(), [](const Rec &x, const Rec &y) {
          return x.src != y.src ? x.src < y.src : x.seq < y.seq;
        });
        for (const Rec &x : in) {
          link[size_t(x.a.k)] = head[size_t(x.a.r)];
          head[size_t(x.a.r)] = x.a.k;
        }
        run(tr0[size_t(t)], tr1[size_t(t)], w, &outs[size_t(t)], bad[size_t(t)]);
      }
    };
    const int nth = int(std::min<size_t>(size_t(threads), ts.size()));
    std::vector<std::thread> pool;
    for (int i = 1; i < nth; ++i) pool.emplace_back(worker, i);
    worker(0);
    for (auto &th : pool) th.join();
    for (int32_t t : ts) {
      if (bad[size_t(t)] >= 0) continue;
      const std::vector<Arrival> &o = outs[size_t(t)];
      for (size_t i = 0; i < o.size(); ++i) {
        const int32_t u = rtask[size_t(o[i].r)];
        if (level[size_t(u)] <= L) { dag_ok = false; break; }
        inbox[size_t(u)].push_back({t, int64_t(i), o[i]});
      }
      std::vector<Arrival>().swap(outs[size_t(t)]);
    }
  }
  int32_t first_bad = -1;
  for (int32_t b : bad)
    if (b >= 0 && (first_bad < 0 || b < first_bad)) first_bad = b;
  if (first_bad >= 0) return pivot_error(first_bad);
  if (!dag_ok) {  // an arrival outside the dependency structure: not expected, redo sequentially
    std::fill(nxt.begin(), nxt.end(), 0);
    std::fill(head.begin(), head.end(), -1);
    std::fill(link.begin(), link.end(), -1);
    std::vector<double> w(size_t(m), 0.0);
    int32_t b = -1;
    run(0, m, w, nullptr, b);
    return b >= 0 ? pivot_error(b) : STROM_OK;
  }
  return STROM_OK;
}

// Inverse of the unit lower-triangular diagonal block of L over the component rows [c0, c1)
// (final order, CSR of L), row-major in inv (cn x cn).
void component_inverse(const HostAnalysis &H, int32_t c0, int32_t c1, std::vector<double> &blk,
                       std::vector<double> &inv) {
  const int32_t cn = c1 - c0;
  blk.assign(size_t(cn) * cn, 0.0);
  inv.assign(size_t(cn) * cn, 0.0);
  for (int32_t i = c0; i < c1; ++i)
    for (int64_t p = H.Lrp[size_t(i)]; p < H.Lrp[size_t(i) + 1]; ++p) {
      const int32_t j = H.Lci[size_t(p)];
      if (j >= c0) blk[size_t(i - c0) * cn + size_t(j - c0)] = H.Lv[size_t(p)];
    }
  for (int32_t c = 0; c < cn; ++c) {
    inv[size_t(c) * cn + size_t(c)] = 1.0;
    for (int32_t i = c + 1; i < cn; ++i) {
      double sacc = 0.0;
      for (int32_t k = c; k < i; ++k) sacc -= blk[size_t(i) * cn + size_t(k)] * inv[size_t(k) * cn + size_t(c)];
      inv[size_t(i) * cn + size_t(c)] = sacc;
    }
  }
}

}  // namespace

namespace {
// One analysis with a given row order inside the groups' interior runs (md_order: minimum
// degree, else the order of the rows as given).
strom_status analyze_order(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
                           const int32_t *col, const double *val, double eps_reg, HostAnalysis &H,
                           std::string &err, int split_mode, int block_rows, NumericMaps *mp, bool md_order) {
  // ---------------------------------------------------------------- validation
  if (nblocks <= 0 || !bsize || m <= 0 || !rowptr || !col || !val) {
    err = "empty problem or NULL array";
    return STROM_E_INVAL;
  }
  if (m >= kPartFlag) {
    err = "too many constraints";
    return STROM_E_INVAL;
  }
  H = HostAnalysis();
  H.m = m;
  H.nblocks = nblocks;
  H.bsize.assign(bsize, bsize + nblocks);
  H.boff.resize(static_cast<size_t>(nblocks) + 1);
  H.boff[0] = 0;
  for (int32_t k = 0; k < nblocks; ++k) {
    if (bsize[k] <= 0) { err = "block size <= 0"; return STROM_E_INVAL; }
    H.boff[size_t(k) + 1] = H.boff[size_t(k)] + int64_t(bsize[k]) * (bsize[k] + 1) / 2;
  }
  H.nsvec = H.boff[size_t(nblocks)];
  if (H.nsvec >= (int64_t(1) << 31)) { err = "svec length exceeds int32 column indices"; return STROM_E_INVAL; }
  if (rowptr[0] != 0) { err = "rowptr[0] != 0"; return STROM_E_INVAL; }
  for (int32_t i = 0; i < m; ++i)
    if (rowptr[i + 1] < rowptr[i]) { err = "rowptr not monotone"; return STROM_E_INVAL; }
  const int64_t nnz = rowptr[m];
  for (int64_t p = 0; p < nnz; ++p)
    if (col[p] < 0 || int64_t(col[p]) >= H.nsvec) { err = "column index out of range"; return STROM_E_INVAL; }
  for (int64_t p = 0; p < nnz; ++p)
    if (!std::isfinite(val[p])) { err = "non-finite value in A"; return STROM_E_INVAL; }

  // column -> block
  std::vector<int32_t> colblock(static_cast<size_t>(H.nsvec));
  for (int32_t k = 0; k < nblocks; ++k)
    std::fill(colblock.begin() + H.boff[size_t(k)], colblock.begin() + H.boff[size_t(k) + 1], k);

  // A^T
  H.Atrp.assign(size_t(H.nsvec) + 1, 0);
  for (int64_t p = 0; p < nnz; ++p) H.Atrp[size_t(col[p]) + 1]++;
  for (int64_t c = 0; c < H.nsvec; ++c) H.Atrp[size_t(c) + 1] += H.Atrp[size_t(c)];
  H.Atci.resize(size_t(nnz));
  H.Atv.resize(size_t(nnz));
  if (mp) mp->at_src.resize(size_t(nnz));
  {
    std::vector<int64_t> fill(H.Atrp.begin(), H.Atrp.end() - 1);
    for (int32_t i = 0; i < m; ++i)
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int64_t q = fill[size_t(col[p])]++;
        H.Atci[size_t(q)] = i;
        H.Atv[size_t(q)] = val[p];
        if (mp) mp->at_src[size_t(q)] = p;
      }
  }

  // ---------------------------------------------------------------- grouping and order
  // A block is attached to the largest block that shares a row with it, if that one is larger.
  std::vector<int32_t> attach(static_cast<size_t>(nblocks), -1);
  std::vector<int32_t> rb;  // blocks of the current row
  for (int32_t i = 0; i < m; ++i) {
    rb.clear();
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) rb.push_back(colblock[size_t(col[p])]);
    std::sort(rb.begin(), rb.end());
    rb.erase(std::unique(rb.begin(), rb.end()), rb.end());
    if (rb.size() < 2) continue;
    for (int32_t a : rb)
      for (int32_t c : rb)
        if (bsize[c] > bsize[a] && (attach[size_t(a)] < 0 || bsize[c] > bsize[attach[size_t(a)]]))
          attach[size_t(a)] = c;
  }
  std::vector<int32_t> bgroup(static_cast<size_t>(nblocks), -1);
  int32_t ngroups = 0;
  for (int32_t k = 0; k < nblocks; ++k)
    if (attach[size_t(k)] < 0) bgroup[size_t(k)] = ngroups++;
  for (int32_t k = 0; k < nblocks; ++k) {
    int32_t r = k, hops = 0;
    while (attach[size_t(r)] >= 0 && hops++ < nblocks) r = attach[size_t(r)];
    bgroup[size_t(k)] = bgroup[size_t(r)];
  }
  // row class: interior of group g -> (0, g); coupling of groups g, g+1 -> (1, g); other -> (2, 0)
  std::vector<int32_t> rclass(static_cast<size_t>(m)), rkey(static_cast<size_t>(m));
  std::vector<int32_t> rg;
  for (int32_t i = 0; i < m; ++i) {
    rg.clear();
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) rg.push_back(bgroup[size_t(colblock[size_t(col[p])])]);
    std::sort(rg.begin(), rg.end());
    rg.erase(std::unique(rg.begin(), rg.end()), rg.end());
    if (rg.size() <= 1) { rclass[size_t(i)] = 0; rkey[size_t(i)] = rg.empty() ? 0 : rg[0]; }
    else if (rg.size() == 2 && rg[1] == rg[0] + 1) { rclass[size_t(i)] = 1; rkey[size_t(i)] = rg[0]; }
    else { rclass[size_t(i)] = 2; rkey[size_t(i)] = 0; }
  }
  std::vector<int> sep_pos, sep_depth(static_cast<size_t>(std::max(1, ngroups)), 0);
  chain_nd(0, std::max(0, ngroups - 2), sep_pos, sep_depth);
  std::vector<int32_t> sep_rank(static_cast<size_t>(std::max(1, ngroups)), 0);
  for (size_t r = 0; r < sep_pos.size(); ++r) sep_rank[size_t(sep_pos[r])] = int32_t(r);
  // the coupling sets of the top levels of the dissection tree go last and form one task
  std::vector<int64_t> rows_at_depth;
  for (int32_t i = 0; i < m; ++i)
    if (rclass[size_t(i)] == 1) {
      const size_t dd = size_t(sep_depth[size_t(rkey[size_t(i)])]);
      if (rows_at_depth.size() <= dd) rows_at_depth.resize(dd + 1, 0);
      rows_at_depth[dd]++;
    }
  const int ntop = top_levels(rows_at_depth);
  auto top = [&](int32_t i) { return rclass[size_t(i)] == 1 && sep_depth[size_t(rkey[size_t(i)])] < ntop; };
  H.perm.resize(size_t(m));
  std::iota(H.perm.begin(), H.perm.end(), 0);
  std::stable_sort(H.perm.begin(), H.perm.end(), [&](int32_t a, int32_t b) {
    if (rclass[size_t(a)] != rclass[size_t(b)]) return rclass[size_t(a)] < rclass[size_t(b)];
    if (rclass[size_t(a)] == 0) return rkey[size_t(a)] < rkey[size_t(b)];
    if (rclass[size_t(a)] == 1) {
      const bool ta = top(a), tb = top(b);
      if (ta != tb) return tb;  // the top sets after every lower one
      return sep_rank[size_t(rkey[size_t(a)])] < sep_rank[size_t(rkey[size_t(b)])];
    }
    return false;
  });
  // inside each group's interior run: minimum degree, or the rows' own order
  if (md_order) {
    std::vector<std::pair<int32_t, int32_t>> runs;  // the interior runs, ordered in parallel threads
    int32_t r0 = 0;
    for (int32_t k = 1; k <= m; ++k) {
      const int32_t a = H.perm[size_t(r0)];
      if (k < m && rclass[size_t(H.perm[size_t(k)])] == rclass[size_t(a)] &&
          rkey[size_t(H.perm[size_t(k)])] == rkey[size_t(a)])
        continue;
      if (rclass[size_t(a)] == 0) runs.emplace_back(r0, k);
      r0 = k;
    }
    int threads = int(std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency())));
    if (const char *ev = std::getenv("STROM_SETUP_THREADS")) threads = std::max(1, std::atoi(ev));
    threads = std::max(1, std::min(threads, int(runs.size())));
    std::atomic<size_t> next(0);
    auto worker = [&]() {
      std::vector<int32_t> loc(size_t(m), -1), run;
      for (size_t q; (q = next.fetch_add(1)) < runs.size();) {
        run.assign(H.perm.begin() + runs[q].first, H.perm.begin() + runs[q].second);
        min_degree(run, rowptr, col, H, loc);
        std::copy(run.begin(), run.end(), H.perm.begin() + runs[q].first);
      }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
  }
  H.pinv.resize(size_t(m));
  for (int32_t k = 0; k < m; ++k) H.pinv[size_t(H.perm[size_t(k)])] = k;

  // task ranges: maximal runs of rows with the same (class, key), the top coupling sets as one
  {
    auto tkey = [&](int32_t i) { return top(i) ? -1 : rkey[size_t(i)]; };
    int32_t r0 = 0;
    for (int32_t k = 1; k <= m; ++k) {
      const bool brk = (k == m) || rclass[size_t(H.perm[size_t(k)])] != rclass[size_t(H.perm[size_t(r0)])] ||
                       tkey(H.perm[size_t(k)]) != tkey(H.perm[size_t(r0)]);
      if (brk) { H.task_r0.push_back(r0); H.task_r1.push_back(k); r0 = k; }
    }
  }

  // ---------------------------------------------------------------- K = P A A^* P^T (lower)
  std::vector<int64_t> Kp;
  std::vector<int32_t> Ki;
  std::vector<double> Kx;
  const double maxdiag = assemble_K(m, rowptr, col, val, H.perm, H.pinv, H, Kp, Ki, Kx);
  if (mp) { mp->perm0 = H.perm; mp->pinv0 = H.pinv; }
  H.eps = (eps_reg > 0 ? eps_reg : 1e-12) * (maxdiag > 0 ? maxdiag : 1.0);
  for (int32_t j = 0; j < m; ++j) Kx[size_t(Kp[size_t(j)])] += H.eps;  // first entry is the diagonal

  // ---------------------------------------------------------------- symbolic factorization
  // struct(L_{:,j}) = struct(K_{j+1:,j}) U (union of struct(L_{:,c}) \ {j} over etree children c)
  std::vector<int64_t> Cp(size_t(m) + 1, 0);
  std::vector<int32_t> Ci;
  {
    std::vector<std::vector<int32_t>> children(static_cast<size_t>(m));
    std::vector<int32_t> mark(size_t(m), -1), buf;
    for (int32_t j = 0; j < m; ++j) {
      buf.clear();
      mark[size_t(j)] = j;
      Cp[size_t(j)] = int64_t(Ci.size());  // also closes column j - 1 for the merge below
      for (int64_t p = Kp[size_t(j)] + 1; p < Kp[size_t(j) + 1]; ++p) {
        const int32_t i = Ki[size_t(p)];
        if (mark[size_t(i)] != j) { mark[size_t(i)] = j; buf.push_back(i); }
      }
      for (int32_t c : children[size_t(j)])
        for (int64_t p = Cp[size_t(c)]; p < Cp[size_t(c) + 1]; ++p) {
          const int32_t i = Ci[size_t(p)];
          if (mark[size_t(i)] != j) { mark[size_t(i)] = j; buf.push_back(i); }
        }
      std::sort(buf.begin(), buf.end());
      Ci.insert(Ci.end(), buf.begin(), buf.end());
      if (!buf.empty()) children[size_t(buf[0])].push_back(j);
      if (Ci.size() > size_t(1) << 31) { err = "factor too large"; return STROM_E_NOMEM; }
    }
    Cp[size_t(m)] = int64_t(Ci.size());
  }

  // ---------------------------------------------------------------- numeric, left-looking
  const int64_t nnzL = Cp[size_t(m)];
  std::vector<double> Cx, Dn;
  {
    const strom_status fst = numeric_factor(m, Kp, Ki, Kx, Cp, Ci, H.task_r0, H.task_r1, Cx, Dn, err);
    if (fst != STROM_OK) return fst;
  }
  if (mp) { mp->Cp0 = Cp; mp->Ci0 = Ci; mp->tr0 = H.task_r0; mp->tr1 = H.task_r1; }
  // where each factor value and pivot of the final order comes from (tracked through relabeling)
  std::vector<int64_t> xsrc;
  std::vector<int32_t> dsrc;
  if (mp) {
    xsrc.resize(size_t(nnzL));
    std::iota(xsrc.begin(), xsrc.end(), int64_t(0));
    dsrc.resize(size_t(m));
    std::iota(dsrc.begin(), dsrc.end(), 0);
  }
  H.nnzL = nnzL;
  Kp.clear(); Ki.clear(); Kx.clear();

  // ---------------------------------------------------------------- phases and relabeling
  // Forward dependency level of every row inside its task (longest dependency path from a
  // row of the task that depends on no other row of it).  The levels of a task are cut
  // greedily into phases: a phase is a run of consecutive levels whose rows, joined by the
  // dependencies among them, form connected components of at most kMaxBlockRows rows (at
  // most kMaxPhaseBlockRows rows in components of two or more).  Rows of a task are then
  // relabeled in (phase, component, level) order.  Every relabeling here is a topological
  // order of the factor's dependencies, so the relabeled L stays unit lower triangular and is
  // the factor of the relabeled matrix (nothing is refactored).
  //
  // Load balance: the group tasks run first, one workgroup each, on far fewer CUs than the
  // device has, and the first clique of a trajectory carries the boundary-condition rows (its
  // task costs several times the others).  So every group task is split: the components of
  // its first phase, which do not depend on each other, are dealt to parts of about half the
  // typical group task's cost (stream entries per thread, see rows_cost); its later phases
  // become a task of their own when the coupling task next to it (which depends on them) is
  // at depth 2 or more, else they move into that coupling task.  Either way the split adds
  // no depth.
  // largest component: block_rows if given, else STROM_BLOCK_ROWS if set, else kMaxBlockRows
  int32_t max_block = kMaxBlockRows;
  if (block_rows > 0) {
    max_block = block_rows;
  } else if (const char *ev = std::getenv("STROM_BLOCK_ROWS")) {
    const long v = std::strtol(ev, nullptr, 10);
    if (v >= 1 && v <= 256) max_block = int32_t(v);
  }
  // 0 no split, 1 overweight group tasks only, 2 every group task; -1: STROM_TASK_SPLIT, else 2
  if (split_mode < 0) {
    split_mode = 2;
    if (const char *ev = std::getenv("STROM_TASK_SPLIT")) split_mode = int(std::strtol(ev, nullptr, 10));
  }
  const bool allow_split = split_mode != 0;
  int32_t ntask = int32_t(H.task_r0.size());
  std::vector<int32_t> row_task(static_cast<size_t>(m));
  auto set_row_task = [&]() {
    ntask = int32_t(H.task_r0.size());
    for (int32_t t = 0; t < ntask; ++t)
      for (int32_t r = H.task_r0[size_t(t)]; r < H.task_r1[size_t(t)]; ++r) row_task[size_t(r)] = t;
  };
  std::vector<int32_t> rphase(size_t(m), 0), rcomp(size_t(m), 0), rcsize(size_t(m), 1);
  std::vector<int32_t> lev(size_t(m), 0);
  std::vector<int32_t> newpos(static_cast<size_t>(m));
  std::vector<int32_t> task_nph;
  // Levels and phases of every task; newpos = the (phase, component, level) order.
  auto partition = [&]() {
    std::fill(lev.begin(), lev.end(), 0);
    std::vector<int64_t> predp(size_t(m) + 1, 0);  // predecessors inside the task, CSR by row
    std::vector<int32_t> predi;
    for (int32_t j = 0; j < m; ++j)
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
        const int32_t i = Ci[size_t(p)];
        if (row_task[size_t(i)] == row_task[size_t(j)]) {
          lev[size_t(i)] = std::max(lev[size_t(i)], lev[size_t(j)] + 1);
          predp[size_t(i) + 1]++;
        }
      }
    for (int32_t i = 0; i < m; ++i) predp[size_t(i) + 1] += predp[size_t(i)];
    predi.resize(size_t(predp[size_t(m)]));
    {
      std::vector<int64_t> f(predp.begin(), predp.end() - 1);
      for (int32_t j = 0; j < m; ++j)
        for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
          const int32_t i = Ci[size_t(p)];
          if (row_task[size_t(i)] == row_task[size_t(j)]) predi[size_t(f[size_t(i)]++)] = j;
        }
    }
    task_nph.assign(size_t(ntask), 0);
    for (int32_t t = 0; t < ntask; ++t) {
      const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)], nt = r1 - r0;
      int32_t L = 0;
      for (int32_t i = r0; i < r1; ++i) L = std::max(L, lev[size_t(i)] + 1);
      std::vector<std::vector<int32_t>> bylev(static_cast<size_t>(L));
      for (int32_t i = r0; i < r1; ++i) bylev[size_t(lev[size_t(i)])].push_back(i);
      std::vector<int32_t> par(static_cast<size_t>(nt)), sz(static_cast<size_t>(nt), 1);
      std::iota(par.begin(), par.end(), 0);
      auto find = [&](std::vector<int32_t> &pa, int32_t x) {
        while (pa[size_t(x)] != x) { pa[size_t(x)] = pa[size_t(pa[size_t(x)])]; x = pa[size_t(x)]; }
        return x;
      };
      int32_t l = 0, ph = 0;
      while (l < L) {
        int32_t l1 = l, maxc = 1;
        int64_t nns = 0;  // rows in components of two or more
        while (l1 < L) {
          std::vector<int32_t> par2 = par, sz2 = sz;
          int32_t maxc2 = maxc;
          for (int32_t i : bylev[size_t(l1)])
            for (int64_t p = predp[size_t(i)]; p < predp[size_t(i) + 1]; ++p) {
              const int32_t j = predi[size_t(p)];
              if (lev[size_t(j)] < l) continue;  // earlier phase
              int32_t a = find(par2, i - r0), b = find(par2, j - r0);
              if (a == b) continue;
              if (sz2[size_t(a)] < sz2[size_t(b)]) std::swap(a, b);
              par2[size_t(b)] = a;
              sz2[size_t(a)] += sz2[size_t(b)];
              maxc2 = std::max(maxc2, sz2[size_t(a)]);
            }
          int64_t nns2 = 0;
          if (maxc2 > 1) {
            for (int32_t q = l; q <= l1; ++q)
              for (int32_t i : bylev[size_t(q)]) nns2 += sz2[size_t(find(par2, i - r0))] > 1;
          }
          if (l1 > l && (maxc2 > max_block || nns2 > kMaxPhaseBlockRows)) break;
          par.swap(par2);
          sz.swap(sz2);
          maxc = maxc2;
          nns = nns2;
          ++l1;
        }
        (void)nns;
        for (int32_t q = l; q < l1; ++q)
          for (int32_t i : bylev[size_t(q)]) {
            const int32_t root = find(par, i - r0);
            rphase[size_t(i)] = ph;
            rcomp[size_t(i)] = root;
            rcsize[size_t(i)] = sz[size_t(root)];
          }
        ++ph;
        l = l1;
      }
      task_nph[size_t(t)] = ph;
      std::vector<int32_t> rows(static_cast<size_t>(nt));
      std::iota(rows.begin(), rows.end(), r0);
      std::stable_sort(rows.begin(), rows.end(), [&](int32_t a, int32_t b) {
        if (rphase[size_t(a)] != rphase[size_t(b)]) return rphase[size_t(a)] < rphase[size_t(b)];
        const bool sa = rcsize[size_t(a)] == 1, sb = rcsize[size_t(b)] == 1;
        if (sa != sb) return !sa;  // components of two or more first, singletons last
        if (rcomp[size_t(a)] != rcomp[size_t(b)]) return rcomp[size_t(a)] < rcomp[size_t(b)];
        return lev[size_t(a)] < lev[size_t(b)];
      });
      for (int32_t k = 0; k < nt; ++k) newpos[size_t(rows[size_t(k)])] = r0 + k;
    }
  };
  // Relabel row i -> np[i]: the factor (Cp/Ci/Cx by columns), D, the order and the per-row
  // phase data follow.
  auto relabel = [&](const std::vector<int32_t> &np) {
    std::vector<int64_t> Cp2(size_t(m) + 1, 0);
    std::vector<int32_t> Ci2(static_cast<size_t>(nnzL));
    std::vector<double> Cx2(static_cast<size_t>(nnzL));
    std::vector<int64_t> xs2(xsrc.size());
    for (int32_t j = 0; j < m; ++j) Cp2[size_t(np[size_t(j)]) + 1] = Cp[size_t(j) + 1] - Cp[size_t(j)];
    for (int32_t j = 0; j < m; ++j) Cp2[size_t(j) + 1] += Cp2[size_t(j)];
    for (int32_t j = 0; j < m; ++j) {
      int64_t q = Cp2[size_t(np[size_t(j)])];
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p, ++q) {
        Ci2[size_t(q)] = np[size_t(Ci[size_t(p)])];
        Cx2[size_t(q)] = Cx[size_t(p)];
        if (mp) xs2[size_t(q)] = xsrc[size_t(p)];
      }
    }
    Cp.swap(Cp2);
    Ci.swap(Ci2);
    Cx.swap(Cx2);
    xsrc.swap(xs2);
    auto permute = [&](auto &v) {
      auto w = v;
      for (int32_t i = 0; i < m; ++i) w[size_t(np[size_t(i)])] = v[size_t(i)];
      v.swap(w);
    };
    permute(H.perm);
    permute(Dn);
    if (mp) permute(dsrc);
    permute(rphase);
    permute(rcomp);
    permute(rcsize);
    for (int32_t k = 0; k < m; ++k) H.pinv[size_t(H.perm[size_t(k)])] = k;
  };
  set_row_task();
  partition();
  relabel(newpos);
  if (allow_split && ntask > 1) {
    // Component starts, and the factor entries every row gathers from outside its component.
    std::vector<int32_t> cst(static_cast<size_t>(m));
    for (int32_t i = 0; i < m; ++i)
      cst[size_t(i)] = (i > 0 && row_task[size_t(i)] == row_task[size_t(i - 1)] &&
                        rphase[size_t(i)] == rphase[size_t(i - 1)] && rcsize[size_t(i)] > 1 &&
                        rcomp[size_t(i)] == rcomp[size_t(i - 1)])
                           ? cst[size_t(i - 1)]
                           : i;
    std::vector<int64_t> gext(static_cast<size_t>(m), 0);
    for (int32_t j = 0; j < m; ++j)
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p)
        if (j < cst[size_t(Ci[size_t(p)])]) gext[size_t(Ci[size_t(p)])]++;
    // Cost of the rows [a, b) (whole components): packed inverses plus gathered entries.
    auto rows_cost = [&](int32_t a, int32_t b) {
      int64_t e = 0;
      for (int32_t i = a; i < b; ++i) {
        e += gext[size_t(i)];
        if (cst[size_t(i)] == i && rcsize[size_t(i)] > 1) e += int64_t(rcsize[size_t(i)]) * (rcsize[size_t(i)] + 1) / 2;
      }
      return double(e) / kSolveThreads;
    };
    const double phase_overhead = 4.0;  // per-phase cost of the barriers, in entries per thread
    std::vector<double> tcost(static_cast<size_t>(ntask), 0.0), p0cost(static_cast<size_t>(ntask), 0.0);
    std::vector<int32_t> p0end(static_cast<size_t>(ntask));
    std::vector<double> group_costs;
    for (int32_t t = 0; t < ntask; ++t) {
      const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)];
      for (int32_t a = r0; a < r1;) {
        int32_t b = a;
        while (b < r1 && rphase[size_t(b)] == rphase[size_t(a)]) ++b;
        const double c = rows_cost(a, b) + phase_overhead;
        if (a == r0) { p0end[size_t(t)] = b; p0cost[size_t(t)] = c; }
        tcost[size_t(t)] += c;
        a = b;
      }
      if (rclass[size_t(H.perm[size_t(r0)])] == 0) group_costs.push_back(tcost[size_t(t)]);
    }
    double ref = 0.0;
    if (!group_costs.empty()) {
      std::nth_element(group_costs.begin(), group_costs.begin() + group_costs.size() / 2, group_costs.end());
      ref = group_costs[group_costs.size() / 2];
    }
    // Forward dependency depth of the tasks as they are.
    std::vector<int32_t> depth0(static_cast<size_t>(ntask), 0);
    for (int32_t j = 0; j < m; ++j)
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
        const int32_t ti = row_task[size_t(Ci[size_t(p)])], tj = row_task[size_t(j)];
        if (ti != tj) depth0[size_t(ti)] = std::max(depth0[size_t(ti)], depth0[size_t(tj)] + 1);
      }
    // Plan: parts of the first phase (cut at component boundaries, balanced by cost) and the
    // task that receives the later phases (-1: they stay a task of their own).
    std::vector<std::vector<int32_t>> cuts(static_cast<size_t>(ntask));
    std::vector<int32_t> dest(static_cast<size_t>(ntask), -1);
    std::vector<std::vector<int32_t>> front(static_cast<size_t>(ntask));
    bool any = false;
    for (int32_t t = 0; ref > 0.0 && t < ntask; ++t) {
      const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)];
      const int32_t o0 = H.perm[size_t(r0)];
      if (rclass[size_t(o0)] != 0 || (split_mode < 2 && tcost[size_t(t)] <= 1.5 * ref)) continue;
      const double target = split_mode >= 2 ? 0.5 * ref : ref;  // cost of one part
      const int32_t nparts = std::min<int32_t>(8, std::max<int32_t>(1, int32_t(std::ceil(p0cost[size_t(t)] / target))));
      if (nparts == 1 && p0end[size_t(t)] == r1) continue;
      const double total = rows_cost(r0, p0end[size_t(t)]);
      double acc = 0.0;
      int32_t k = 1;
      for (int32_t i = r0; i < p0end[size_t(t)];) {
        int32_t c1 = i + 1;
        while (c1 < p0end[size_t(t)] && cst[size_t(c1)] == i) ++c1;
        acc += rows_cost(i, c1);
        i = c1;
        if (k < nparts && i < p0end[size_t(t)] && acc >= total * k / nparts) { cuts[size_t(t)].push_back(i); ++k; }
      }
      cuts[size_t(t)].push_back(p0end[size_t(t)]);
      if (p0end[size_t(t)] < r1) {
        const int32_t g = rkey[size_t(o0)];
        for (int32_t u = t + 1; u < ntask; ++u) {
          const int32_t ou = H.perm[size_t(H.task_r0[size_t(u)])];
          if (rclass[size_t(ou)] == 1 && (rkey[size_t(ou)] == g || rkey[size_t(ou)] == g - 1)) { dest[size_t(t)] = u; break; }
        }
        // a coupling task deeper than 1 waits for another coupling task anyway: the later
        // phases then run as a task of their own beside that one, at no extra depth
        if (dest[size_t(t)] >= 0 && depth0[size_t(dest[size_t(t)])] >= 2) dest[size_t(t)] = -1;
        if (dest[size_t(t)] >= 0)
          for (int32_t r = p0end[size_t(t)]; r < r1; ++r) front[size_t(dest[size_t(t)])].push_back(r);
      }
      any = true;
    }
    if (any) {
      std::vector<int32_t> ord, nr0, nr1;
      ord.reserve(size_t(m));
      for (int32_t t = 0; t < ntask; ++t) {
        const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)];
        if (!cuts[size_t(t)].empty()) {
          int32_t a = r0;
          for (int32_t c : cuts[size_t(t)]) {
            nr0.push_back(int32_t(ord.size()));
            for (int32_t r = a; r < c; ++r) ord.push_back(r);
            nr1.push_back(int32_t(ord.size()));
            a = c;
          }
          if (dest[size_t(t)] < 0 && a < r1) {
            nr0.push_back(int32_t(ord.size()));
            for (int32_t r = a; r < r1; ++r) ord.push_back(r);
            nr1.push_back(int32_t(ord.size()));
          }
        } else {
          nr0.push_back(int32_t(ord.size()));
          for (int32_t r : front[size_t(t)]) ord.push_back(r);
          for (int32_t r = r0; r < r1; ++r) ord.push_back(r);
          nr1.push_back(int32_t(ord.size()));
        }
      }
      std::vector<int32_t> np(static_cast<size_t>(m));
      for (int32_t k = 0; k < m; ++k) np[size_t(ord[size_t(k)])] = k;
      bool topo = int32_t(ord.size()) == m;
      for (int32_t j = 0; topo && j < m; ++j)
        for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p)
          if (np[size_t(Ci[size_t(p)])] <= np[size_t(j)]) { topo = false; break; }
      if (topo) {  // else the split would need a refactorization: keep the tasks as they are
        relabel(np);
        H.task_r0.swap(nr0);
        H.task_r1.swap(nr1);
        set_row_task();
        partition();
        relabel(newpos);
      }
    }
  }
  H.D = Dn;
  // CSR of L (rows ascending columns) and of L^T, in the final order
  H.Lrp.assign(size_t(m) + 1, 0);
  H.Urp.assign(size_t(m) + 1, 0);
  for (int32_t j = 0; j < m; ++j)
    for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
      H.Lrp[size_t(Ci[size_t(p)]) + 1]++;
      H.Urp[size_t(j) + 1]++;
    }
  for (int32_t i = 0; i < m; ++i) { H.Lrp[size_t(i) + 1] += H.Lrp[size_t(i)]; H.Urp[size_t(i) + 1] += H.Urp[size_t(i)]; }
  H.Lci.resize(size_t(nnzL)); H.Lv.resize(size_t(nnzL));
  H.Uci.resize(size_t(nnzL)); H.Uv.resize(size_t(nnzL));
  {
    std::vector<int64_t> lsrc(mp ? size_t(nnzL) : 0), usrc(mp ? size_t(nnzL) : 0);
    std::vector<int64_t> fl(H.Lrp.begin(), H.Lrp.end() - 1), fu(H.Urp.begin(), H.Urp.end() - 1);
    for (int32_t j = 0; j < m; ++j)
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
        const int32_t ni = Ci[size_t(p)], nj = j;
        const int64_t ql = fl[size_t(ni)]++, qu = fu[size_t(nj)]++;
        H.Lci[size_t(ql)] = nj; H.Lv[size_t(ql)] = Cx[size_t(p)];
        H.Uci[size_t(qu)] = ni; H.Uv[size_t(qu)] = Cx[size_t(p)];
        if (mp) { lsrc[size_t(ql)] = xsrc[size_t(p)]; usrc[size_t(qu)] = xsrc[size_t(p)]; }
      }
    // rows by ascending column (the column indices of a row are distinct); sources follow
    auto sort_rows = [&](std::vector<int64_t> &rp, std::vector<int32_t> &ci, std::vector<double> &v,
                         std::vector<int64_t> &src, int32_t mm) {
      std::vector<std::pair<int32_t, int64_t>> tmp;
      std::vector<double> vv;
      for (int32_t i = 0; i < mm; ++i) {
        tmp.clear();
        vv.clear();
        for (int64_t p = rp[size_t(i)]; p < rp[size_t(i) + 1]; ++p) tmp.emplace_back(ci[size_t(p)], p);
        std::sort(tmp.begin(), tmp.end());
        for (auto &e : tmp) vv.push_back(v[size_t(e.second)]);
        std::vector<int64_t> ss;
        if (mp) for (auto &e : tmp) ss.push_back(src[size_t(e.second)]);
        int64_t q = rp[size_t(i)];
        for (size_t k = 0; k < tmp.size(); ++k, ++q) {
          ci[size_t(q)] = tmp[k].first;
          v[size_t(q)] = vv[k];
          if (mp) src[size_t(q)] = ss[k];
        }
      }
    };
    sort_rows(H.Lrp, H.Lci, H.Lv, lsrc, m);
    sort_rows(H.Urp, H.Uci, H.Uv, usrc, m);
    if (mp) { mp->lv_src.swap(lsrc); mp->uv_src.swap(usrc); mp->d_src = dsrc; }
  }
  for (int32_t i = 0; i < m; ++i)  // relabeling kept L lower triangular
    for (int64_t p = H.Lrp[size_t(i)]; p < H.Lrp[size_t(i) + 1]; ++p)
      if (H.Lci[size_t(p)] >= i) { err = "internal: relabeled factor not lower triangular"; return STROM_E_FACTOR; }
  Cp.clear(); Ci.clear(); Cx.clear();

  // ---------------------------------------------------------------- phase descriptors
  // Per phase: rows [ph_a, ph_b), of which the first ph_nns lie in components of two or
  // more rows.  Per row: its component [rcs, rce) and the offset rio of the component's
  // inverse (-1 for a single row).  The inverse of the component's unit lower-triangular
  // diagonal block of L is stored as a packed lower triangle, by rows in invR (row r at
  // r(r+1)/2) and by columns in invC (column c at c*n - c(c-1)/2), at the same offset.
  H.rcs.resize(size_t(m));
  H.rce.resize(size_t(m));
  H.rio.assign(size_t(m), -1);
  H.Lin.resize(size_t(m));
  H.Lend.resize(size_t(m));
  H.Ubeg.resize(size_t(m));
  std::vector<int32_t> fdepth(size_t(ntask), 0), bdepth(size_t(ntask), 0);
  for (int32_t t = 0; t < ntask; ++t) {
    const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)], nt = r1 - r0;
    H.max_task_rows = std::max(H.max_task_rows, nt);
    for (int32_t i = r0; i < r1; ++i)
      for (int64_t p = H.Lrp[size_t(i)]; p < H.Lrp[size_t(i) + 1]; ++p) {
        const int32_t j = H.Lci[size_t(p)];
        if (j < r0) fdepth[size_t(t)] = std::max(fdepth[size_t(t)], fdepth[size_t(row_task[size_t(j)])] + 1);
      }
    H.task_ph0.push_back(int32_t(H.ph_a.size()));
    int32_t a = r0;
    while (a < r1) {
      int32_t b = a;
      while (b < r1 && rphase[size_t(b)] == rphase[size_t(a)]) ++b;
      int32_t nns = 0;
      int64_t mf = 0, mb = 0;
      int32_t c0 = a;
      while (c0 < b) {  // components: runs of equal rcomp
        int32_t c1 = c0;
        while (c1 < b && rcomp[size_t(c1)] == rcomp[size_t(c0)]) ++c1;
        const int32_t cn = c1 - c0;
        int64_t io = -1;
        if (cn > 1) {
          nns += cn;
          for (int32_t i = c0; i < c1; ++i)
            for (int64_t p = H.Lrp[size_t(i)]; p < H.Lrp[size_t(i) + 1]; ++p) {
              const int32_t j = H.Lci[size_t(p)];
              if (j < c0 && j >= a) { err = "internal: dependency between components of a phase"; return STROM_E_FACTOR; }
            }
          std::vector<double> blk, inv;
          component_inverse(H, c0, c1, blk, inv);
          io = int64_t(H.invR.size());
          for (int32_t i = 0; i < cn; ++i)
            for (int32_t j = 0; j <= i; ++j) H.invR.push_back(inv[size_t(i) * cn + size_t(j)]);
          for (int32_t j = 0; j < cn; ++j)
            for (int32_t i = j; i < cn; ++i) H.invC.push_back(inv[size_t(i) * cn + size_t(j)]);
        }
        for (int32_t i = c0; i < c1; ++i) {
          H.rcs[size_t(i)] = c0;
          H.rce[size_t(i)] = c1;
          H.rio[size_t(i)] = io;
          int64_t q = H.Lrp[size_t(i)];
          while (q < H.Lrp[size_t(i) + 1] && H.Lci[size_t(q)] < r0) ++q;
          H.Lin[size_t(i)] = q;
          while (q < H.Lrp[size_t(i) + 1] && H.Lci[size_t(q)] < a) ++q;
          H.Lend[size_t(i)] = q;
          int64_t u = H.Urp[size_t(i)];
          while (u < H.Urp[size_t(i) + 1] && H.Uci[size_t(u)] < c1) ++u;
          H.Ubeg[size_t(i)] = u;
          mb = std::max(mb, H.Urp[size_t(i) + 1] - u);
        }
        c0 = c1;
      }
      for (int32_t i = a; i < b; ++i) mf = std::max(mf, H.Lend[size_t(i)] - H.Lin[size_t(i)]);
      H.ph_a.push_back(a);
      H.ph_b.push_back(b);
      H.ph_nns.push_back(nns);
      H.ph_gf.push_back(lanes_for(mf));
      H.ph_gb.push_back(lanes_for(mb));
      H.max_phase_nns = std::max(H.max_phase_nns, nns);
      a = b;
    }
    H.task_ph1.push_back(int32_t(H.ph_a.size()));
  }

  // ---------------------------------------------------------------- push segments
  // The forward entries of row i in columns of other tasks, [Lrp[i], Lin[i]), are split by
  // the owner task of the columns; each run is one segment, summed by its owner.
  H.sptr.assign(size_t(m) + 1, 0);
  std::vector<std::vector<int32_t>> owned(static_cast<size_t>(ntask));
  std::vector<int64_t> seg_max(static_cast<size_t>(ntask), 0);
  for (int32_t i = 0; i < m; ++i) {
    int64_t p = H.Lrp[size_t(i)];
    const int64_t q = H.Lin[size_t(i)];
    while (p < q) {
      const int32_t ot = row_task[size_t(H.Lci[size_t(p)])];
      int64_t pe = p;
      while (pe < q && row_task[size_t(H.Lci[size_t(pe)])] == ot) ++pe;
      owned[size_t(ot)].push_back(int32_t(H.seg_pb.size()));
      seg_max[size_t(ot)] = std::max(seg_max[size_t(ot)], pe - p);
      H.seg_pb.push_back(p);
      H.seg_pe.push_back(pe);
      p = pe;
    }
    H.sptr[size_t(i) + 1] = int64_t(H.seg_pb.size());
  }
  if (int64_t(H.seg_pb.size()) >= int64_t(kPartFlag)) {
    err = "too many push segments";
    return STROM_E_INVAL;
  }
  // the row gathers also sum their segments: widen the phase lanes by the segment count
  for (size_t ph = 0; ph < H.ph_a.size(); ++ph) {
    int64_t mf = 0;
    for (int32_t i = H.ph_a[ph]; i < H.ph_b[ph]; ++i)
      mf = std::max(mf, H.Lend[size_t(i)] - H.Lin[size_t(i)] + H.sptr[size_t(i) + 1] - H.sptr[size_t(i)]);
    H.ph_gf[ph] = lanes_for(mf);
  }
  H.push_off.assign(1, 0);
  for (size_t sg = 0; sg < H.seg_pb.size(); ++sg) {
    for (int64_t p = H.seg_pb[sg]; p < H.seg_pe[sg]; ++p) {
      H.push_ci.push_back(H.Lci[size_t(p)]);
      H.push_v.push_back(H.Lv[size_t(p)]);
      if (mp) mp->push_src.push_back(p);
    }
    H.push_off.push_back(int64_t(H.push_ci.size()));
  }
  H.tsptr.assign(1, 0);
  for (int32_t t = 0; t < ntask; ++t) {
    H.tseg.insert(H.tseg.end(), owned[size_t(t)].begin(), owned[size_t(t)].end());
    H.tsptr.push_back(int32_t(H.tseg.size()));
    H.task_sg.push_back(std::min<int32_t>(16, lanes_for(seg_max[size_t(t)])));
  }

  // ---------------------------------------------------------------- task-local staging
  int64_t max_stage = kMaxLdsTaskRows;  // STROM_STAGE_ROWS lowers it (0: every task in place)
  if (const char *ev = std::getenv("STROM_STAGE_ROWS")) {
    const long v = std::strtol(ev, nullptr, 10);
    if (v >= 0 && v < max_stage) max_stage = v;
  }
  H.task_pin.assign(size_t(ntask) + 1, 0);
  H.task_xoff.assign(size_t(ntask) + 1, 0);
  H.task_inl.assign(size_t(ntask), 0);
  std::vector<int32_t> ph_task(H.ph_a.size());
  for (int32_t t = 0; t < ntask; ++t) {
    const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)], nt = r1 - r0;
    for (int32_t ph = H.task_ph0[size_t(t)]; ph < H.task_ph1[size_t(t)]; ++ph) ph_task[size_t(ph)] = t;
    H.task_pin[size_t(t)] = int32_t(H.sptr[size_t(r0)]);
    H.task_pin[size_t(t) + 1] = int32_t(H.sptr[size_t(r1)]);
    std::vector<int32_t> ext;
    for (int32_t i = r0; i < r1; ++i)
      for (int64_t p = H.Ubeg[size_t(i)]; p < H.Urp[size_t(i) + 1]; ++p)
        if (H.Uci[size_t(p)] >= r1) ext.push_back(H.Uci[size_t(p)]);
    std::sort(ext.begin(), ext.end());
    ext.erase(std::unique(ext.begin(), ext.end()), ext.end());
    const int64_t stage = int64_t(nt) + std::max<int64_t>(H.sptr[size_t(r1)] - H.sptr[size_t(r0)], int64_t(ext.size()));
    if (stage <= max_stage) {
      H.task_inl[size_t(t)] = 1;
      H.max_task_stage = std::max(H.max_task_stage, int32_t(stage));
      H.task_xrow.insert(H.task_xrow.end(), ext.begin(), ext.end());
    }
    H.task_xoff[size_t(t) + 1] = int64_t(H.task_xrow.size());
  }

  // ---------------------------------------------------------------- phase streams
  // Every phase is solved from four entry streams.  The entries of the phase's rows (in row
  // order; a row with no entry gets one zero entry) are cut into Tp equal slices of K
  // entries (Tp <= kSolveThreads a multiple of 64, K a multiple of kStreamBatch, as few slices as
  // cover the phase), slice t for thread t, entry k of it at off + k * Tp + t so that every
  // load of a wave is contiguous.  A row may span several slices; its pieces are added in
  // slice order.  An entry is a value and an index; the index of the last entry of a row
  // carries kLastFlag.  s_ra holds per thread the phase-relative row of its first entry,
  // with kStartFlag when that entry starts the row.  Streams:
  //   fg: forward gather, the row's pushed partial sums (value 1) and L(i, j) for own-task
  //       columns j of earlier phases;
  //   fi: forward inverse, row i of its component's inverse (index: position in the phase
  //       right-hand side buffer);
  //   bg: backward gather, L(i, j) for rows i after the row's component;
  //   bi: backward inverse, column j of its component's inverse (index as fi);
  //   push (kind 4, per task): the task's push segments as rows.
  // fg / bg / push indices are task-local for a task staged in LDS (see task_inl), else the row
  // (and s | kPartFlag for the partial sum s).
  {
    const int32_t T = kSolveThreads;
    // Lays out the entries of nrows rows (row r's entries contiguous, the last one flagged) as
    // the stream of one phase (or task) of the given kind.
    // value codes of the stream entries (see NumericMaps): factor entry p of L (p) or of L^T
    // (nnzL + p), packed inverse entry r by rows (2 nnzL + r) or by columns (2 nnzL + ninv + r)
    const int64_t c_uv = nnzL, c_ir = 2 * nnzL, c_ic = 2 * nnzL + int64_t(H.invR.size());
    std::vector<int64_t> esrc;  // code of each entry of the current phase (with mp)
    auto emit = [&](const std::vector<std::pair<int32_t, double>> &ent, const std::vector<int32_t> &erow,
                    const std::vector<char> &efirst, int32_t nrows, int kind, int32_t pad_idx) {
      const int64_t E = int64_t(ent.size());
      int64_t K = kStreamBatch;
      int32_t Tp = int32_t(std::min<int64_t>(T, (E + K - 1) / K));
      if (int64_t(Tp) * K < E) K = ((E + Tp - 1) / Tp + kStreamBatch - 1) / kStreamBatch * kStreamBatch;
      Tp = std::min<int32_t>(T, std::max<int32_t>(64, (Tp + 63) / 64 * 64));
      std::vector<int32_t> ra(size_t(T) + 1, nrows);
      std::vector<double> &V = H.sval[size_t(kind)];
      std::vector<int32_t> &X = H.sidx[size_t(kind)];
      const int64_t off = int64_t(V.size());
      V.resize(size_t(off + K * Tp), 0.0);
      X.resize(size_t(off + K * Tp), pad_idx);
      if (mp) mp->s_src[size_t(kind)].resize(size_t(off + K * Tp), -1);
      for (int32_t t = 0; t < Tp; ++t) {
        const int64_t e0 = int64_t(t) * K;
        if (e0 < E) ra[size_t(t)] = erow[size_t(e0)] | (efirst[size_t(e0)] ? kStartFlag : 0);
      }
      // entry k of slice t (entry t K + k of the phase) at off + k Tp + t, written in
      // destination order so that the stores run contiguously
      for (int64_t k = 0; k < K; ++k) {
        double *vd = V.data() + off + k * Tp;
        int32_t *xd = X.data() + off + k * Tp;
        for (int32_t t = 0; t < Tp; ++t) {
          const int64_t e = int64_t(t) * K + k;
          if (e >= E) break;  // later slices hold no more entries
          vd[t] = ent[size_t(e)].second;
          xd[t] = ent[size_t(e)].first;
          if (mp) mp->s_src[size_t(kind)][size_t(off + k * Tp + t)] = esrc[size_t(e)];
        }
      }
      H.s_off[size_t(kind)].push_back(off);
      H.s_K[size_t(kind)].push_back(int32_t(K));
      H.s_T[size_t(kind)].push_back(Tp);
      H.s_ra[size_t(kind)].insert(H.s_ra[size_t(kind)].end(), ra.begin(), ra.end());
    };
    auto build = [&](int32_t ph, int32_t rbeg, int32_t rend, int kind) {
      const int32_t t = ph_task[size_t(ph)], r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)];
      const bool inl = H.task_inl[size_t(t)] != 0;
      const int32_t *xr = H.task_xrow.data() + H.task_xoff[size_t(t)];
      const int64_t nx = H.task_xoff[size_t(t) + 1] - H.task_xoff[size_t(t)];
      auto fidx = [&](int32_t j) { return inl ? j - r0 : j; };
      auto bidx = [&](int32_t i) {
        if (!inl) return i;
        if (i < r1) return i - r0;
        return (r1 - r0) + int32_t(std::lower_bound(xr, xr + nx, i) - xr);
      };
      const int32_t pad_idx = (kind == 0 || kind == 2) ? (inl ? rbeg - r0 : rbeg) : 0;
      std::vector<std::pair<int32_t, double>> ent;  // the whole phase, rows in order
      std::vector<int32_t> erow;                    // phase-relative row of each entry
      std::vector<char> efirst;                     // entry starts its row
      esrc.clear();
      auto put = [&](int32_t idx, double v, int64_t code) {
        ent.emplace_back(idx, v);
        if (mp) esrc.push_back(code);
      };
      for (int32_t i = rbeg; i < rend; ++i) {
        const size_t e0 = ent.size();
        if (kind == 0) {
          for (int64_t q = H.sptr[size_t(i)]; q < H.sptr[size_t(i) + 1]; ++q)
            put(inl ? (r1 - r0) + int32_t(q - H.task_pin[size_t(t)]) : (int32_t(q) | kPartFlag), 1.0, -2);
          for (int64_t p = H.Lin[size_t(i)]; p < H.Lend[size_t(i)]; ++p) put(fidx(H.Lci[size_t(p)]), H.Lv[size_t(p)], p);
        } else if (kind == 2) {
          for (int64_t p = H.Ubeg[size_t(i)]; p < H.Urp[size_t(i) + 1]; ++p)
            put(bidx(H.Uci[size_t(p)]), H.Uv[size_t(p)], c_uv + p);
        } else {
          const int32_t cs = H.rcs[size_t(i)], cn = H.rce[size_t(i)] - cs, kk = i - cs;
          const int32_t base = cs - H.ph_a[size_t(ph)];
          if (kind == 1)
            for (int32_t j = 0; j <= kk; ++j) {
              const int64_t r = H.rio[size_t(i)] + int64_t(kk) * (kk + 1) / 2 + j;
              put(base + j, H.invR[size_t(r)], c_ir + r);
            }
          else
            for (int32_t e = 0; e < cn - kk; ++e) {
              const int64_t r = H.rio[size_t(i)] + int64_t(kk) * cn - int64_t(kk) * (kk - 1) / 2 + e;
              put(base + kk + e, H.invC[size_t(r)], c_ic + r);
            }
        }
        if (ent.size() == e0) put(pad_idx, 0.0, -1);
        ent.back().first |= kLastFlag;
        for (size_t e = e0; e < ent.size(); ++e) {
          erow.push_back(i - rbeg);
          efirst.push_back(e == e0);
        }
      }
      emit(ent, erow, efirst, rend - rbeg, kind, pad_idx);
    };
    for (size_t ph = 0; ph < H.ph_a.size(); ++ph) {
      const int32_t a = H.ph_a[ph], b = H.ph_b[ph], nns = H.ph_nns[ph];
      build(int32_t(ph), a, b, 0);
      build(int32_t(ph), a, a + nns, 1);
      build(int32_t(ph), a, b, 2);
      build(int32_t(ph), a, a + nns, 3);
    }
    // kind 4, one stream per task: its push segments (rows: the segments tseg[tsptr[t] ..] in
    // order; entries: the factor entries of the segment, index of the column as in fg)
    for (int32_t t = 0; t < ntask; ++t) {
      const int32_t r0 = H.task_r0[size_t(t)];
      const bool inl = H.task_inl[size_t(t)] != 0;
      std::vector<std::pair<int32_t, double>> ent;
      std::vector<int32_t> erow;
      std::vector<char> efirst;
      const int32_t nseg = H.tsptr[size_t(t) + 1] - H.tsptr[size_t(t)];
      esrc.clear();
      for (int32_t r = 0; r < nseg; ++r) {
        const int32_t sg = H.tseg[size_t(H.tsptr[size_t(t)] + r)];
        const size_t e0 = ent.size();
        for (int64_t e = H.push_off[size_t(sg)]; e < H.push_off[size_t(sg) + 1]; ++e) {
          ent.emplace_back(inl ? H.push_ci[size_t(e)] - r0 : H.push_ci[size_t(e)], H.push_v[size_t(e)]);
          if (mp) esrc.push_back(mp->push_src[size_t(e)]);
        }
        if (ent.size() == e0) {
          ent.emplace_back(inl ? 0 : r0, 0.0);
          if (mp) esrc.push_back(-1);
        }
        ent.back().first |= kLastFlag;
        for (size_t e = e0; e < ent.size(); ++e) {
          erow.push_back(r);
          efirst.push_back(e == e0);
        }
      }
      emit(ent, erow, efirst, nseg, 4, inl ? 0 : r0);
    }
  }

  // ---------------------------------------------------------------- launch schedule
  for (int32_t t = ntask - 1; t >= 0; --t) {
    const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)];
    for (int32_t j = r0; j < r1; ++j)
      for (int64_t p = H.Urp[size_t(j)]; p < H.Urp[size_t(j) + 1]; ++p) {
        const int32_t i = H.Uci[size_t(p)];
        if (i >= r1) bdepth[size_t(t)] = std::max(bdepth[size_t(t)], bdepth[size_t(row_task[size_t(i)])] + 1);
      }
  }
  auto group_by = [&](const std::vector<int32_t> &depth, std::vector<int32_t> &order, std::vector<int32_t> &gptr) {
    const int32_t maxd = ntask ? *std::max_element(depth.begin(), depth.end()) : 0;
    order.clear();
    gptr.assign(1, 0);
    for (int32_t d = 0; d <= maxd; ++d) {
      for (int32_t t = 0; t < ntask; ++t)
        if (depth[size_t(t)] == d) order.push_back(t);
      gptr.push_back(int32_t(order.size()));
    }
  };
  group_by(fdepth, H.fwd_order, H.fwd_gptr);
  group_by(bdepth, H.bwd_order, H.bwd_gptr);
  (void)task_nph;
  return STROM_OK;
}

// The numbers of an analysis for new values of A on the pattern the maps were made for: A^T,
// K and its factor in the same order with the same arithmetic, then every value derived from
// the factor through the maps.  H holds the cached analysis on entry.
strom_status refresh_numeric(const NumericMaps &mp, int32_t m, const int64_t *rowptr, const int32_t *col,
                             const double *val, double eps_reg, HostAnalysis &H, std::string &err) {
  const int64_t nnz = rowptr[m];
  for (int64_t p = 0; p < nnz; ++p)
    if (!std::isfinite(val[p])) { err = "non-finite value in A"; return STROM_E_INVAL; }
  for (size_t q = 0; q < mp.at_src.size(); ++q) H.Atv[q] = val[mp.at_src[q]];
  std::vector<int64_t> Kp;
  std::vector<int32_t> Ki;
  std::vector<double> Kx;
  const double maxdiag = assemble_K(m, rowptr, col, val, mp.perm0, mp.pinv0, H, Kp, Ki, Kx);
  H.eps = (eps_reg > 0 ? eps_reg : 1e-12) * (maxdiag > 0 ? maxdiag : 1.0);
  for (int32_t j = 0; j < m; ++j) Kx[size_t(Kp[size_t(j)])] += H.eps;
  std::vector<double> Cx, Dn;
  const strom_status fst = numeric_factor(m, Kp, Ki, Kx, mp.Cp0, mp.Ci0, mp.tr0, mp.tr1, Cx, Dn, err);
  if (fst != STROM_OK) return fst;
  for (size_t p = 0; p < mp.lv_src.size(); ++p) H.Lv[p] = Cx[size_t(mp.lv_src[p])];
  for (size_t p = 0; p < mp.uv_src.size(); ++p) H.Uv[p] = Cx[size_t(mp.uv_src[p])];
  for (int32_t i = 0; i < m; ++i) H.D[size_t(i)] = Dn[size_t(mp.d_src[size_t(i)])];
  std::vector<double> blk, inv;
  for (int32_t i = 0; i < m; ++i) {  // components of two or more rows, at their first row
    if (H.rcs[size_t(i)] != i || H.rio[size_t(i)] < 0) continue;
    const int32_t c0 = i, c1 = H.rce[size_t(i)], cn = c1 - c0;
    component_inverse(H, c0, c1, blk, inv);
    int64_t o = H.rio[size_t(i)];
    for (int32_t r = 0; r < cn; ++r)
      for (int32_t c = 0; c <= r; ++c) H.invR[size_t(o++)] = inv[size_t(r) * cn + size_t(c)];
    o = H.rio[size_t(i)];
    for (int32_t c = 0; c < cn; ++c)
      for (int32_t r = c; r < cn; ++r) H.invC[size_t(o++)] = inv[size_t(r) * cn + size_t(c)];
  }
  for (size_t e = 0; e < mp.push_src.size(); ++e) H.push_v[e] = H.Lv[size_t(mp.push_src[e])];
  const int64_t nnzL = int64_t(H.Lv.size()), ninv = int64_t(H.invR.size());
  for (int k = 0; k < kStreamKinds; ++k) {
    const std::vector<int64_t> &src = mp.s_src[size_t(k)];
    std::vector<double> &V = H.sval[size_t(k)];
    for (size_t e = 0; e < src.size(); ++e) {
      const int64_t c = src[e];
      V[e] = c == -1 ? 0.0 : c == -2 ? 1.0 : c < nnzL ? H.Lv[size_t(c)] : c < 2 * nnzL ? H.Uv[size_t(c - nnzL)]
             : c < 2 * nnzL + ninv ? H.invR[size_t(c - 2 * nnzL)] : H.invC[size_t(c - 2 * nnzL - ninv)];
    }
  }
  return STROM_OK;
}

// Cache of analyses by sparsity pattern and schedule options (LRU, bounded by memory): a hit
// copies the cached analysis and refreshes its numbers.  A pattern is cached on its second
// analysis (recording the maps costs about half an analysis), so one-off instances pay
// nothing.  STROM_SETUP_CACHE=0 turns it off.
struct CacheEntry {
  std::vector<int32_t> bsize;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  double eps_reg = 0;
  int split_mode = 0, block_rows = 0;
  std::string env;  // schedule knobs read from the environment by the analysis
  HostAnalysis H;
  NumericMaps maps;
  size_t bytes = 0;
};

struct SetupCache {
  std::mutex mu;
  std::list<std::shared_ptr<const CacheEntry>> lru;  // most recent first
  size_t bytes = 0;
  std::vector<uint64_t> seen;  // keys of patterns analysed once (cached on their second analysis)
};

SetupCache &setup_cache() {
  static SetupCache c;
  return c;
}

constexpr size_t kCacheBytes = size_t(6) << 30;

template <class T>
size_t vbytes(const std::vector<T> &v) { return v.size() * sizeof(T); }

size_t entry_bytes(const CacheEntry &e) {
  const HostAnalysis &H = e.H;
  size_t b = vbytes(e.rowptr) + vbytes(e.col) + vbytes(H.Atci) + vbytes(H.Atv) + vbytes(H.Lci) + vbytes(H.Lv) +
             vbytes(H.Uci) + vbytes(H.Uv) + vbytes(H.invR) + vbytes(H.invC) + vbytes(H.push_ci) + vbytes(H.push_v) +
             vbytes(e.maps.at_src) + vbytes(e.maps.Ci0) + vbytes(e.maps.lv_src) + vbytes(e.maps.uv_src) +
             vbytes(e.maps.push_src);
  for (int k = 0; k < kStreamKinds; ++k)
    b += vbytes(H.sval[size_t(k)]) + vbytes(H.sidx[size_t(k)]) + vbytes(e.maps.s_src[size_t(k)]);
  return b;
}

std::string env_knobs() {
  std::string s;
  for (const char *name : {"STROM_STAGE_ROWS", "STROM_TASK_SPLIT", "STROM_BLOCK_ROWS", "STROM_TOP_LEVELS", "STROM_ROW_ORDER"}) {
    const char *v = std::getenv(name);
    s += std::string(name) + "=" + (v ? v : "") + ";";
  }
  return s;
}

// H = src with the large arrays copied by parallel threads (first touches of fresh pages
// dominate a single-threaded copy of a few hundred MB).  Every field of HostAnalysis is listed
// here (the cache test compares them all).
void copy_analysis(const HostAnalysis &src, HostAnalysis &H) {
  std::vector<std::function<void()>> jobs;
  HostAnalysis &d = H;
  auto add = [&](auto member) { jobs.emplace_back([&src, &d, member] { d.*member = src.*member; }); };
  add(&HostAnalysis::Atci); add(&HostAnalysis::Atv); add(&HostAnalysis::Lci); add(&HostAnalysis::Lv);
  add(&HostAnalysis::Uci); add(&HostAnalysis::Uv); add(&HostAnalysis::invR); add(&HostAnalysis::invC);
  add(&HostAnalysis::push_ci); add(&HostAnalysis::push_v);
  for (int k = 0; k < kStreamKinds; ++k) {
    jobs.emplace_back([&src, &d, k] { d.sval[k] = src.sval[k]; });
    jobs.emplace_back([&src, &d, k] { d.sidx[k] = src.sidx[k]; });
  }
  // the small arrays and scalars: everything else
  HostAnalysis rest;
  {
    HostAnalysis &r = rest;
    r.m = src.m; r.nsvec = src.nsvec; r.nblocks = src.nblocks; r.bsize = src.bsize; r.boff = src.boff;
    r.Atrp = src.Atrp; r.perm = src.perm; r.pinv = src.pinv; r.eps = src.eps; r.Lrp = src.Lrp; r.Urp = src.Urp;
    r.D = src.D; r.task_r0 = src.task_r0; r.task_r1 = src.task_r1; r.task_ph0 = src.task_ph0;
    r.task_ph1 = src.task_ph1; r.ph_a = src.ph_a; r.ph_b = src.ph_b; r.ph_nns = src.ph_nns; r.ph_gf = src.ph_gf;
    r.ph_gb = src.ph_gb; r.rcs = src.rcs; r.rce = src.rce; r.rio = src.rio; r.Lin = src.Lin; r.Lend = src.Lend;
    r.Ubeg = src.Ubeg; r.sptr = src.sptr; r.seg_pb = src.seg_pb; r.seg_pe = src.seg_pe; r.tsptr = src.tsptr;
    r.tseg = src.tseg; r.task_sg = src.task_sg; r.push_off = src.push_off;
    for (int k = 0; k < kStreamKinds; ++k) {
      r.s_off[k] = src.s_off[k]; r.s_K[k] = src.s_K[k]; r.s_T[k] = src.s_T[k]; r.s_ra[k] = src.s_ra[k];
    }
    r.task_pin = src.task_pin; r.task_xoff = src.task_xoff; r.task_xrow = src.task_xrow; r.task_inl = src.task_inl;
    r.max_task_stage = src.max_task_stage; r.fwd_order = src.fwd_order; r.fwd_gptr = src.fwd_gptr;
    r.bwd_order = src.bwd_order; r.bwd_gptr = src.bwd_gptr; r.max_task_rows = src.max_task_rows;
    r.max_phase_nns = src.max_phase_nns; r.nnzL = src.nnzL;
  }
  H = std::move(rest);
  std::atomic<size_t> next(0);
  auto worker = [&] {
    for (size_t q; (q = next.fetch_add(1)) < jobs.size();) jobs[q]();
  };
  const size_t nth = std::min<size_t>(jobs.size(), std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  std::vector<std::thread> pool;
  for (size_t i = 1; i < nth; ++i) pool.emplace_back(worker);
  worker();
  for (auto &th : pool) th.join();
}

bool cache_on() {
  const char *v = std::getenv("STROM_SETUP_CACHE");
  return !(v && v[0] == '0');
}

// FNV-1a over the pattern, the options and the schedule knobs.
uint64_t pattern_hash(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr, const int32_t *col,
                      double eps_reg, int split_mode, int block_rows, const std::string &env) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  };
  mix(&nblocks, sizeof nblocks);
  mix(bsize, sizeof(int32_t) * size_t(nblocks));
  mix(&m, sizeof m);
  mix(rowptr, sizeof(int64_t) * size_t(m + 1));
  mix(col, sizeof(int32_t) * size_t(rowptr[m]));
  mix(&eps_reg, sizeof eps_reg);
  mix(&split_mode, sizeof split_mode);
  mix(&block_rows, sizeof block_rows);
  mix(env.data(), env.size());
  return h;
}

bool same_key(const CacheEntry &e, int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
              const int32_t *col, double eps_reg, int split_mode, int block_rows, const std::string &env) {
  if (int32_t(e.bsize.size()) != nblocks || int32_t(e.rowptr.size()) != m + 1 || e.eps_reg != eps_reg ||
      e.split_mode != split_mode || e.block_rows != block_rows || e.env != env)
    return false;
  if (std::memcmp(e.bsize.data(), bsize, sizeof(int32_t) * size_t(nblocks)) != 0) return false;
  if (std::memcmp(e.rowptr.data(), rowptr, sizeof(int64_t) * size_t(m + 1)) != 0) return false;
  return int64_t(e.col.size()) == rowptr[m] && std::memcmp(e.col.data(), col, sizeof(int32_t) * e.col.size()) == 0;
}

// Modelled y-solve time of a schedule, in stream entries: over the launch groups of both
// directions, the entries of the group's largest task (a launch lasts as long as its slowest
// workgroup; a task streams its phases' gathers and inverse blocks, and forward its pushes);
// with total set, the entries of every task (a merged batch fills its launches, so it pays
// for all of them).
int64_t modelled_solve_entries(const HostAnalysis &H, bool total) {
  auto task = [&](int32_t t, int k0, bool push) {
    int64_t e = push ? int64_t(H.s_K[4][size_t(t)]) * H.s_T[4][size_t(t)] : 0;
    for (int32_t p = H.task_ph0[size_t(t)]; p < H.task_ph1[size_t(t)]; ++p)
      for (int k = k0; k <= k0 + 1; ++k) e += int64_t(H.s_K[k][size_t(p)]) * H.s_T[k][size_t(p)];
    return e;
  };
  int64_t entries = 0;
  for (int dir = 0; dir < 2; ++dir) {
    const std::vector<int32_t> &gp = dir ? H.bwd_gptr : H.fwd_gptr, &ord = dir ? H.bwd_order : H.fwd_order;
    for (size_t g = 0; g + 1 < gp.size(); ++g) {
      int64_t mx = 0;
      int64_t sum = 0;
      for (int32_t i = gp[g]; i < gp[g + 1]; ++i) {
        const int64_t e = task(ord[size_t(i)], dir ? 2 : 0, dir == 0);
        mx = std::max(mx, e);
        sum += e;
      }
      entries += total ? sum : mx;
    }
  }
  return entries;
}

// Row order inside the groups' interior runs.  STROM_ROW_ORDER if set (0: the rows' own order,
// 1: minimum degree).  Else, up to kAutoOrderRows rows, both orders are analysed and the one
// whose schedule has the shorter modelled solve is kept: the longest path for the default
// schedule, the total stream entries for the throughput schedule of merged batches (task split
// of overweight tasks only, split mode 1: cart-pole N = 30 5.03 -> 4.41 M entries under
// minimum degree, its longest path 3% longer).  The choice is remembered per sparsity pattern
// and schedule options, so a pattern pays the second analysis once.  Larger problems keep
// their own order.
// Minimum degree cuts the fill of L by a third or more on every family, but the solve follows
// the largest task of each launch group, most often the one with the first clique (it carries
// the initial-state rows), and that one gains or loses with the family.  Measured on MI355X,
// y-solve per iteration: car N = 50 (bicycle) 1.27 -> 0.76 ms with minimum degree, the paper's
// cart-pole N = 30 2.51 -> 2.41 ms; cart-pole N = 30 0.475 -> 0.484 ms (so its own order is
// kept).  The flying robot at N = 60 (1.57M rows) models 14% longer under minimum degree.
constexpr int32_t kAutoOrderRows = 500000;

struct OrderMemo {
  std::mutex mu;
  std::vector<std::pair<uint64_t, bool>> choice;  // (pattern key, minimum degree), oldest first
};

OrderMemo &order_memo() {
  static OrderMemo o;
  return o;
}

strom_status analyze_full(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
                          const int32_t *col, const double *val, double eps_reg, HostAnalysis &H,
                          std::string &err, int split_mode, int block_rows, NumericMaps *mp) {
  if (const char *ev = std::getenv("STROM_ROW_ORDER"))
    return analyze_order(nblocks, bsize, m, rowptr, col, val, eps_reg, H, err, split_mode, block_rows, mp,
                         std::atoi(ev) != 0);
  bool csr_ok = nblocks > 0 && bsize && m > 0 && m <= kAutoOrderRows && rowptr && col && val && rowptr[0] == 0;
  for (int32_t i = 0; csr_ok && i < m; ++i) csr_ok = rowptr[i + 1] >= rowptr[i];
  if (!csr_ok)  // large, or invalid (the analysis reports it)
    return analyze_order(nblocks, bsize, m, rowptr, col, val, eps_reg, H, err, split_mode, block_rows, mp, false);
  const uint64_t key = pattern_hash(nblocks, bsize, m, rowptr, col, eps_reg, split_mode, block_rows, env_knobs());
  OrderMemo &M = order_memo();
  int known = -1;
  {
    std::lock_guard<std::mutex> lk(M.mu);
    for (const auto &c : M.choice)
      if (c.first == key) known = c.second;
  }
  if (known >= 0)
    return analyze_order(nblocks, bsize, m, rowptr, col, val, eps_reg, H, err, split_mode, block_rows, mp,
                         known != 0);
  // the two analyses share nothing but the inputs: the minimum-degree one runs in a thread of its own
  HostAnalysis H1;
  NumericMaps m1;
  std::string err1;
  strom_status rc1 = STROM_E_INVAL;
  std::thread other([&] {
    rc1 = analyze_order(nblocks, bsize, m, rowptr, col, val, eps_reg, H1, err1, split_mode, block_rows,
                        mp ? &m1 : nullptr, true);
  });
  const strom_status rc =
      analyze_order(nblocks, bsize, m, rowptr, col, val, eps_reg, H, err, split_mode, block_rows, mp, false);
  other.join();
  if (rc != STROM_OK) return rc;
  int mode = split_mode;  // the split mode the analysis resolves (see analyze_instance)
  if (mode < 0) {
    mode = 2;
    if (const char *ev = std::getenv("STROM_TASK_SPLIT")) mode = int(std::strtol(ev, nullptr, 10));
  }
  const bool total = mode == 1;
  const bool md = rc1 == STROM_OK && modelled_solve_entries(H1, total) < modelled_solve_entries(H, total);
  if (md) {
    H = std::move(H1);
    if (mp) *mp = std::move(m1);
  }
  std::lock_guard<std::mutex> lk(M.mu);
  M.choice.emplace_back(key, md);
  if (M.choice.size() > 4096) M.choice.erase(M.choice.begin());
  return STROM_OK;
}
}  // namespace

strom_status analyze_instance(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
                              const int32_t *col, const double *val, double eps_reg, HostAnalysis &H,
                              std::string &err, int split_mode, int block_rows) {
  if (!cache_on() || nblocks <= 0 || !bsize || m <= 0 || !rowptr || !col || !val || m >= kPartFlag || rowptr[0] != 0)
    return analyze_full(nblocks, bsize, m, rowptr, col, val, eps_reg, H, err, split_mode, block_rows, nullptr);
  const std::string env = env_knobs();
  SetupCache &C = setup_cache();
  std::shared_ptr<const CacheEntry> hit;
  {
    std::lock_guard<std::mutex> lk(C.mu);
    for (auto it = C.lru.begin(); it != C.lru.end(); ++it)
      if (same_key(**it, nblocks, bsize, m, rowptr, col, eps_reg, split_mode, block_rows, env)) {
        hit = *it;
        C.lru.splice(C.lru.begin(), C.lru, it);
        break;
      }
  }
  if (hit) {
    copy_analysis(hit->H, H);
    return refresh_numeric(hit->maps, m, rowptr, col, val, eps_reg, H, err);
  }
  // a pattern's first analysis runs plain; its second records the maps and fills the cache
  const uint64_t key = pattern_hash(nblocks, bsize, m, rowptr, col, eps_reg, split_mode, block_rows, env);
  {
    std::lock_guard<std::mutex> lk(C.mu);
    if (std::find(C.seen.begin(), C.seen.end(), key) == C.seen.end()) {
      C.seen.push_back(key);
      if (C.seen.size() > 4096) C.seen.erase(C.seen.begin());
      hit = nullptr;
    } else {
      hit = std::make_shared<const CacheEntry>();  // marker: seen before
    }
  }
  if (!hit) return analyze_full(nblocks, bsize, m, rowptr, col, val, eps_reg, H, err, split_mode, block_rows, nullptr);
  auto e = std::make_shared<CacheEntry>();
  const strom_status rc =
      analyze_full(nblocks, bsize, m, rowptr, col, val, eps_reg, H, err, split_mode, block_rows, &e->maps);
  if (rc != STROM_OK) return rc;
  e->bsize.assign(bsize, bsize + nblocks);
  e->rowptr.assign(rowptr, rowptr + m + 1);
  e->col.assign(col, col + rowptr[m]);
  e->eps_reg = eps_reg;
  e->split_mode = split_mode;
  e->block_rows = block_rows;
  e->env = env;
  copy_analysis(H, e->H);
  e->bytes = entry_bytes(*e);
  if (e->bytes > kCacheBytes / 2) return STROM_OK;  // too large to keep
  std::lock_guard<std::mutex> lk(C.mu);
  for (auto &x : C.lru)
    if (same_key(*x, nblocks, bsize, m, rowptr, col, eps_reg, split_mode, block_rows, env)) return STROM_OK;
  C.lru.push_front(e);
  C.bytes += e->bytes;
  while (C.bytes > kCacheBytes && C.lru.size() > 1) {
    C.bytes -= C.lru.back()->bytes;
    C.lru.pop_back();
  }
  return STROM_OK;
}

}  // namespace strom
