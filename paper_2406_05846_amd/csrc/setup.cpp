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
//    one task, solved by one workgroup.  Inside a task the rows are relabeled in order of
//    their dependency level (a topological order, so the relabeled L is the factor of the
//    relabeled matrix and nothing is refactored).  Wide levels become level phases (the
//    rows of a level are independent); runs of narrow levels become dense phases of at most
//    kMaxDenseRows rows, solved through the explicit inverse of their unit lower-triangular
//    diagonal block.  Tasks are launched by dependency depth, computed from L.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "strom_internal.h"

namespace strom {
namespace {

// Nested-dissection post-order of the chain positions [lo, hi].
void chain_nd(int lo, int hi, std::vector<int> &out) {
  if (lo > hi) return;
  const int mid = lo + (hi - lo) / 2;
  chain_nd(lo, mid - 1, out);
  chain_nd(mid + 1, hi, out);
  out.push_back(mid);
}

// Lanes per row for a gather of up to `len` entries.
int32_t lanes_for(int64_t len) {
  int32_t g = 1;
  while (g < 64 && int64_t(g) * 4 < len) g *= 2;
  return g;
}

}  // namespace

strom_status analyze_instance(int32_t nblocks, const int32_t *bsize, int32_t m, const int64_t *rowptr,
                              const int32_t *col, const double *val, double eps_reg, HostAnalysis &H,
                              std::string &err) {
  // ---------------------------------------------------------------- validation
  if (nblocks <= 0 || !bsize || m <= 0 || !rowptr || !col || !val) {
    err = "empty problem or NULL array";
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
  {
    std::vector<int64_t> fill(H.Atrp.begin(), H.Atrp.end() - 1);
    for (int32_t i = 0; i < m; ++i)
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int64_t q = fill[size_t(col[p])]++;
        H.Atci[size_t(q)] = i;
        H.Atv[size_t(q)] = val[p];
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
  std::vector<int> sep_pos;
  chain_nd(0, std::max(0, ngroups - 2), sep_pos);
  std::vector<int32_t> sep_rank(static_cast<size_t>(std::max(1, ngroups)), 0);
  for (size_t r = 0; r < sep_pos.size(); ++r) sep_rank[size_t(sep_pos[r])] = int32_t(r);
  H.perm.resize(size_t(m));
  std::iota(H.perm.begin(), H.perm.end(), 0);
  std::stable_sort(H.perm.begin(), H.perm.end(), [&](int32_t a, int32_t b) {
    if (rclass[size_t(a)] != rclass[size_t(b)]) return rclass[size_t(a)] < rclass[size_t(b)];
    if (rclass[size_t(a)] == 0) return rkey[size_t(a)] < rkey[size_t(b)];
    if (rclass[size_t(a)] == 1) return sep_rank[size_t(rkey[size_t(a)])] < sep_rank[size_t(rkey[size_t(b)])];
    return false;
  });
  H.pinv.resize(size_t(m));
  for (int32_t k = 0; k < m; ++k) H.pinv[size_t(H.perm[size_t(k)])] = k;

  // task ranges: maximal runs of rows with the same (class, key)
  {
    int32_t r0 = 0;
    for (int32_t k = 1; k <= m; ++k) {
      const bool brk = (k == m) || rclass[size_t(H.perm[size_t(k)])] != rclass[size_t(H.perm[size_t(r0)])] ||
                       rkey[size_t(H.perm[size_t(k)])] != rkey[size_t(H.perm[size_t(r0)])];
      if (brk) { H.task_r0.push_back(r0); H.task_r1.push_back(k); r0 = k; }
    }
  }

  // ---------------------------------------------------------------- K = P A A^* P^T (lower)
  std::vector<int64_t> Kp(size_t(m) + 1, 0);
  std::vector<int32_t> Ki;
  std::vector<double> Kx;
  double maxdiag = 0.0;
  {
    std::vector<double> acc(size_t(m), 0.0);
    std::vector<int32_t> seen(size_t(m), -1), list;
    Ki.reserve(size_t(nnz) * 6);
    Kx.reserve(size_t(nnz) * 6);
    for (int32_t j = 0; j < m; ++j) {  // column j of the lower triangle (new order)
      const int32_t oj = H.perm[size_t(j)];
      list.clear();
      for (int64_t p = rowptr[oj]; p < rowptr[oj + 1]; ++p) {
        const int32_t c = col[p];
        for (int64_t q = H.Atrp[size_t(c)]; q < H.Atrp[size_t(c) + 1]; ++q) {
          const int32_t ni = H.pinv[size_t(H.Atci[size_t(q)])];
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
  }
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
  std::vector<double> Cx(size_t(nnzL), 0.0);
  std::vector<double> Dn(size_t(m), 0.0);
  {
    std::vector<double> w(size_t(m), 0.0);
    std::vector<int64_t> nxt(size_t(m), 0);        // next unused entry of column k
    std::vector<int32_t> head(size_t(m), -1), link(size_t(m), -1);  // columns waiting on row j
    for (int32_t j = 0; j < m; ++j) {
      for (int64_t p = Kp[size_t(j)]; p < Kp[size_t(j) + 1]; ++p) w[size_t(Ki[size_t(p)])] = Kx[size_t(p)];
      int32_t k = head[size_t(j)];
      while (k >= 0) {
        const int32_t knext = link[size_t(k)];
        const int64_t p0 = nxt[size_t(k)], pend = Cp[size_t(k) + 1];
        const double f = Cx[size_t(p0)] * Dn[size_t(k)];  // L(j,k) D(k)
        for (int64_t p = p0; p < pend; ++p) w[size_t(Ci[size_t(p)])] -= Cx[size_t(p)] * f;
        nxt[size_t(k)] = p0 + 1;
        if (p0 + 1 < pend) {
          const int32_t r = Ci[size_t(p0 + 1)];
          link[size_t(k)] = head[size_t(r)];
          head[size_t(r)] = k;
        }
        k = knext;
      }
      const double dj = w[size_t(j)];
      w[size_t(j)] = 0.0;
      if (!(dj > 0.0) || !std::isfinite(dj)) {
        err = "non-positive pivot in LDL^T of eps*I + A A^* at row " + std::to_string(j);
        return STROM_E_FACTOR;
      }
      Dn[size_t(j)] = dj;
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
        const int32_t i = Ci[size_t(p)];
        Cx[size_t(p)] = w[size_t(i)] / dj;
        w[size_t(i)] = 0.0;
      }
      if (Cp[size_t(j)] < Cp[size_t(j) + 1]) {
        nxt[size_t(j)] = Cp[size_t(j)];
        const int32_t r = Ci[size_t(Cp[size_t(j)])];
        link[size_t(j)] = head[size_t(r)];
        head[size_t(r)] = j;
      }
    }
  }
  H.nnzL = nnzL;
  Kp.clear(); Ki.clear(); Kx.clear();

  // ---------------------------------------------------------------- relabel by level
  // Forward dependency level of every row inside its task; rows of a task are relabeled
  // in (level, old position) order.  Dependencies point to lower levels, so the relabeled
  // L stays unit lower triangular and is the factor of the relabeled matrix.
  const int32_t ntask = int32_t(H.task_r0.size());
  std::vector<int32_t> lev(size_t(m), 0);  // longest dependency path inside the row's task
  std::vector<int32_t> newpos(static_cast<size_t>(m));
  {
    std::vector<int32_t> row_task(static_cast<size_t>(m));
    for (int32_t t = 0; t < ntask; ++t)
      for (int32_t r = H.task_r0[size_t(t)]; r < H.task_r1[size_t(t)]; ++r) row_task[size_t(r)] = t;
    for (int32_t j = 0; j < m; ++j)
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
        const int32_t i = Ci[size_t(p)];
        if (row_task[size_t(i)] == row_task[size_t(j)]) lev[size_t(i)] = std::max(lev[size_t(i)], lev[size_t(j)] + 1);
      }
    for (int32_t t = 0; t < ntask; ++t) {
      const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)];
      std::vector<int32_t> rows(size_t(r1 - r0));
      std::iota(rows.begin(), rows.end(), r0);
      std::stable_sort(rows.begin(), rows.end(), [&](int32_t a, int32_t b) { return lev[size_t(a)] < lev[size_t(b)]; });
      for (int32_t k = 0; k < r1 - r0; ++k) newpos[size_t(rows[size_t(k)])] = r0 + k;
    }
  }
  {
    std::vector<int32_t> perm2(static_cast<size_t>(m));
    std::vector<double> D2(static_cast<size_t>(m));
    std::vector<int32_t> lev2(static_cast<size_t>(m));
    for (int32_t i = 0; i < m; ++i) {
      perm2[size_t(newpos[size_t(i)])] = H.perm[size_t(i)];
      D2[size_t(newpos[size_t(i)])] = Dn[size_t(i)];
      lev2[size_t(newpos[size_t(i)])] = lev[size_t(i)];
    }
    H.perm.swap(perm2);
    H.D.swap(D2);
    lev.swap(lev2);
    for (int32_t k = 0; k < m; ++k) H.pinv[size_t(H.perm[size_t(k)])] = k;
  }
  // CSR of L (rows ascending columns) and of L^T, in the relabeled order
  H.Lrp.assign(size_t(m) + 1, 0);
  H.Urp.assign(size_t(m) + 1, 0);
  for (int32_t j = 0; j < m; ++j)
    for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
      H.Lrp[size_t(newpos[size_t(Ci[size_t(p)])]) + 1]++;
      H.Urp[size_t(newpos[size_t(j)]) + 1]++;
    }
  for (int32_t i = 0; i < m; ++i) { H.Lrp[size_t(i) + 1] += H.Lrp[size_t(i)]; H.Urp[size_t(i) + 1] += H.Urp[size_t(i)]; }
  H.Lci.resize(size_t(nnzL)); H.Lv.resize(size_t(nnzL));
  H.Uci.resize(size_t(nnzL)); H.Uv.resize(size_t(nnzL));
  {
    std::vector<int64_t> fl(H.Lrp.begin(), H.Lrp.end() - 1), fu(H.Urp.begin(), H.Urp.end() - 1);
    for (int32_t j = 0; j < m; ++j)
      for (int64_t p = Cp[size_t(j)]; p < Cp[size_t(j) + 1]; ++p) {
        const int32_t ni = newpos[size_t(Ci[size_t(p)])], nj = newpos[size_t(j)];
        const int64_t ql = fl[size_t(ni)]++, qu = fu[size_t(nj)]++;
        H.Lci[size_t(ql)] = nj; H.Lv[size_t(ql)] = Cx[size_t(p)];
        H.Uci[size_t(qu)] = ni; H.Uv[size_t(qu)] = Cx[size_t(p)];
      }
    auto sort_rows = [](std::vector<int64_t> &rp, std::vector<int32_t> &ci, std::vector<double> &v, int32_t mm) {
      std::vector<std::pair<int32_t, double>> tmp;
      for (int32_t i = 0; i < mm; ++i) {
        tmp.clear();
        for (int64_t p = rp[size_t(i)]; p < rp[size_t(i) + 1]; ++p) tmp.emplace_back(ci[size_t(p)], v[size_t(p)]);
        std::sort(tmp.begin(), tmp.end());
        int64_t q = rp[size_t(i)];
        for (auto &e : tmp) { ci[size_t(q)] = e.first; v[size_t(q)] = e.second; ++q; }
      }
    };
    sort_rows(H.Lrp, H.Lci, H.Lv, m);
    sort_rows(H.Urp, H.Uci, H.Uv, m);
  }
  for (int32_t i = 0; i < m; ++i)  // relabeling kept L lower triangular
    for (int64_t p = H.Lrp[size_t(i)]; p < H.Lrp[size_t(i) + 1]; ++p)
      if (H.Lci[size_t(p)] >= i) { err = "internal: relabeled factor not lower triangular"; return STROM_E_FACTOR; }
  Cp.clear(); Ci.clear(); Cx.clear();

  // ---------------------------------------------------------------- phases and schedule
  std::vector<int32_t> row_task(static_cast<size_t>(m));
  for (int32_t t = 0; t < ntask; ++t)
    for (int32_t r = H.task_r0[size_t(t)]; r < H.task_r1[size_t(t)]; ++r) row_task[size_t(r)] = t;
  std::vector<int32_t> fdepth(size_t(ntask), 0), bdepth(size_t(ntask), 0);
  for (int32_t t = 0; t < ntask; ++t) {
    const int32_t r0 = H.task_r0[size_t(t)], r1 = H.task_r1[size_t(t)], nt = r1 - r0;
    H.max_task_rows = std::max(H.max_task_rows, nt);
    for (int32_t i = r0; i < r1; ++i)
      for (int64_t p = H.Lrp[size_t(i)]; p < H.Lrp[size_t(i) + 1]; ++p) {
        const int32_t j = H.Lci[size_t(p)];
        if (j < r0) fdepth[size_t(t)] = std::max(fdepth[size_t(t)], fdepth[size_t(row_task[size_t(j)])] + 1);
      }
    // level boundaries (rows of one level are contiguous after the relabeling)
    std::vector<int32_t> lb;
    for (int32_t i = r0; i < r1; ++i)
      if (i == r0 || lev[size_t(i)] != lev[size_t(i) - 1]) lb.push_back(i);
    lb.push_back(r1);
    H.task_ph0.push_back(int32_t(H.ph_type.size()));
    const int32_t nl = int32_t(lb.size()) - 1;
    const int32_t wide = 16;  // levels with fewer rows are merged into dense phases
    int32_t l = 0;
    while (l < nl) {
      if (lb[size_t(l) + 1] - lb[size_t(l)] >= wide || nl == 1) {
        int32_t l1 = l;  // maximal run of wide levels
        while (l1 < nl && (lb[size_t(l1) + 1] - lb[size_t(l1)] >= wide || nl == 1)) ++l1;
        H.ph_type.push_back(kPhaseLevels);
        H.ph_a.push_back(lb[size_t(l)]);
        H.ph_b.push_back(lb[size_t(l1)]);
        H.ph_l0.push_back(int32_t(H.levptr.size()));
        H.ph_nl.push_back(l1 - l);
        for (int32_t q = l; q <= l1; ++q) H.levptr.push_back(lb[size_t(q)]);
        for (int32_t q = l; q < l1; ++q) {
          int64_t mf = 0, mb = 0;
          for (int32_t i = lb[size_t(q)]; i < lb[size_t(q) + 1]; ++i) {
            mf = std::max(mf, H.Lrp[size_t(i) + 1] - H.Lrp[size_t(i)]);
            mb = std::max(mb, H.Urp[size_t(i) + 1] - H.Urp[size_t(i)]);
          }
          H.lvl_gf.push_back(lanes_for(mf));
          H.lvl_gb.push_back(lanes_for(mb));
        }
        H.lvl_gf.push_back(1);  // entry of the closing boundary: lvl_g* stays aligned with levptr
        H.lvl_gb.push_back(1);
        H.ph_gf.push_back(0);
        H.ph_gb.push_back(0);
        H.ph_inv.push_back(-1);
        l = l1;
      } else {
        int32_t l1 = l;  // narrow levels up to kMaxDenseRows rows
        while (l1 < nl && (lb[size_t(l1) + 1] - lb[size_t(l1)] < wide) &&
               lb[size_t(l1) + 1] - lb[size_t(l)] <= kMaxDenseRows)
          ++l1;
        if (l1 == l) l1 = l + 1;
        const int32_t a = lb[size_t(l)], b = lb[size_t(l1)], nd = b - a;
        H.max_dense_rows = std::max(H.max_dense_rows, nd);
        int64_t mf = 0, mb = 0;
        std::vector<double> blk(size_t(nd) * nd, 0.0);
        for (int32_t i = a; i < b; ++i) {
          int64_t ext = 0;
          for (int64_t p = H.Lrp[size_t(i)]; p < H.Lrp[size_t(i) + 1]; ++p) {
            const int32_t j = H.Lci[size_t(p)];
            if (j >= a) blk[size_t(i - a) * nd + size_t(j - a)] = H.Lv[size_t(p)];
            else ++ext;
          }
          mf = std::max(mf, ext);
          int64_t extb = 0;
          for (int64_t p = H.Urp[size_t(i)]; p < H.Urp[size_t(i) + 1]; ++p) extb += H.Uci[size_t(p)] >= b;
          mb = std::max(mb, extb);
        }
        // inverse of the unit lower-triangular block, row-major: inv(i, j) for j <= i
        std::vector<double> inv(size_t(nd) * nd, 0.0);
        for (int32_t c = 0; c < nd; ++c) {
          inv[size_t(c) * nd + size_t(c)] = 1.0;
          for (int32_t i = c + 1; i < nd; ++i) {
            double s = 0.0;
            for (int32_t k = c; k < i; ++k) s -= blk[size_t(i) * nd + size_t(k)] * inv[size_t(k) * nd + size_t(c)];
            inv[size_t(i) * nd + size_t(c)] = s;
          }
        }
        H.ph_type.push_back(kPhaseDense);
        H.ph_a.push_back(a);
        H.ph_b.push_back(b);
        H.ph_l0.push_back(0);
        H.ph_nl.push_back(0);
        H.ph_gf.push_back(lanes_for(mf));
        H.ph_gb.push_back(lanes_for(mb));
        H.ph_inv.push_back(int64_t(H.invR.size()));
        for (int32_t i = 0; i < nd; ++i)  // packed lower triangle by rows
          for (int32_t j = 0; j <= i; ++j) H.invR.push_back(inv[size_t(i) * nd + size_t(j)]);
        for (int32_t j = 0; j < nd; ++j)  // packed lower triangle by columns
          for (int32_t i = j; i < nd; ++i) H.invC.push_back(inv[size_t(i) * nd + size_t(j)]);
        l = l1;
      }
    }
    H.task_ph1.push_back(int32_t(H.ph_type.size()));
  }
  // entry ranges of the gathers and the push segments
  H.Lin.resize(size_t(m));
  H.Lend.resize(size_t(m));
  H.Ubeg.resize(size_t(m));
  H.sptr.assign(size_t(m) + 1, 0);
  std::vector<std::vector<int32_t>> owned(static_cast<size_t>(ntask));
  std::vector<int64_t> seg_max(static_cast<size_t>(ntask), 0);
  for (int32_t t = 0; t < ntask; ++t)
    for (int32_t ph = H.task_ph0[size_t(t)]; ph < H.task_ph1[size_t(t)]; ++ph) {
      const int32_t a = H.ph_a[size_t(ph)], b = H.ph_b[size_t(ph)];
      const bool dense = H.ph_type[size_t(ph)] == kPhaseDense;
      for (int32_t i = a; i < b; ++i) {
        const int32_t r0 = H.task_r0[size_t(t)];
        int64_t p = H.Lrp[size_t(i)];
        const int64_t e = H.Lrp[size_t(i) + 1];
        int64_t q = p;
        while (q < e && H.Lci[size_t(q)] < r0) ++q;
        H.Lin[size_t(i)] = q;
        int64_t qe = q;
        if (dense) while (qe < e && H.Lci[size_t(qe)] < a) ++qe;
        else qe = e;
        H.Lend[size_t(i)] = qe;
        while (p < q) {  // split the columns of other tasks by owner
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
        int64_t u = H.Urp[size_t(i)];
        if (dense) while (u < H.Urp[size_t(i) + 1] && H.Uci[size_t(u)] < b) ++u;
        H.Ubeg[size_t(i)] = u;
      }
    }
  H.tsptr.assign(1, 0);
  for (int32_t t = 0; t < ntask; ++t) {
    H.tseg.insert(H.tseg.end(), owned[size_t(t)].begin(), owned[size_t(t)].end());
    H.tsptr.push_back(int32_t(H.tseg.size()));
    H.task_sg.push_back(std::min<int32_t>(16, lanes_for(seg_max[size_t(t)])));
  }
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
  return STROM_OK;
}

}  // namespace strom
