// solve_schedule_sim.cpp -- test program: runs the host analysis of the library on an
// instance and executes the resulting solve schedule on the CPU, reading exactly what the
// device solve kernels read (task order by dependency group, phase streams with their
// slices and row flags, task-local staging, pushed partial sums, component inverses), then
// writes y = (eps I + A A^*)^{-1} r.  A test compares y with the oracle's factorization, so
// a wrong schedule (an entry missing or doubled, a bad index, a task run before one it
// depends on) shows up as a wrong solution or a failed check here, without a GPU.
//
// usage: solve_schedule_sim DIR   (DIR holds bs, rp, ci, av, r as raw arrays; writes DIR/y)
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <string>
#include <vector>

#include "../../paper_2406_05846_amd/csrc/strom_internal.h"

namespace {

template <class T>
std::vector<T> read_all(const std::string &f) {
  std::vector<T> v;
  FILE *fp = std::fopen(f.c_str(), "rb");
  if (!fp) return v;
  std::fseek(fp, 0, SEEK_END);
  const long n = std::ftell(fp);
  std::fseek(fp, 0, SEEK_SET);
  v.resize(size_t(n) / sizeof(T));
  const size_t got = std::fread(v.data(), sizeof(T), v.size(), fp);
  std::fclose(fp);
  v.resize(got);
  return v;
}

#define REQ(c)                                                   \
  do {                                                           \
    if (!(c)) {                                                  \
      std::printf("FAIL %s (line %d)\n", #c, __LINE__);          \
      std::exit(1);                                              \
    }                                                            \
  } while (0)

using strom::kLastFlag;
using strom::kPartFlag;
using strom::kSolveThreads;
using strom::kStartFlag;

}  // namespace

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  const std::string d = argv[1];
  const auto bs = read_all<int32_t>(d + "/bs");
  const auto rp = read_all<int64_t>(d + "/rp");
  const auto ci = read_all<int32_t>(d + "/ci");
  const auto av = read_all<double>(d + "/av");
  const auto r = read_all<double>(d + "/r");
  REQ(!rp.empty());
  const int m = int(rp.size()) - 1;
  REQ(int(r.size()) == m);
  strom::HostAnalysis H;
  std::string err;
  const auto rc = strom::analyze_instance(int32_t(bs.size()), bs.data(), m, rp.data(), ci.data(), av.data(), 1e-12, H, err);
  if (rc != STROM_OK) {
    std::printf("analysis failed %d %s\n", int(rc), err.c_str());
    return 1;
  }
  const long nph = long(H.ph_a.size());
  const int ntask = int(H.task_r0.size());
  for (int k = 0; k < strom::kStreamKinds; ++k) {
    const long nd = k < 4 ? nph : long(ntask);  // descriptors per phase, or per task for the push
    REQ(long(H.s_off[k].size()) == nd && long(H.s_K[k].size()) == nd);
    REQ(long(H.s_ra[k].size()) == nd * (kSolveThreads + 1));
    for (long p = 0; p < nd; ++p) REQ(H.s_off[k][p] + long(H.s_K[k][p]) * H.s_T[k][p] <= long(H.sval[k].size()));
  }
  // tasks cover the rows in order; every task is in exactly one group of each direction
  REQ(H.task_r0[0] == 0 && H.task_r1[ntask - 1] == m);
  for (int t = 1; t < ntask; ++t) REQ(H.task_r0[t] == H.task_r1[t - 1]);
  for (const auto *order : {&H.fwd_order, &H.bwd_order}) {
    std::vector<int> seen(size_t(ntask), 0);
    for (int t : *order) seen[size_t(t)]++;
    for (int x : seen) REQ(x == 1);
  }

  // One stream phase: every slice of the phase in turn, then the rows that span slices
  // (completed after the barrier from the open pieces of the slices before).
  auto walk = [&](int kind, long ph, int nrows, const std::function<double(int)> &get,
                  const std::function<void(int, double)> &fin) {
    const int *fr = H.s_ra[kind].data() + ph * (kSolveThreads + 1);
    const long off = H.s_off[kind][ph];
    const int K = H.s_K[kind][ph], Tp = H.s_T[kind][ph];
    REQ(K % strom::kStreamBatch == 0 && Tp % 64 == 0 && Tp <= kSolveThreads);
    std::vector<double> tv(kSolveThreads), hv(kSolveThreads);
    std::vector<int> tr(kSolveThreads), hr(kSolveThreads, -1);
    for (int t = 0; t < Tp; ++t) {
      const int f = fr[t];
      int row = f & (kStartFlag - 1);
      bool own = (f & kStartFlag) != 0;
      double acc = 0.0;
      for (int k = 0; k < K; ++k) {
        const double v = H.sval[kind][size_t(off + long(k) * Tp + t)];
        const int x = H.sidx[kind][size_t(off + long(k) * Tp + t)];
        REQ(x >= 0);
        acc += v * get(x & (kLastFlag - 1));
        if (x & kLastFlag) {
          REQ(row < nrows);
          if (own) fin(row, acc);
          else { REQ(hr[t] < 0); hr[t] = row; hv[t] = acc; }
          acc = 0.0;
          ++row;
          own = true;
        }
      }
      tv[t] = acc;
      tr[t] = own ? row : -1 - row;
    }
    for (int t = 0; t < Tp; ++t)
      if (hr[t] >= 0) {
        int u = t - 1;
        while (u >= 0 && tr[u] == -1 - hr[t]) --u;
        REQ(u >= 0 && tr[u] == hr[t]);
        double s = 0.0;
        for (int q = u; q < t; ++q) s += tv[q];
        fin(hr[t], s + hv[t]);
      }
  };

  std::vector<double> w(static_cast<size_t>(m)), y(static_cast<size_t>(m)), c(static_cast<size_t>(H.max_phase_nns) + 1);
  std::vector<double> part(std::max<size_t>(1, H.seg_pb.size()), NAN);
  for (int i = 0; i < m; ++i) w[size_t(H.pinv[i])] = r[size_t(i)];
  int staged = 0;
  for (int t = 0; t < ntask; ++t) staged += H.task_inl[size_t(t)] != 0;

  // forward: L z = P r, task by task in group order
  for (size_t g = 0; g + 1 < H.fwd_gptr.size(); ++g)
    for (int q = H.fwd_gptr[g]; q < H.fwd_gptr[g + 1]; ++q) {
      const int t = H.fwd_order[size_t(q)], r0 = H.task_r0[t], r1 = H.task_r1[t], nt = r1 - r0;
      const bool inl = H.task_inl[size_t(t)] != 0;
      const int p0 = H.task_pin[t], npin = H.task_pin[t + 1] - p0;
      std::vector<double> xs(size_t(nt + npin));
      for (int i = 0; i < nt; ++i) xs[size_t(i)] = w[size_t(r0 + i)];
      for (int k = 0; k < npin; ++k) {
        REQ(!std::isnan(part[size_t(p0 + k)]));  // pushed by a task of an earlier group
        xs[size_t(nt + k)] = part[size_t(p0 + k)];
      }
      auto X = [&](int row) -> double & { return inl ? xs[size_t(row - r0)] : w[size_t(row)]; };
      for (int p = H.task_ph0[t]; p < H.task_ph1[t]; ++p) {
        const int pa = H.ph_a[p], nns = H.ph_nns[p];
        std::vector<char> done(size_t(H.ph_b[p] - pa), 0);
        walk(0, p, H.ph_b[p] - pa,
             [&](int j) {
               if (inl) {  // own rows of earlier phases (or the padding row), then partial sums
                 REQ(j >= 0 && j < nt + npin && (j >= nt || j < pa - r0 || j == pa - r0));
                 return xs[size_t(j)];
               }
               if (j & kPartFlag) {
                 const double v = part[size_t(j & (kPartFlag - 1))];
                 REQ(!std::isnan(v));
                 return v;
               }
               REQ((j >= r0 && j < pa) || j == pa);
               return w[size_t(j)];
             },
             [&](int rr, double acc) {
               REQ(!done[size_t(rr)]);
               done[size_t(rr)] = 1;
               const double v = X(pa + rr) - acc;
               if (rr < nns) c[size_t(rr)] = v;
               else X(pa + rr) = v;
             });
        for (char x : done) REQ(x);
        std::vector<char> done2(size_t(nns), 0);
        if (nns)
          walk(1, p, nns, [&](int j) { REQ(j >= 0 && j < nns); return c[size_t(j)]; },
               [&](int rr, double acc) {
                 REQ(!done2[size_t(rr)]);
                 done2[size_t(rr)] = 1;
                 X(pa + rr) = acc;
               });
        for (char x : done2) REQ(x);
      }
      if (inl)
        for (int i = 0; i < nt; ++i) w[size_t(r0 + i)] = xs[size_t(i)];
      const int nseg = H.tsptr[t + 1] - H.tsptr[t];
      if (nseg > 0) {  // the push stream: one row per owned segment
        std::vector<char> pdone(size_t(nseg), 0);
        walk(4, t, nseg,
             [&](int j) {
               if (inl) { REQ(j >= 0 && j < nt); return w[size_t(r0 + j)]; }
               REQ(j >= r0 && j < r1);
               return w[size_t(j)];
             },
             [&](int rr, double acc) {
               REQ(!pdone[size_t(rr)]);
               pdone[size_t(rr)] = 1;
               part[size_t(H.tseg[size_t(H.tsptr[t] + rr)])] = acc;
             });
        for (char x : pdone) REQ(x);
      }
    }
  // backward: L^T x = D^{-1} z
  std::vector<char> bdone(size_t(ntask), 0);
  for (size_t g = 0; g + 1 < H.bwd_gptr.size(); ++g)
    for (int q = H.bwd_gptr[g]; q < H.bwd_gptr[g + 1]; ++q) {
      const int t = H.bwd_order[size_t(q)], r0 = H.task_r0[t], r1 = H.task_r1[t], nt = r1 - r0;
      const bool inl = H.task_inl[size_t(t)] != 0;
      const long x0 = H.task_xoff[size_t(t)];
      const int nx = int(H.task_xoff[size_t(t) + 1] - x0);
      std::vector<double> xs(size_t(nt + nx));
      for (int i = 0; i < nt; ++i) xs[size_t(i)] = w[size_t(r0 + i)];
      for (int k = 0; k < nx; ++k) {
        const int row = H.task_xrow[size_t(x0 + k)];
        REQ(row >= r1 && row < m);
        int ot = t + 1;
        while (H.task_r1[ot] <= row) ++ot;
        REQ(bdone[size_t(ot)]);  // solved by a task of an earlier backward group
        xs[size_t(nt + k)] = w[size_t(row)];
      }
      auto X = [&](int row) -> double & { return inl ? xs[size_t(row - r0)] : w[size_t(row)]; };
      for (int p = H.task_ph1[t] - 1; p >= H.task_ph0[t]; --p) {
        const int pa = H.ph_a[p], pb = H.ph_b[p], nns = H.ph_nns[p];
        std::vector<char> done(size_t(pb - pa), 0);
        walk(2, p, pb - pa,
             [&](int i) {
               if (inl) {
                 REQ(i >= 0 && i < nt + nx && (i >= pb - r0 || i == pa - r0));
                 return xs[size_t(i)];
               }
               REQ(i >= pb || i == pa);
               return w[size_t(i)];
             },
             [&](int rr, double acc) {
               REQ(!done[size_t(rr)]);
               done[size_t(rr)] = 1;
               const int j = pa + rr;
               const double v = X(j) / H.D[size_t(j)] - acc;
               if (rr < nns) c[size_t(rr)] = v;
               else X(j) = v;
             });
        for (char x : done) REQ(x);
        std::vector<char> done2(size_t(nns), 0);
        if (nns)
          walk(3, p, nns, [&](int j) { REQ(j >= 0 && j < nns); return c[size_t(j)]; },
               [&](int rr, double acc) {
                 REQ(!done2[size_t(rr)]);
                 done2[size_t(rr)] = 1;
                 X(pa + rr) = acc;
               });
        for (char x : done2) REQ(x);
      }
      if (inl)
        for (int i = 0; i < nt; ++i) w[size_t(r0 + i)] = xs[size_t(i)];
      for (int i = r0; i < r1; ++i) y[size_t(H.perm[size_t(i)])] = w[size_t(i)];
      bdone[size_t(t)] = 1;
    }
  // stream entries of the largest task of every launch group, both directions, and of all tasks
  long entries = 0, total_entries = 0;
  for (int dir = 0; dir < 2; ++dir) {
    const std::vector<int32_t> &gp = dir ? H.bwd_gptr : H.fwd_gptr, &ord = dir ? H.bwd_order : H.fwd_order;
    for (size_t g = 0; g + 1 < gp.size(); ++g) {
      long mx = 0;
      for (int32_t i = gp[g]; i < gp[g + 1]; ++i) {
        const int32_t t = ord[size_t(i)];
        long e = dir ? 0 : long(H.s_K[4][size_t(t)]) * H.s_T[4][size_t(t)];
        for (int32_t p = H.task_ph0[size_t(t)]; p < H.task_ph1[size_t(t)]; ++p)
          for (int k = dir ? 2 : 0; k <= (dir ? 3 : 1); ++k) e += long(H.s_K[k][size_t(p)]) * H.s_T[k][size_t(p)];
        mx = e > mx ? e : mx;
        total_entries += e;
      }
      entries += mx;
    }
  }
  std::printf("m %d tasks %d staged %d fwd_groups %zu bwd_groups %zu phases %ld nnzL %ld solve_entries %ld "
              "total_entries %ld\n",
              m, ntask, staged, H.fwd_gptr.size() - 1, H.bwd_gptr.size() - 1, nph, long(H.nnzL), entries,
              total_entries);
  FILE *fo = std::fopen((d + "/y").c_str(), "wb");
  REQ(fo);
  std::fwrite(y.data(), sizeof(double), size_t(m), fo);
  std::fclose(fo);
  return 0;
}
