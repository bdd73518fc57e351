// setup_cache_check.cpp -- test program: the host analysis of an instance set up from the
// pattern cache (the analysis of another instance with the same sparsity pattern, its numbers
// recomputed) must equal the analysis of the same instance from scratch, field by field and
// bit for bit, and the parallel factorization must equal the one-thread one.  Prints the setup
// times.
//
// usage: setup_cache_check DIR  (DIR holds bs, rp, ci as raw arrays and the values of two
//        instances, av_a and av_b); exit status 0 when every field agrees
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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

int g_fail = 0;

template <class T>
void same(const char *name, const std::vector<T> &a, const std::vector<T> &b) {
  if (a.size() != b.size() || (a.size() && std::memcmp(a.data(), b.data(), a.size() * sizeof(T)) != 0)) {
    std::printf("DIFF %s (%zu vs %zu entries)\n", name, a.size(), b.size());
    g_fail = 1;
  }
}

template <class T>
void same1(const char *name, const T &a, const T &b) {
  if (std::memcmp(&a, &b, sizeof(T)) != 0) {
    std::printf("DIFF %s\n", name);
    g_fail = 1;
  }
}

double analyze(const std::vector<int32_t> &bs, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
               const std::vector<double> &av, strom::HostAnalysis &H) {
  std::string err;
  const auto t0 = std::chrono::steady_clock::now();
  const auto rc = strom::analyze_instance(int32_t(bs.size()), bs.data(), int32_t(rp.size()) - 1, rp.data(),
                                          ci.data(), av.data(), 1e-12, H, err, 1, 64);
  if (rc != STROM_OK) {
    std::printf("analysis failed: %s\n", err.c_str());
    std::exit(1);
  }
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  const std::string d = argv[1];
  const auto bs = read_all<int32_t>(d + "/bs");
  const auto rp = read_all<int64_t>(d + "/rp");
  const auto ci = read_all<int32_t>(d + "/ci");
  const auto a = read_all<double>(d + "/av_a");
  const auto b = read_all<double>(d + "/av_b");
  if (rp.empty() || a.size() != ci.size() || b.size() != ci.size()) return 2;
  strom::HostAnalysis HA, HB, HF;
  setenv("STROM_SETUP_CACHE", "1", 1);
  const double t_first = analyze(bs, rp, ci, a, HA);   // first sight of the pattern: plain
  const double t_second = analyze(bs, rp, ci, a, HA);  // second: records the maps, fills the cache
  const double t_cached = analyze(bs, rp, ci, b, HB);  // same pattern: cache hit
  setenv("STROM_SETUP_CACHE", "0", 1);
  const double t_fresh = analyze(bs, rp, ci, b, HF);
  std::printf("setup first %.3f s, second (recording) %.3f s, cached %.3f s, from scratch %.3f s\n", t_first,
              t_second, t_cached, t_fresh);
#define CMP(f) same(#f, HB.f, HF.f)
#define CMP1(f) same1(#f, HB.f, HF.f)
  CMP1(m); CMP1(nsvec); CMP1(nblocks); CMP1(eps); CMP1(max_task_stage); CMP1(max_task_rows);
  CMP1(max_phase_nns); CMP1(nnzL);
  CMP(bsize); CMP(boff); CMP(Atrp); CMP(Atci); CMP(Atv); CMP(perm); CMP(pinv); CMP(Lrp); CMP(Lci); CMP(Lv);
  CMP(Urp); CMP(Uci); CMP(Uv); CMP(D); CMP(task_r0); CMP(task_r1); CMP(task_ph0); CMP(task_ph1); CMP(ph_a);
  CMP(ph_b); CMP(ph_nns); CMP(ph_gf); CMP(ph_gb); CMP(rcs); CMP(rce); CMP(rio); CMP(invR); CMP(invC); CMP(Lin);
  CMP(Lend); CMP(Ubeg); CMP(sptr); CMP(seg_pb); CMP(seg_pe); CMP(tsptr); CMP(tseg); CMP(task_sg); CMP(push_off);
  CMP(push_ci); CMP(push_v); CMP(task_pin); CMP(task_xoff); CMP(task_xrow); CMP(task_inl); CMP(fwd_order);
  CMP(fwd_gptr); CMP(bwd_order); CMP(bwd_gptr);
  for (int k = 0; k < strom::kStreamKinds; ++k) {
    same("sval", HB.sval[k], HF.sval[k]);
    same("sidx", HB.sidx[k], HF.sidx[k]);
    same("s_off", HB.s_off[k], HF.s_off[k]);
    same("s_K", HB.s_K[k], HF.s_K[k]);
    same("s_T", HB.s_T[k], HF.s_T[k]);
    same("s_ra", HB.s_ra[k], HF.s_ra[k]);
  }
  // the factorization's threads change nothing: the sequential loop gives the same bits
  {
    strom::HostAnalysis HS;
    setenv("STROM_SETUP_THREADS", "1", 1);
    analyze(bs, rp, ci, b, HS);
    unsetenv("STROM_SETUP_THREADS");
    same("Lv (one thread)", HS.Lv, HF.Lv);
    same("D (one thread)", HS.D, HF.D);
    same("invR (one thread)", HS.invR, HF.invR);
    for (int k = 0; k < strom::kStreamKinds; ++k) same("sval (one thread)", HS.sval[k], HF.sval[k]);
  }
  // and the numbers really changed with the instance
  if (HA.Lv == HB.Lv) { std::printf("the two instances have the same factor\n"); g_fail = 1; }
  std::printf(g_fail ? "MISMATCH\n" : "identical\n");
  return g_fail;
}
