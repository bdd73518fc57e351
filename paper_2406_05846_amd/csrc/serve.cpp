// serve.cpp -- continuous batching of SDP solves on one device.
//
// A setup thread takes submitted problems in arrival order, builds each instance (host
// analysis + upload) as soon as its device footprint fits the context's HBM budget, and
// hands it to the solver thread.  The solver thread keeps up to `max_slots` instances in
// flight, each on its own non-blocking stream, so that kernels of different instances overlap
// on the device; it advances every instance by a few iterations per round, reads back the
// residuals, retires instances that converged (or hit maxiter, or diverged), frees their
// memory and admits the next ready instance into the free slot.
#include "serve.h"

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace strom {

namespace {
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

struct Job {
  uint64_t id = 0;
  std::vector<int32_t> bs;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> av, b, C, X0, S0;
  int32_t m = 0;
  int64_t nsvec = 0;
  strom_opts o{};
  double t_arrive = 0, t_admit = 0, t_done = 0;
  strom_sdp *sdp = nullptr;
  int slot = -1;
  bool done = false;
  strom_status err = STROM_OK;
  std::string errmsg;
  strom_info info{};
  std::vector<double> X, y, S;
};

struct Server {
  strom_ctx *ctx = nullptr;
  int device = 0;
  std::thread setup_th, solve_th;
  std::mutex mu;
  std::condition_variable cv_setup, cv_solve;
  std::deque<Job *> queued, ready;
  std::vector<Job *> active;
  std::map<uint64_t, Job *> jobs;
  bool stop = false;
  uint64_t next = 1;
  std::vector<hipStream_t> streams;
  std::vector<char> slot_busy;
  int iters_per_round = 10;
  uint64_t retired_since_wait = 0;
  std::FILE *log = nullptr;  // round timing, when STROM_SERVE_LOG names a file
};

namespace {

void finish(Server *S, Job *j, strom_status err, const std::string &msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  j->err = err;
  j->errmsg = msg;
  j->done = true;
  j->t_done = now_s();
}

void setup_loop(Server *S) {
  hipSetDevice(S->device);
  for (;;) {
    Job *j = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_setup.wait(lk, [&] { return S->stop || !S->queued.empty(); });
      if (S->stop) return;
      j = S->queued.front();
    }
    strom_problem P{};
    P.nblocks = int32_t(j->bs.size());
    P.block_sizes = j->bs.data();
    P.m = j->m;
    P.nnz = int64_t(j->ci.size());
    P.A_rowptr = j->rp.data();
    P.A_col = j->ci.data();
    P.A_val = j->av.data();
    P.b = j->b.data();
    P.C_svec = j->C.data();
    P.X0_svec = j->X0.empty() ? nullptr : j->X0.data();
    P.S0_svec = j->S0.empty() ? nullptr : j->S0.data();
    strom_sdp *sdp = nullptr;
    strom_status rc = strom_sdp_setup(S->ctx, &P, &j->o, &sdp);
    if (rc == STROM_E_NOMEM) {
      // wait for a retirement to free memory; fail only if nothing else holds any
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->active.empty() && S->ready.empty()) {
        S->queued.pop_front();
        lk.unlock();
        finish(S, j, rc, strom_last_error());
        continue;
      }
      const uint64_t seen = S->retired_since_wait;
      S->cv_setup.wait_for(lk, std::chrono::milliseconds(50),
                           [&] { return S->stop || S->retired_since_wait != seen; });
      continue;
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->queued.pop_front();
    }
    if (rc != STROM_OK) {
      finish(S, j, rc, strom_last_error());
      continue;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    j->sdp = sdp;
    j->nsvec = int64_t(j->C.size());
    S->ready.push_back(j);
    S->cv_solve.notify_one();
  }
}

void retire(Server *S, Job *j) {
  strom_sdp *sdp = j->sdp;
  sdp_info(sdp, &j->info);
  j->X.resize(size_t(j->nsvec));
  j->S.resize(size_t(j->nsvec));
  j->y.resize(size_t(j->m));
  strom_status rc = strom_get_iterate(sdp, j->X.data(), j->y.data(), j->S.data());
  const double t_setup = j->info.t_setup_s;
  strom_sdp_destroy(sdp);
  std::lock_guard<std::mutex> lk(S->mu);
  j->sdp = nullptr;
  S->slot_busy[size_t(j->slot)] = 0;
  j->t_done = now_s();
  j->info.t_queue_s = j->t_admit - j->t_arrive;
  j->info.t_solve_s = j->t_done - j->t_admit;
  j->info.t_setup_s = t_setup;
  j->err = rc;
  j->done = true;
  S->retired_since_wait++;
  S->cv_setup.notify_one();
}

void solve_loop(Server *S) {
  hipSetDevice(S->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_solve.wait(lk, [&] { return S->stop || !S->ready.empty() || !S->active.empty(); });
      if (S->stop) return;
      while (!S->ready.empty()) {
        int slot = -1;
        for (size_t k = 0; k < S->slot_busy.size(); ++k)
          if (!S->slot_busy[k]) { slot = int(k); break; }
        if (slot < 0) break;
        Job *j = S->ready.front();
        S->ready.pop_front();
        S->slot_busy[size_t(slot)] = 1;
        j->slot = slot;
        j->t_admit = now_s();
        sdp_set_stream(j->sdp, S->streams[size_t(slot)]);
        S->active.push_back(j);
      }
    }
    // one round: enqueue on every slot's stream first, then read back, so instances overlap
    std::vector<Job *> act;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      act = S->active;
    }
    std::vector<char> bad(act.size(), 0);
    const double t_round = now_s();
    for (size_t k = 0; k < act.size(); ++k) {
      const strom_opts &o = sdp_opts(act[k]->sdp);
      int n = S->iters_per_round;
      (void)o;
      if (sdp_enqueue(act[k]->sdp, n, true) != hipSuccess) bad[k] = 1;
    }
    const double t_enq = now_s();
    std::vector<Job *> keep;
    for (size_t k = 0; k < act.size(); ++k) {
      Job *j = act[k];
      const double t_s0 = now_s();
      const bool rd_ok = !bad[k] && sdp_read_state(j->sdp) == hipSuccess;
      if (S->log) std::fprintf(S->log, "  job %llu wait %.3f ms\n", (unsigned long long)j->id, 1e3 * (now_s() - t_s0));
      if (!rd_ok) {
        strom_sdp_destroy(j->sdp);
        j->sdp = nullptr;
        {
          std::lock_guard<std::mutex> lk(S->mu);
          S->slot_busy[size_t(j->slot)] = 0;
          S->retired_since_wait++;
        }
        finish(S, j, STROM_E_HIP, "device error while solving");
        continue;
      }
      if (sdp_classify(j->sdp) != STROM_RUNNING) retire(S, j);
      else keep.push_back(j);
    }
    if (S->log)
      std::fprintf(S->log, "round t=%.3f active %zu enqueue %.3f ms total %.3f ms\n", t_round, act.size(),
                   1e3 * (t_enq - t_round), 1e3 * (now_s() - t_round));
    std::lock_guard<std::mutex> lk(S->mu);
    S->active = keep;
  }
}

}  // namespace

Server *server_start(strom_ctx *ctx) {
  auto *S = new Server();
  S->ctx = ctx;
  hipGetDevice(&S->device);
  if (const char *lp = std::getenv("STROM_SERVE_LOG")) S->log = std::fopen(lp, "w");
  const int slots = 8;
  S->streams.resize(slots);
  S->slot_busy.assign(slots, 0);
  for (int k = 0; k < slots; ++k) hipStreamCreateWithFlags(&S->streams[size_t(k)], hipStreamNonBlocking);
  S->setup_th = std::thread(setup_loop, S);
  S->solve_th = std::thread(solve_loop, S);
  return S;
}

void server_stop(Server *S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_setup.notify_all();
  S->cv_solve.notify_all();
  S->setup_th.join();
  S->solve_th.join();
  for (auto &kv : S->jobs) {
    if (kv.second->sdp) strom_sdp_destroy(kv.second->sdp);
    delete kv.second;
  }
  for (auto q : S->streams) hipStreamDestroy(q);
  if (S->log) std::fclose(S->log);
  delete S;
}

strom_status server_submit(Server *S, const strom_problem *P, const strom_opts *opts, uint64_t *ticket,
                           std::string &err) {
  if (P->m <= 0 || P->nblocks <= 0 || !P->A_rowptr || !P->A_col || !P->A_val || !P->b || !P->C_svec ||
      !P->block_sizes) {
    err = "malformed problem";
    return STROM_E_INVAL;
  }
  auto *j = new Job();
  j->t_arrive = now_s();
  j->bs.assign(P->block_sizes, P->block_sizes + P->nblocks);
  int64_t n = 0;
  for (int32_t v : j->bs) {
    if (v <= 0) { delete j; err = "block size <= 0"; return STROM_E_INVAL; }
    n += int64_t(v) * (v + 1) / 2;
  }
  j->m = P->m;
  j->rp.assign(P->A_rowptr, P->A_rowptr + P->m + 1);
  const int64_t nnz = j->rp.back();
  if (nnz != P->nnz || j->rp[0] != 0) { delete j; err = "nnz != rowptr[m]"; return STROM_E_INVAL; }
  j->ci.assign(P->A_col, P->A_col + nnz);
  j->av.assign(P->A_val, P->A_val + nnz);
  j->b.assign(P->b, P->b + P->m);
  j->C.assign(P->C_svec, P->C_svec + n);
  if (P->X0_svec) j->X0.assign(P->X0_svec, P->X0_svec + n);
  if (P->S0_svec) j->S0.assign(P->S0_svec, P->S0_svec + n);
  if (opts) j->o = *opts; else strom_default_opts(&j->o);
  std::lock_guard<std::mutex> lk(S->mu);
  j->id = S->next++;
  S->jobs[j->id] = j;
  S->queued.push_back(j);
  *ticket = j->id;
  S->cv_setup.notify_one();
  return STROM_OK;
}

strom_status server_poll(Server *S, uint64_t ticket, strom_info *out, double *X, double *y, double *Sv,
                         std::string &err) {
  Job *j = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) { err = "unknown ticket"; return STROM_E_NOTFOUND; }
    j = it->second;
    if (!j->done) return STROM_E_AGAIN;
    S->jobs.erase(it);
  }
  if (j->err != STROM_OK) {
    err = j->errmsg.empty() ? "solve failed" : j->errmsg;
    const strom_status e = j->err;
    delete j;
    return e;
  }
  if (out) *out = j->info;
  if (X) std::copy(j->X.begin(), j->X.end(), X);
  if (y) std::copy(j->y.begin(), j->y.end(), y);
  if (Sv) std::copy(j->S.begin(), j->S.end(), Sv);
  delete j;
  return STROM_OK;
}

}  // namespace strom
