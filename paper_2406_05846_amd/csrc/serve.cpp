// serve.cpp -- continuous batching of SDP solves on one device.
//
// Setup workers take submitted problems in arrival order, build each instance (host analysis,
// in parallel across workers, + upload) as soon as its device footprint fits the context's HBM
// budget, and hand it to the solver thread.  The solver thread keeps every admitted instance in a merged
// batch (strom_batch_*: one launch per step over all of them) of instances with the same
// round length and sigma period; it advances each batch one round at a time, retires the
// instances that converged (or hit maxiter, or diverged), frees their memory, and rebuilds the
// batch with the instances admitted meanwhile.  A batch's instances have run whole rounds, so
// a fresh one (at iteration 0) can join it.
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
  bool done = false;
  strom_status err = STROM_OK;
  std::string errmsg;
  strom_info info{};
  std::vector<double> X, y, S;
};

// Instances iterated together: same kkt_every and sigma_every, iteration counts equal modulo
// kkt_every (phase).
struct Group {
  int kk = 10, se = 50, phase = 0;
  std::vector<Job *> act;
  strom_batch *bat = nullptr;
  bool dirty = true;  // membership changed since the batch was built
};

struct Server {
  strom_ctx *ctx = nullptr;
  int device = 0;
  std::vector<std::thread> setup_th;
  std::thread solve_th;
  int in_setup = 0;  // jobs taken by a setup worker and not yet handed on
  std::mutex mu;
  std::condition_variable cv_setup, cv_solve;
  std::deque<Job *> queued, ready;
  size_t n_active = 0;
  std::map<uint64_t, Job *> jobs;
  bool stop = false;
  uint64_t next = 1;
  std::vector<Group> groups;  // solver thread only
  uint64_t retired_since_wait = 0;
  std::FILE *log = nullptr;  // round timing, when STROM_SERVE_LOG names a file
};

namespace {

constexpr int kSetupWorkers = 8;  // host analyses in parallel (the uploads are serialized)

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
      S->queued.pop_front();
      S->in_setup++;
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
      // back to the front of the queue until a retirement frees memory; fail only if nothing
      // else holds or is about to hold any
      std::unique_lock<std::mutex> lk(S->mu);
      S->in_setup--;
      if (S->n_active == 0 && S->ready.empty() && S->in_setup == 0) {
        lk.unlock();
        finish(S, j, rc, strom_last_error());
        continue;
      }
      S->queued.push_front(j);
      const uint64_t seen = S->retired_since_wait;
      S->cv_setup.wait_for(lk, std::chrono::milliseconds(50),
                           [&] { return S->stop || S->retired_since_wait != seen; });
      continue;
    }
    if (rc != STROM_OK) {
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_setup--;
      }
      finish(S, j, rc, strom_last_error());
      continue;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->in_setup--;
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
  S->n_active--;
  j->t_done = now_s();
  j->info.t_queue_s = j->t_admit - j->t_arrive;
  j->info.t_solve_s = j->t_done - j->t_admit;
  j->info.t_setup_s = t_setup;
  j->err = rc;
  j->done = true;
  S->retired_since_wait++;
  S->cv_setup.notify_one();
}

void drop_batch(Group &g) {
  if (g.bat) strom_batch_destroy(g.bat);
  g.bat = nullptr;
  g.dirty = true;
}

// Every job of the group fails (device error): their instances are released.
void fail_group(Server *S, Group &g, const std::string &msg) {
  drop_batch(g);
  for (Job *j : g.act) {
    strom_sdp_destroy(j->sdp);
    j->sdp = nullptr;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->n_active--;
      S->retired_since_wait++;
    }
    finish(S, j, STROM_E_HIP, msg);
  }
  g.act.clear();
  S->cv_setup.notify_one();
}

void solve_loop(Server *S) {
  hipSetDevice(S->device);
  for (;;) {
    std::vector<Job *> admit;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_solve.wait(lk, [&] { return S->stop || !S->ready.empty() || S->n_active > 0; });
      if (S->stop) return;
      while (!S->ready.empty()) {
        Job *j = S->ready.front();
        S->ready.pop_front();
        j->t_admit = now_s();
        admit.push_back(j);
        S->n_active++;
      }
    }
    for (Job *j : admit) {  // join a group at phase 0 with the same round structure, else open one
      const strom_opts &o = sdp_opts(j->sdp);
      Group *g = nullptr;
      for (auto &c : S->groups)
        if (c.kk == o.kkt_every && c.se == o.sigma_every && (c.phase == 0 || c.act.empty())) { g = &c; break; }
      if (!g) {
        S->groups.emplace_back();
        g = &S->groups.back();
        g->kk = o.kkt_every;
        g->se = o.sigma_every;
      }
      if (g->act.empty()) g->phase = 0;
      g->act.push_back(j);
      g->dirty = true;
    }
    for (auto &g : S->groups) {
      if (g.act.empty()) continue;
      const double t_round = now_s();
      if (g.dirty) {
        drop_batch(g);
        std::vector<strom_sdp *> h;
        for (Job *j : g.act) h.push_back(j->sdp);
        if (strom_batch_create(S->ctx, int32_t(h.size()), h.data(), &g.bat) != STROM_OK) {
          fail_group(S, g, std::string("batch creation failed: ") + strom_last_error());
          continue;
        }
        g.dirty = false;
      }
      std::vector<strom_info> infos(g.act.size());
      if (strom_batch_step(g.bat, g.kk - g.phase, infos.data()) != STROM_OK) {
        fail_group(S, g, std::string("device error while solving: ") + strom_last_error());
        continue;
      }
      bool any_done = false;
      for (const auto &inf : infos) {
        any_done |= inf.state != STROM_RUNNING;
        if (inf.state == STROM_RUNNING) g.phase = int(inf.iters % g.kk);
      }
      if (any_done) {
        drop_batch(g);  // the retiring instances leave the batch before they are destroyed
        std::vector<Job *> keep;
        for (size_t k = 0; k < g.act.size(); ++k) {
          if (infos[k].state != STROM_RUNNING) retire(S, g.act[k]);
          else keep.push_back(g.act[k]);
        }
        g.act = keep;
      }
      if (S->log)
        std::fprintf(S->log, "round t=%.3f group kk %d active %zu retired %d total %.3f ms\n", t_round, g.kk,
                     infos.size(), any_done ? 1 : 0, 1e3 * (now_s() - t_round));
    }
  }
}

}  // namespace

Server *server_start(strom_ctx *ctx) {
  auto *S = new Server();
  S->ctx = ctx;
  hipGetDevice(&S->device);
  if (const char *lp = std::getenv("STROM_SERVE_LOG")) S->log = std::fopen(lp, "w");
  for (int k = 0; k < kSetupWorkers; ++k) S->setup_th.emplace_back(setup_loop, S);
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
  for (auto &t : S->setup_th) t.join();
  S->solve_th.join();
  for (auto &g : S->groups) drop_batch(g);
  for (auto &kv : S->jobs) {
    if (kv.second->sdp) strom_sdp_destroy(kv.second->sdp);
    delete kv.second;
  }
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
