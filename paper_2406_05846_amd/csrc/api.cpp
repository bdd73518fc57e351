// api.cpp -- the C ABI of include/strom.h: contexts, instance setup and upload, the device
// iteration driver, KKT readback and the dense batched projection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/strom.h"
#include "kernels.h"
#include "serve.h"
#include "strom_internal.h"

using strom::dev::DevState;

namespace {
thread_local std::string g_err;

strom_status fail(strom_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(STROM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Serializes graph captures with the library's synchronous copies, allocations and frees:
// while a stream is being captured, work that touches the legacy default stream fails.
std::recursive_mutex &device_lock() {
  static std::recursive_mutex mu;
  return mu;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Bump allocator over one device allocation.
struct Arena {
  size_t bytes = 0;
  template <typename T>
  size_t reserve(size_t count) {
    const size_t off = bytes;
    bytes += ((count * sizeof(T) + 255) / 256) * 256;
    return off;
  }
};
}  // namespace

struct strom_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t used = 0;
  int32_t *err_flag = nullptr;  // device flag of the dense projection
  bool own_stream = false;      // stream created by the context
  int64_t live = 0;             // instances set up directly (not through the server)
  size_t max_lds = 0;
  std::mutex mu;
  strom::Server *server = nullptr;
};

struct strom_sdp {
  strom_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;  // stream the instance is enqueued on (the ctx stream by default)
  strom_opts opts{};
  int32_t m = 0, nblocks = 0;
  int64_t nsvec = 0, nnz = 0, nnzL = 0;
  unsigned char *arena = nullptr;
  size_t arena_bytes = 0;
  // device arrays
  int64_t *A_rp = nullptr; int32_t *A_ci = nullptr; double *A_v = nullptr;
  int64_t *At_rp = nullptr; int32_t *At_ci = nullptr; double *At_v = nullptr;
  double *b = nullptr, *C = nullptr, *X = nullptr, *S = nullptr, *Xb = nullptr, *y = nullptr, *w = nullptr;
  int32_t *pinv = nullptr;
  int64_t *boff = nullptr; int32_t *bsz = nullptr; int32_t *blk_ids = nullptr;
  DevState *st = nullptr;
  double *part_rows = nullptr, *part_cols = nullptr, *part_cone = nullptr;
  double *Q = nullptr;         // eigenvectors of every block from the last ADMM projection
  int64_t *qoff = nullptr;     // offset of block k in Q
  bool q_valid = false;        // Q holds eigenvectors of the current iterate's blocks
  // reduced-precision projection: active until the polish switch (FP64 from then on)
  bool f32_active = false;
  // HIP graphs of one round of kkt_every iterations (KKT on the last), indexed by
  // [sigma rule on the last iteration][FP32 projection]; captured on first use
  hipGraphExec_t round_graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipStream_t capture_stream = nullptr;
  bool graphs = true;
  double f32_ref_eta = 0.0;    // eta at the last progress check of the FP32 phase
  int64_t f32_ref_iter = 0;
  strom::dev::SolveArgs sa{};
  strom::dev::SolveSchedule sch;
  std::vector<int> cls_n, cls_off, cls_cnt;  // projection launches, one per block size
  strom::dev::BigArgs big;                   // blocks beyond one workgroup's LDS (big.count may be 0)
  double normb = 0, normC = 0;
  int64_t iters = 0;
  strom_solve_state state = STROM_RUNNING;
  double t_setup = 0, t_solve = 0;
  DevState *st_host = nullptr;  // pinned mirror
  int32_t max_n = 0;
  std::vector<int32_t> bsize_h;  // block sizes (host copy)
  strom_batch *batch = nullptr;  // the batch the instance is iterated in, if any
};

extern "C" void strom_default_opts(strom_opts *o) {
  if (!o) return;
  o->sigma0 = 1.0;
  o->tau = 1.6;
  o->eps_reg = 1e-12;
  o->tol = 1e-6;
  o->maxiter = 100000;
  o->kkt_every = 10;
  o->proj_dtype = STROM_F64;
  o->polish_eta = 1e-5;
  o->sigma_every = 50;
  o->task_split = -1;
  o->block_rows = 0;
}

extern "C" const char *strom_last_error(void) { return g_err.c_str(); }

extern "C" strom_status strom_ctx_create(int device, void *hip_stream, size_t hbm_budget_bytes, strom_ctx **out) {
  if (!out) return fail(STROM_E_INVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(STROM_E_INVAL, "bad device index");
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  auto *c = new strom_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->budget = hbm_budget_bytes;
  c->max_lds = prop.sharedMemPerBlock;
  if (!c->stream) {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(STROM_E_HIP, "stream creation failed");
    }
    c->own_stream = true;
  }
  if (hipMalloc(&c->err_flag, 256) != hipSuccess) {
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    return fail(STROM_E_NOMEM, "hipMalloc of the context flag failed");
  }
  const strom_status sst = strom::scratch_init(device);  // the static work buffer's address on this device
  if (sst != STROM_OK) {
    hipFree(c->err_flag);
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    return sst;
  }
  *out = c;
  return STROM_OK;
}

extern "C" strom_status strom_ctx_destroy(strom_ctx *c) {
  if (!c) return fail(STROM_E_INVAL, "ctx is NULL");
  if (c->server) { strom::server_stop(c->server); c->server = nullptr; }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->live > 0) return fail(STROM_E_STATE, std::to_string(c->live) + " instance(s) still set up on this ctx");
  }
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  hipSetDevice(c->device);
  hipFree(c->err_flag);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete c;
  return STROM_OK;
}

// Blocks whose FP64 projection fits one workgroup's LDS take the one-workgroup kernel (in FP64 or
// FP32); larger ones the multi-workgroup block Jacobi of big.hip, always in FP64.
static bool fits_lds(const strom_ctx *ctx, int n) { return strom::dev::project_fits(n, false, ctx->max_lds); }

extern "C" strom_status strom_sdp_setup(strom_ctx *ctx, const strom_problem *P, const strom_opts *opts,
                                        strom_sdp **out) {
  if (!ctx || !P || !out) return fail(STROM_E_INVAL, "NULL argument");
  *out = nullptr;
  const double t0 = now_s();
  strom_opts o;
  if (opts) o = *opts; else strom_default_opts(&o);
  if (!(o.sigma0 > 0) || !(o.tau > 0 && o.tau < 2) || o.kkt_every <= 0 || o.maxiter <= 0 || o.sigma_every < 0 ||
      (o.sigma_every > 0 && o.sigma_every % o.kkt_every != 0) || o.task_split < -1 || o.task_split > 2 ||
      o.block_rows < 0 || o.block_rows > 256)
    return fail(STROM_E_INVAL, "invalid options");
  if (!P->A_rowptr || !P->A_col || !P->A_val || !P->b || !P->C_svec || !P->block_sizes)
    return fail(STROM_E_INVAL, "NULL problem array");
  if (P->nnz != (P->m > 0 ? P->A_rowptr[P->m] : 0)) return fail(STROM_E_INVAL, "nnz != rowptr[m]");
  strom::HostAnalysis H;
  std::string err;
  strom_status rc = strom::analyze_instance(P->nblocks, P->block_sizes, P->m, P->A_rowptr, P->A_col, P->A_val,
                                            o.eps_reg, H, err, o.task_split, o.block_rows);
  if (rc != STROM_OK) return fail(rc, err);
  int32_t max_n = 0, big_max = 0;
  for (int32_t n : H.bsize) {
    max_n = std::max(max_n, n);
    if (!fits_lds(ctx, n)) big_max = std::max(big_max, n);
  }
  if (big_max > strom::dev::kBigMaxN)
    return fail(STROM_E_INVAL, "block of size " + std::to_string(big_max) + " is over the largest supported size " +
                                   std::to_string(strom::dev::kBigMaxN));

  auto *s = new strom_sdp();
  s->ctx = ctx;
  s->stream = ctx->stream;
  s->opts = o;
  s->f32_active = o.proj_dtype == STROM_F32;
  s->m = P->m;
  s->nblocks = P->nblocks;
  s->nsvec = H.nsvec;
  s->nnz = P->nnz;
  s->nnzL = H.nnzL;
  s->max_n = max_n;
  s->bsize_h.assign(P->block_sizes, P->block_sizes + P->nblocks);
  const int32_t m = P->m;
  const int64_t n = H.nsvec, nnz = P->nnz;
  const int ntask = int(H.task_r0.size());
  const int nrb = (m + 255) / 256, ncb = int((n + 255) / 256);

  // projection launches: one launch over every block (largest first) when they fit the chip
  // in one wave of workgroups, else one launch per block size
  std::map<int, std::vector<int32_t>> by_n;
  std::vector<int32_t> big_ids;
  for (int32_t k = 0; k < P->nblocks; ++k) {
    if (fits_lds(ctx, H.bsize[size_t(k)])) by_n[H.bsize[size_t(k)]].push_back(k);
    else big_ids.push_back(k);
  }
  const int32_t nsmall = P->nblocks - int32_t(big_ids.size());
  std::vector<int32_t> ids;
  for (auto it = by_n.rbegin(); it != by_n.rend(); ++it) {
    if (nsmall > 256 || s->cls_n.empty()) {
      s->cls_n.push_back(it->first);
      s->cls_off.push_back(int(ids.size()));
      s->cls_cnt.push_back(0);
    }
    s->cls_cnt.back() += int(it->second.size());
    ids.insert(ids.end(), it->second.begin(), it->second.end());
  }

  Arena ar;
  const size_t oArp = ar.reserve<int64_t>(size_t(m) + 1), oAci = ar.reserve<int32_t>(size_t(nnz)),
               oAv = ar.reserve<double>(size_t(nnz));
  const size_t oTrp = ar.reserve<int64_t>(size_t(n) + 1), oTci = ar.reserve<int32_t>(size_t(nnz)),
               oTv = ar.reserve<double>(size_t(nnz));
  const size_t ob = ar.reserve<double>(size_t(m)), oC = ar.reserve<double>(size_t(n)),
               oX = ar.reserve<double>(size_t(n)), oS = ar.reserve<double>(size_t(n)),
               oXb = ar.reserve<double>(size_t(n)), oy = ar.reserve<double>(size_t(m)),
               ow = ar.reserve<double>(size_t(m));
  const size_t operm = ar.reserve<int32_t>(size_t(m)), opinv = ar.reserve<int32_t>(size_t(m));
  const size_t oD = ar.reserve<double>(size_t(m));
  const size_t nph = H.ph_a.size();
  const size_t oTk = ar.reserve<int32_t>(size_t(ntask) * 4), oPh = ar.reserve<int32_t>(std::max<size_t>(1, nph) * 2);
  const size_t oFo = ar.reserve<int32_t>(H.fwd_order.size()), oBo = ar.reserve<int32_t>(H.bwd_order.size());
  const size_t nseg = std::max<size_t>(1, H.seg_pb.size());
  const size_t oTsp = ar.reserve<int32_t>(size_t(ntask) + 1), oTseg = ar.reserve<int32_t>(nseg),
               oPart = ar.reserve<double>(nseg);
  const size_t oTpin = ar.reserve<int32_t>(size_t(ntask) + 1), oTinl = ar.reserve<int32_t>(size_t(ntask)),
               oTxoff = ar.reserve<int64_t>(size_t(ntask) + 1),
               oTxrow = ar.reserve<int32_t>(std::max<size_t>(1, H.task_xrow.size()));
  size_t oSv[strom::kStreamKinds], oSi[strom::kStreamKinds], oSoff[strom::kStreamKinds], oSK[strom::kStreamKinds],
      oST[strom::kStreamKinds], oSra[strom::kStreamKinds];
  for (int k = 0; k < strom::kStreamKinds; ++k) {
    oSv[k] = ar.reserve<double>(std::max<size_t>(1, H.sval[k].size()));
    oSi[k] = ar.reserve<int32_t>(std::max<size_t>(1, H.sidx[k].size()));
    oSoff[k] = ar.reserve<int64_t>(std::max<size_t>(1, H.s_off[k].size()));
    oSK[k] = ar.reserve<int32_t>(std::max<size_t>(1, H.s_K[k].size()));
    oST[k] = ar.reserve<int32_t>(std::max<size_t>(1, H.s_T[k].size()));
    oSra[k] = ar.reserve<int32_t>(std::max<size_t>(1, H.s_ra[k].size()));
  }
  const size_t oBoff = ar.reserve<int64_t>(size_t(P->nblocks)), oBsz = ar.reserve<int32_t>(size_t(P->nblocks)),
               oIds = ar.reserve<int32_t>(ids.size());
  const size_t oSt = ar.reserve<DevState>(1);
  const size_t oPr = ar.reserve<double>(2 * size_t(nrb)), oPc = ar.reserve<double>(2 * size_t(ncb)),
               oPk = ar.reserve<double>(2 * size_t(ncb));
  std::vector<int64_t> qoff(size_t(P->nblocks));
  int64_t qtot = 0;
  for (int32_t k = 0; k < P->nblocks; ++k) {
    qoff[size_t(k)] = qtot;
    const int64_t nb = H.bsize[size_t(k)];
    qtot += nb * (nb + (nb & 1));  // eigenvectors n x (n rounded up to even) of the projection
  }
  const size_t oQ = ar.reserve<double>(size_t(qtot)), oQoff = ar.reserve<int64_t>(size_t(P->nblocks));
  s->big.np = big_max > 0 ? strom::dev::big_padded(big_max) : 0;
  s->big.count = int32_t(big_ids.size());
  const size_t oBig = ar.reserve<int32_t>(std::max<size_t>(1, big_ids.size())),
               oBigW = ar.reserve<double>(big_ids.empty() ? 1 : strom::dev::big_work_doubles(s->big.np, s->big.count));
  s->arena_bytes = ar.bytes;

  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->budget && ctx->used + ar.bytes > ctx->budget) {
      delete s;
      return fail(STROM_E_NOMEM, "instance needs " + std::to_string(ar.bytes) + " bytes, over the HBM budget");
    }
    ctx->used += ar.bytes;
    ctx->live++;
  }
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  auto undo = [&](strom_status st, const std::string &msg) {
    { std::lock_guard<std::mutex> lk(ctx->mu); ctx->used -= s->arena_bytes; ctx->live--; }
    if (s->arena) hipFree(s->arena);
    if (s->st_host) hipHostFree(s->st_host);
    delete s;
    return fail(st, msg);
  };
  if (hipSetDevice(ctx->device) != hipSuccess) return undo(STROM_E_HIP, "hipSetDevice failed");
  if (hipMalloc(&s->arena, ar.bytes) != hipSuccess) return undo(STROM_E_NOMEM, "hipMalloc of the instance failed");
  if (hipHostMalloc(&s->st_host, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
    return undo(STROM_E_NOMEM, "hipHostMalloc failed");
  unsigned char *base = s->arena;
  auto P64 = [&](size_t o) { return reinterpret_cast<int64_t *>(base + o); };
  auto P32 = [&](size_t o) { return reinterpret_cast<int32_t *>(base + o); };
  auto PD = [&](size_t o) { return reinterpret_cast<double *>(base + o); };
  s->A_rp = P64(oArp); s->A_ci = P32(oAci); s->A_v = PD(oAv);
  s->At_rp = P64(oTrp); s->At_ci = P32(oTci); s->At_v = PD(oTv);
  s->b = PD(ob); s->C = PD(oC); s->X = PD(oX); s->S = PD(oS); s->Xb = PD(oXb); s->y = PD(oy); s->w = PD(ow);
  s->pinv = P32(opinv);
  s->boff = P64(oBoff); s->bsz = P32(oBsz); s->blk_ids = P32(oIds);
  s->st = reinterpret_cast<DevState *>(base + oSt);
  s->part_rows = PD(oPr); s->part_cols = PD(oPc); s->part_cone = PD(oPk);
  s->Q = PD(oQ); s->qoff = P64(oQoff);
  s->big.ids = P32(oBig); s->big.boff = s->boff; s->big.bsz = s->bsz; s->big.work = PD(oBigW);
  int32_t *tk = P32(oTk), *ph = P32(oPh);
  auto &sa = s->sa;
  sa.task_r0 = tk; sa.task_r1 = tk + ntask; sa.task_ph0 = tk + 2 * ntask; sa.task_ph1 = tk + 3 * ntask;
  sa.ph_a = ph; sa.ph_nns = ph + nph;
  sa.D = PD(oD); sa.perm = P32(operm);
  sa.tsptr = P32(oTsp); sa.tseg = P32(oTseg); sa.part = PD(oPart);
  sa.task_pin = P32(oTpin); sa.task_inl = P32(oTinl); sa.task_xoff = P64(oTxoff); sa.task_xrow = P32(oTxrow);
  for (int k = 0; k < strom::kStreamKinds; ++k) {
    sa.sval[k] = PD(oSv[k]); sa.sidx[k] = P32(oSi[k]); sa.s_off[k] = P64(oSoff[k]);
    sa.s_K[k] = P32(oSK[k]); sa.s_T[k] = P32(oST[k]); sa.s_ra[k] = P32(oSra[k]);
  }
  sa.c_cap = std::max(1, H.max_phase_nns);
  sa.lds_rows = std::max(1, H.max_task_stage);
  if (size_t(strom::kSolveThreads * 3 / 2 + sa.lds_rows + sa.c_cap) * sizeof(double) > ctx->max_lds)
    return undo(STROM_E_INVAL, "the solve schedule needs more LDS than the device has");
  s->sch.fwd_gptr = H.fwd_gptr;
  s->sch.bwd_gptr = H.bwd_gptr;
  s->sch.fwd_order = H.fwd_order;
  s->sch.bwd_order = H.bwd_order;
  // a task's duration is about the stream entries each of its threads walks, plus a few
  // per phase for the barriers (merged launches start their longest tasks first)
  s->sch.fwd_cost.assign(size_t(ntask), 0);
  s->sch.bwd_cost.assign(size_t(ntask), 0);
  for (int t = 0; t < ntask; ++t) {
    int32_t f = H.s_K[4][size_t(t)], b = 0;
    for (int32_t q = H.task_ph0[size_t(t)]; q < H.task_ph1[size_t(t)]; ++q) {
      f += H.s_K[0][size_t(q)] + H.s_K[1][size_t(q)] + 4;
      b += H.s_K[2][size_t(q)] + H.s_K[3][size_t(q)] + 4;
    }
    s->sch.fwd_cost[size_t(t)] = f;
    s->sch.bwd_cost[size_t(t)] = b;
  }
  s->sch.fwd_order_dev = P32(oFo);
  s->sch.bwd_order_dev = P32(oBo);

  // host staging of the small arrays, then synchronous uploads
  std::vector<int32_t> tkh(size_t(ntask) * 4), phh(std::max<size_t>(1, nph) * 2);
  for (int t = 0; t < ntask; ++t) {
    tkh[size_t(t)] = H.task_r0[size_t(t)];
    tkh[size_t(ntask + t)] = H.task_r1[size_t(t)];
    tkh[size_t(2 * ntask + t)] = H.task_ph0[size_t(t)];
    tkh[size_t(3 * ntask + t)] = H.task_ph1[size_t(t)];
  }
  for (size_t k = 0; k < nph; ++k) {
    phh[k] = H.ph_a[k];
    phh[nph + k] = H.ph_nns[k];
  }
  std::vector<double> zeros;
  hipError_t up_err = hipSuccess;
  auto up = [&](const void *dst, const void *src, size_t bytes) -> bool {
    if (bytes == 0) return true;
    const hipError_t e = hipMemcpy(const_cast<void *>(dst), src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess && up_err == hipSuccess) up_err = e;
    return e == hipSuccess;
  };
  bool ok = true;
  ok &= up(s->A_rp, P->A_rowptr, sizeof(int64_t) * (size_t(m) + 1));
  ok &= up(s->A_ci, P->A_col, sizeof(int32_t) * size_t(nnz));
  ok &= up(s->A_v, P->A_val, sizeof(double) * size_t(nnz));
  ok &= up(s->At_rp, H.Atrp.data(), sizeof(int64_t) * H.Atrp.size());
  ok &= up(s->At_ci, H.Atci.data(), sizeof(int32_t) * H.Atci.size());
  ok &= up(s->At_v, H.Atv.data(), sizeof(double) * H.Atv.size());
  ok &= up(s->b, P->b, sizeof(double) * size_t(m));
  ok &= up(s->C, P->C_svec, sizeof(double) * size_t(n));
  ok &= hipMemset(s->X, 0, sizeof(double) * size_t(n)) == hipSuccess;
  ok &= hipMemset(s->S, 0, sizeof(double) * size_t(n)) == hipSuccess;
  ok &= hipMemset(s->y, 0, sizeof(double) * size_t(m)) == hipSuccess;
  if (P->X0_svec) ok &= up(s->X, P->X0_svec, sizeof(double) * size_t(n));
  if (P->S0_svec) ok &= up(s->S, P->S0_svec, sizeof(double) * size_t(n));
  ok &= up(sa.perm, H.perm.data(), sizeof(int32_t) * size_t(m));
  ok &= up(s->pinv, H.pinv.data(), sizeof(int32_t) * size_t(m));
  ok &= up(const_cast<double *>(sa.D), H.D.data(), sizeof(double) * H.D.size());
  ok &= up(tk, tkh.data(), sizeof(int32_t) * tkh.size());
  ok &= up(ph, phh.data(), sizeof(int32_t) * phh.size());
  ok &= up(const_cast<int32_t *>(sa.tsptr), H.tsptr.data(), sizeof(int32_t) * H.tsptr.size());
  ok &= up(const_cast<int32_t *>(sa.tseg), H.tseg.data(), sizeof(int32_t) * H.tseg.size());
  {
    const std::vector<int32_t> inl(H.task_inl.begin(), H.task_inl.end());
    ok &= up(const_cast<int32_t *>(sa.task_inl), inl.data(), sizeof(int32_t) * inl.size());
  }
  ok &= up(const_cast<int32_t *>(sa.task_pin), H.task_pin.data(), sizeof(int32_t) * H.task_pin.size());
  ok &= up(const_cast<int64_t *>(sa.task_xoff), H.task_xoff.data(), sizeof(int64_t) * H.task_xoff.size());
  ok &= up(const_cast<int32_t *>(sa.task_xrow), H.task_xrow.data(), sizeof(int32_t) * H.task_xrow.size());
  for (int k = 0; k < strom::kStreamKinds; ++k) {
    ok &= up(const_cast<double *>(sa.sval[k]), H.sval[k].data(), sizeof(double) * H.sval[k].size());
    ok &= up(const_cast<int32_t *>(sa.sidx[k]), H.sidx[k].data(), sizeof(int32_t) * H.sidx[k].size());
    ok &= up(const_cast<int64_t *>(sa.s_off[k]), H.s_off[k].data(), sizeof(int64_t) * H.s_off[k].size());
    ok &= up(const_cast<int32_t *>(sa.s_K[k]), H.s_K[k].data(), sizeof(int32_t) * H.s_K[k].size());
    ok &= up(const_cast<int32_t *>(sa.s_T[k]), H.s_T[k].data(), sizeof(int32_t) * H.s_T[k].size());
    ok &= up(const_cast<int32_t *>(sa.s_ra[k]), H.s_ra[k].data(), sizeof(int32_t) * H.s_ra[k].size());
  }
  ok &= up(const_cast<int32_t *>(s->sch.fwd_order_dev), H.fwd_order.data(), sizeof(int32_t) * H.fwd_order.size());
  ok &= up(const_cast<int32_t *>(s->sch.bwd_order_dev), H.bwd_order.data(), sizeof(int32_t) * H.bwd_order.size());
  ok &= up(s->boff, H.boff.data(), sizeof(int64_t) * size_t(P->nblocks));
  ok &= up(s->qoff, qoff.data(), sizeof(int64_t) * qoff.size());
  if (!big_ids.empty()) ok &= up(s->big.ids, big_ids.data(), sizeof(int32_t) * big_ids.size());
  ok &= up(s->bsz, H.bsize.data(), sizeof(int32_t) * size_t(P->nblocks));
  ok &= up(s->blk_ids, ids.data(), sizeof(int32_t) * ids.size());
  DevState st0{};
  st0.sigma = o.sigma0;
  st0.tau = o.tau;
  st0.sigma_used = o.sigma0;
  ok &= up(s->st, &st0, sizeof(DevState));
  if (!ok) return undo(STROM_E_HIP, std::string("upload of the instance failed: ") + hipGetErrorString(up_err));
  double nb2 = 0, nc2 = 0;
  for (int32_t i = 0; i < m; ++i) nb2 += P->b[i] * P->b[i];
  for (int64_t c = 0; c < n; ++c) nc2 += P->C_svec[c] * P->C_svec[c];
  s->normb = std::sqrt(nb2);
  s->normC = std::sqrt(nc2);
  s->t_setup = now_s() - t0;
  *out = s;
  return STROM_OK;
}

extern "C" strom_status strom_sdp_destroy(strom_sdp *s) {
  if (!s) return fail(STROM_E_INVAL, "sdp is NULL");
  if (s->batch) return fail(STROM_E_STATE, "the instance belongs to a batch: destroy the batch first");
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  hipSetDevice(s->ctx->device);
  hipStreamSynchronize(s->stream);
  for (auto &row : s->round_graph)
    for (auto &g : row)
      if (g) hipGraphExecDestroy(g);
  if (s->capture_stream) hipStreamDestroy(s->capture_stream);
  hipFree(s->arena);
  hipHostFree(s->st_host);
  {
    std::lock_guard<std::mutex> lk(s->ctx->mu);
    s->ctx->used -= s->arena_bytes;
    s->ctx->live--;
  }
  delete s;
  return STROM_OK;
}

namespace {

// S_out = (Pi(X_in) - X_in) * scale for every block (scale <= 0: 1 / sigma).  Every call
// warm-starts from, and refreshes, the eigenvectors kept per block (the cone distance of X
// uses them too: X and X_b differ little, and any orthogonal start gives the same result).
hipError_t enqueue_projection(strom_sdp *s, const double *X_in, double *S_out, double scale, bool reorth) {
  const bool f32 = s->f32_active;
  for (size_t c = 0; c < s->cls_n.size(); ++c) {
    hipError_t e = strom::dev::launch_project_admm(s->stream, f32, s->cls_n[c], s->cls_cnt[c],
                                                   s->blk_ids + s->cls_off[c], s->boff, s->bsz, X_in, S_out, s->st,
                                                   scale, s->Q, s->qoff, s->q_valid, reorth);
    if (e != hipSuccess) return e;
  }
  if (s->big.count > 0) {
    hipError_t e = strom::dev::launch_project_big_admm(s->stream, s->big, X_in, S_out, s->st, scale, s->Q, s->qoff,
                                                       s->q_valid, reorth);
    if (e != hipSuccess) return e;
  }
  s->q_valid = true;
  return hipSuccess;
}

// Residuals of the current iterate (part_cols must hold the dual-residual partials); with
// do_sigma, the cone distance of X (through the scratch X_b buffer) and the sigma rule.
hipError_t enqueue_kkt(strom_sdp *s, bool do_sigma) {
  if (do_sigma) {
    hipError_t e = enqueue_projection(s, s->X, s->Xb, 1.0, true);
    if (e != hipSuccess) return e;
  }
  return strom::dev::launch_kkt(s->stream, s->m, s->nsvec, s->A_rp, s->A_ci, s->A_v, s->X, s->b, s->y, s->part_rows,
                                s->part_cols, s->Xb, s->part_cone, s->normb, s->normC, do_sigma ? 1 : 0, s->st);
}

// Enqueue one iteration (steps 1-4); with kkt, also the residuals of the new iterate.  first:
// the iteration opens a round (its projection re-orthogonalizes the kept eigenvectors).
hipError_t enqueue_iteration(strom_sdp *s, bool kkt, bool do_sigma, bool first) {
  hipStream_t q = s->stream;
  hipError_t e;
  // step 1
  if ((e = strom::dev::launch_rhs(q, s->m, s->A_rp, s->A_ci, s->A_v, s->X, s->S, s->C, s->b, s->pinv, s->st, s->w)))
    return e;
  if ((e = strom::dev::launch_solve(q, s->sch, s->sa, s->w, s->y))) return e;
  // step 2
  if ((e = strom::dev::launch_xb(q, s->nsvec, s->At_rp, s->At_ci, s->At_v, s->y, s->X, s->C, s->st, s->Xb))) return e;
  if ((e = enqueue_projection(s, s->Xb, s->S, 0.0, first))) return e;
  // step 3
  if ((e = strom::dev::launch_rhs(q, s->m, s->A_rp, s->A_ci, s->A_v, s->X, s->S, s->C, s->b, s->pinv, s->st, s->w)))
    return e;
  if ((e = strom::dev::launch_solve(q, s->sch, s->sa, s->w, s->y))) return e;
  // step 4
  if ((e = strom::dev::launch_xupdate(q, s->nsvec, s->At_rp, s->At_ci, s->At_v, s->y, s->S, s->C, s->st, s->X,
                                      kkt ? s->part_cols : nullptr, 1)))
    return e;
  if (kkt)
    if ((e = enqueue_kkt(s, do_sigma))) return e;
  return hipSuccess;
}

void fill_info(const strom_sdp *s, strom_info *info) {
  const DevState &d = *s->st_host;
  info->eta_p = d.eta_p;
  info->eta_d = d.eta_d;
  info->eta_g = d.eta_g;
  info->pobj = d.pobj;
  info->dobj = d.dobj;
  info->sigma = d.sigma;
  info->iters = s->iters;
  info->state = s->state;
  info->t_queue_s = 0;
  info->t_setup_s = s->t_setup;
  info->t_solve_s = s->t_solve;
}

strom_solve_state classify(const strom_sdp *s) {
  const DevState &d = *s->st_host;
  const double eta = std::max(d.eta_p, std::max(d.eta_d, d.eta_g));
  if (!std::isfinite(eta)) return STROM_DIVERGED;
  if (eta <= s->opts.tol) return STROM_CONVERGED;
  if (s->iters >= s->opts.maxiter) return STROM_MAXITER;
  return STROM_RUNNING;
}

}  // namespace

namespace strom {
// Used by the serving loop: enqueue n iterations without synchronizing; returns true when
// residuals were computed on the last one.
// Captures one round of kkt_every iterations (residuals on the last, the sigma rule too when
// sigma_last) as a graph; the kernels read sigma, tau and every array from device memory, so
// the graph replays any round of the instance.
static hipError_t capture_round(strom_sdp *s, bool sigma_last, hipGraphExec_t *out) {
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  hipError_t e = hipSuccess;
  if (!s->capture_stream && (e = hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking))) return e;
  hipStream_t saved = s->stream;
  s->stream = s->capture_stream;
  e = hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal);
  hipError_t e2 = hipSuccess;
  const int kk = s->opts.kkt_every;
  for (int k = 0; k < kk && e == hipSuccess && e2 == hipSuccess; ++k)
    e2 = enqueue_iteration(s, k == kk - 1, sigma_last && k == kk - 1, k == 0);
  hipGraph_t g = nullptr;
  if (e == hipSuccess) e = hipStreamEndCapture(s->capture_stream, &g);
  s->stream = saved;
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) hipGraphDestroy(g);
  return e;
}

// Enqueues n iterations.  An iteration computes the residuals when it closes a round of
// kkt_every iterations, when it applies the sigma rule, or when it is the last one asked
// for with kkt_last.  Full rounds that start on a round boundary, after the first
// (cold-start) projection, replay a captured graph.
hipError_t sdp_enqueue(strom_sdp *s, int n_iter, bool kkt_last) {
  const int kk = s->opts.kkt_every;
  const int se = s->opts.sigma_every;
  int k = 0;
  while (k < n_iter) {
    const int64_t it = s->iters;
    if (s->graphs && s->q_valid && it % kk == 0 && n_iter - k >= kk) {
      const int sl = (se > 0 && (it + kk) % se == 0) ? 1 : 0, fl = s->f32_active ? 1 : 0;
      hipError_t e = hipSuccess;
      if (!s->round_graph[sl][fl] && (e = capture_round(s, sl != 0, &s->round_graph[sl][fl]))) {
        s->graphs = false;  // capture not available: launch directly from now on
        (void)hipGetLastError();
        continue;
      }
      if ((e = hipGraphLaunch(s->round_graph[sl][fl], s->stream))) return e;
      s->iters += kk;
      k += kk;
      continue;
    }
    const bool sig = se > 0 && (it + 1) % se == 0;
    const bool kkt = sig || (it + 1) % kk == 0 || (kkt_last && k == n_iter - 1);
    hipError_t e = enqueue_iteration(s, kkt, sig, it % kk == 0);
    if (e != hipSuccess) return e;
    s->iters++;
    ++k;
  }
  return hipSuccess;
}
// Reads the device scalars; applies the polish switch of the reduced-precision form: the
// FP32 projection is replaced by the FP64 one once eta <= polish_eta, or once eta has not
// halved over 500 iterations.
static void apply_polish_switch(strom_sdp *s) {
  if (!s->f32_active) return;
  const DevState &d = *s->st_host;
  const double eta = std::max(d.eta_p, std::max(d.eta_d, d.eta_g));
  if (eta <= s->opts.polish_eta) {
    s->f32_active = false;
  } else if (s->iters - s->f32_ref_iter >= 500) {
    if (s->f32_ref_iter > 0 && !(eta <= 0.5 * s->f32_ref_eta)) s->f32_active = false;
    s->f32_ref_eta = eta;
    s->f32_ref_iter = s->iters;
  }
}
hipError_t sdp_read_state(strom_sdp *s) {
  hipError_t e = hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return e;
  apply_polish_switch(s);
  return hipSuccess;
}
void sdp_info(strom_sdp *s, strom_info *info) { fill_info(s, info); }
const strom_opts &sdp_opts(strom_sdp *s) { return s->opts; }
}  // namespace strom

extern "C" strom_status strom_admm_step(strom_sdp *s, int32_t n_iter, strom_info *info) {
  if (!s || n_iter < 0) return fail(STROM_E_INVAL, "bad argument");
  if (s->batch) return fail(STROM_E_STATE, "the instance is iterated by a batch");
  HIP_TRY(hipSetDevice(s->ctx->device));
  const double t0 = now_s();
  const int kk = s->opts.kkt_every;
  int done = 0;
  s->state = STROM_RUNNING;
  while (done < n_iter && s->iters < s->opts.maxiter) {
    int chunk = int(std::min<int64_t>(kk - (s->iters % kk), int64_t(n_iter - done)));
    chunk = int(std::min<int64_t>(chunk, s->opts.maxiter - s->iters));
    HIP_TRY(strom::sdp_enqueue(s, chunk, true));
    done += chunk;
    HIP_TRY(strom::sdp_read_state(s));
    if (classify(s) != STROM_RUNNING) break;
  }
  if (n_iter == 0) {
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  s->state = classify(s);
  s->t_solve += now_s() - t0;
  if (info) fill_info(s, info);
  return STROM_OK;
}

extern "C" strom_status strom_admm_enqueue(strom_sdp *s, int32_t n_iter) {
  if (!s || n_iter < 0) return fail(STROM_E_INVAL, "bad argument");
  if (s->batch) return fail(STROM_E_STATE, "the instance is iterated by a batch");
  HIP_TRY(hipSetDevice(s->ctx->device));
  HIP_TRY(strom::sdp_enqueue(s, n_iter, false));
  return STROM_OK;
}

extern "C" strom_status strom_profile_iteration(strom_sdp *s, int32_t reps, strom_phase_times *out) {
  if (!s || reps <= 0 || !out) return fail(STROM_E_INVAL, "bad argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t q = s->stream;
  hipEvent_t ev[11];
  for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
  double acc[6] = {0, 0, 0, 0, 0, 0}, total = 0;
  strom_status rc = STROM_OK;
  for (int r = 0; r < reps && rc == STROM_OK; ++r) {
    const int64_t it = s->iters;
    const bool sig = s->opts.sigma_every > 0 && (it + 1) % s->opts.sigma_every == 0;
    hipError_t e = hipSuccess;
    auto rec = [&](int k) { if (e == hipSuccess) e = hipEventRecord(ev[k], q); };
    rec(0);
    if (!e) e = strom::dev::launch_rhs(q, s->m, s->A_rp, s->A_ci, s->A_v, s->X, s->S, s->C, s->b, s->pinv, s->st, s->w);
    rec(1);
    if (!e) e = strom::dev::launch_solve(q, s->sch, s->sa, s->w, s->y);
    rec(2);
    if (!e) e = strom::dev::launch_xb(q, s->nsvec, s->At_rp, s->At_ci, s->At_v, s->y, s->X, s->C, s->st, s->Xb);
    rec(3);
    if (!e) e = enqueue_projection(s, s->Xb, s->S, 0.0, it % s->opts.kkt_every == 0);
    rec(4);
    if (!e) e = strom::dev::launch_rhs(q, s->m, s->A_rp, s->A_ci, s->A_v, s->X, s->S, s->C, s->b, s->pinv, s->st, s->w);
    rec(5);
    if (!e) e = strom::dev::launch_solve(q, s->sch, s->sa, s->w, s->y);
    rec(6);
    if (!e) e = strom::dev::launch_xupdate(q, s->nsvec, s->At_rp, s->At_ci, s->At_v, s->y, s->S, s->C, s->st, s->X,
                                           s->part_cols, 1);
    rec(7);
    if (!e) e = enqueue_kkt(s, sig);
    rec(8);
    if (!e) e = hipEventSynchronize(ev[8]);
    if (e) { rc = fail(STROM_E_HIP, std::string("profile: ") + hipGetErrorString(e)); break; }
    s->iters++;
    float ms[8];
    for (int k = 0; k < 8; ++k) hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]);
    acc[0] += ms[0] + ms[4];  // both right-hand sides
    acc[1] += ms[1] + ms[5];  // both y-solves
    acc[2] += ms[2];
    acc[3] += ms[3];
    acc[4] += ms[6];
    acc[5] += ms[7];
    float tot;
    hipEventElapsedTime(&tot, ev[0], ev[8]);
    total += tot;
  }
  for (auto &e : ev) hipEventDestroy(e);
  if (rc != STROM_OK) return rc;
  out->rhs_ms = acc[0] / reps;
  out->solve_ms = acc[1] / reps;
  out->xb_ms = acc[2] / reps;
  out->project_ms = acc[3] / reps;
  out->xupdate_ms = acc[4] / reps;
  out->kkt_ms = acc[5] / reps;
  out->iteration_ms = total / reps;
  return STROM_OK;
}

extern "C" strom_status strom_kkt_residuals(strom_sdp *s, strom_info *info) {
  if (!s || !info) return fail(STROM_E_INVAL, "bad argument");
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t q = s->stream;
  // dual residual and <C,X> of the current iterate (no update), then the primal part
  HIP_TRY(strom::dev::launch_xupdate(q, s->nsvec, s->At_rp, s->At_ci, s->At_v, s->y, s->S, s->C, s->st, s->X,
                                     s->part_cols, 0));
  HIP_TRY(enqueue_kkt(s, false));
  HIP_TRY(strom::sdp_read_state(s));
  fill_info(s, info);
  info->state = classify(s);
  return STROM_OK;
}

extern "C" strom_status strom_get_iterate(strom_sdp *s, double *X, double *y, double *S) {
  if (!s) return fail(STROM_E_INVAL, "sdp is NULL");
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  HIP_TRY(hipSetDevice(s->ctx->device));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (X) HIP_TRY(hipMemcpy(X, s->X, sizeof(double) * size_t(s->nsvec), hipMemcpyDeviceToHost));
  if (y) HIP_TRY(hipMemcpy(y, s->y, sizeof(double) * size_t(s->m), hipMemcpyDeviceToHost));
  if (S) HIP_TRY(hipMemcpy(S, s->S, sizeof(double) * size_t(s->nsvec), hipMemcpyDeviceToHost));
  return STROM_OK;
}

extern "C" strom_status strom_set_iterate(strom_sdp *s, const double *X, const double *y, const double *S) {
  if (!s) return fail(STROM_E_INVAL, "sdp is NULL");
  if (s->batch) return fail(STROM_E_STATE, "the instance is iterated by a batch");
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  HIP_TRY(hipSetDevice(s->ctx->device));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (X) HIP_TRY(hipMemcpy(s->X, X, sizeof(double) * size_t(s->nsvec), hipMemcpyHostToDevice));
  if (y) HIP_TRY(hipMemcpy(s->y, y, sizeof(double) * size_t(s->m), hipMemcpyHostToDevice));
  if (S) HIP_TRY(hipMemcpy(s->S, S, sizeof(double) * size_t(s->nsvec), hipMemcpyHostToDevice));
  s->iters = 0;
  s->q_valid = false;
  s->f32_active = s->opts.proj_dtype == STROM_F32;
  s->f32_ref_eta = 0.0;
  s->f32_ref_iter = 0;
  s->state = STROM_RUNNING;
  return STROM_OK;
}

extern "C" strom_status strom_sdp_sizes(strom_sdp *s, int64_t *n_svec, int32_t *m, int64_t *nnz_L) {
  if (!s) return fail(STROM_E_INVAL, "sdp is NULL");
  if (n_svec) *n_svec = s->nsvec;
  if (m) *m = s->m;
  if (nnz_L) *nnz_L = s->nnzL;
  return STROM_OK;
}

namespace {
// max_n of the dense batched calls: within one workgroup's LDS in either precision, or up to
// kBigMaxN in FP64 (the multi-workgroup path).
strom_status check_dense_max_n(const strom_ctx *ctx, int32_t max_n, bool f32) {
  if (max_n <= 0 || max_n > strom::dev::kBigMaxN)
    return fail(STROM_E_INVAL, "max_n out of range (1.." + std::to_string(strom::dev::kBigMaxN) + ")");
  if (f32 && !strom::dev::project_fits(max_n, true, ctx->max_lds))
    return fail(STROM_E_INVAL, "max_n beyond the one-workgroup kernel (122 in FP32) needs FP64 blocks");
  return STROM_OK;
}

// Work memory of a dense multi-workgroup call (every block padded to max_n's size), held until
// the call returns (the call synchronizes its stream before).
struct BigDense {
  strom::dev::BigArgs a;
  void *mem = nullptr;
  strom_status init(strom_ctx *ctx, int32_t nblocks, int32_t max_n, const int32_t *nd, const int64_t *od) {
    a.np = strom::dev::big_padded(max_n);
    a.count = nblocks;
    a.nd = nd;
    a.od = od;
    a.err = ctx->err_flag;
    if (hipMalloc(&mem, sizeof(double) * strom::dev::big_work_doubles(a.np, nblocks)) != hipSuccess) {
      mem = nullptr;
      return fail(STROM_E_NOMEM, "device memory for the multi-workgroup eigensolver");
    }
    a.work = static_cast<double *>(mem);
    return STROM_OK;
  }
  ~BigDense() {
    if (mem) hipFree(mem);  // hipFree waits for the device
  }
};
}  // namespace

extern "C" strom_status strom_project_psd_batched(strom_ctx *ctx, int32_t nblocks, int32_t max_n,
                                                  const int32_t *n_dev, const int64_t *offset_dev,
                                                  const void *in_dev, void *out_dev, strom_dtype dtype,
                                                  void *hip_stream) {
  if (!ctx || nblocks < 0 || (nblocks > 0 && (!n_dev || !offset_dev || !in_dev || !out_dev)))
    return fail(STROM_E_INVAL, "bad argument");
  if (nblocks == 0) return STROM_OK;
  const bool f32 = dtype == STROM_F32;
  if (dtype != STROM_F32 && dtype != STROM_F64) return fail(STROM_E_INVAL, "bad dtype");
  const strom_status vst = check_dense_max_n(ctx, max_n, f32);
  if (vst != STROM_OK) return vst;
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t q = (hipStream_t)hip_stream;
  HIP_TRY(hipMemsetAsync(ctx->err_flag, 0, sizeof(int32_t), q));
  if (strom::dev::project_fits(max_n, f32, ctx->max_lds)) {
    HIP_TRY(strom::dev::launch_project_dense(q, f32, nblocks, max_n, n_dev, offset_dev, in_dev, out_dev, ctx->err_flag));
  } else {
    BigDense bd;
    const strom_status bst = bd.init(ctx, nblocks, max_n, n_dev, offset_dev);
    if (bst != STROM_OK) return bst;
    HIP_TRY(strom::dev::launch_project_big_dense(q, bd.a, static_cast<const double *>(in_dev), static_cast<double *>(out_dev)));
  }
  int32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, ctx->err_flag, sizeof(int32_t), hipMemcpyDeviceToHost, q));
  HIP_TRY(hipStreamSynchronize(q));
  if (flag) return fail(STROM_E_INVAL, "a block size is <= 0 or > max_n");
  return STROM_OK;
}

// ------------------------------------------------------------------ serving entry points
extern "C" strom_status strom_eig_batched(strom_ctx *ctx, int32_t nblocks, int32_t max_n, const int32_t *n_dev,
                                          const int64_t *offset_dev, const void *in_dev, const int64_t *woff_dev,
                                          void *w_dev, void *v_dev, strom_dtype dtype, void *hip_stream) {
  if (!ctx || nblocks < 0 || (nblocks > 0 && (!n_dev || !offset_dev || !in_dev || !woff_dev || !w_dev)))
    return fail(STROM_E_INVAL, "bad argument");
  if (nblocks == 0) return STROM_OK;
  const bool f32 = dtype == STROM_F32;
  if (dtype != STROM_F32 && dtype != STROM_F64) return fail(STROM_E_INVAL, "bad dtype");
  const strom_status vst = check_dense_max_n(ctx, max_n, f32);
  if (vst != STROM_OK) return vst;
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t q = (hipStream_t)hip_stream;
  HIP_TRY(hipMemsetAsync(ctx->err_flag, 0, sizeof(int32_t), q));
  if (strom::dev::project_fits(max_n, f32, ctx->max_lds)) {
    HIP_TRY(strom::dev::launch_eig_dense(q, f32, nblocks, max_n, n_dev, offset_dev, in_dev, woff_dev, w_dev, v_dev,
                                         ctx->err_flag));
  } else {
    BigDense bd;
    const strom_status bst = bd.init(ctx, nblocks, max_n, n_dev, offset_dev);
    if (bst != STROM_OK) return bst;
    HIP_TRY(strom::dev::launch_eig_big_dense(q, bd.a, static_cast<const double *>(in_dev), woff_dev,
                                             static_cast<double *>(w_dev), static_cast<double *>(v_dev)));
  }
  int32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, ctx->err_flag, sizeof(int32_t), hipMemcpyDeviceToHost, q));
  HIP_TRY(hipStreamSynchronize(q));
  if (flag) return fail(STROM_E_INVAL, "a block size is <= 0 or > max_n");
  return STROM_OK;
}

namespace {
// Eigenvalues (and, with want_v, eigenvectors) of the listed blocks of the svec vector sv of
// an instance, through dense copies in temporary device memory.  w: per listed block its n
// eigenvalues in ascending order, concatenated; v: per listed block its n x n eigenvectors
// (column j for eigenvalue j), concatenated.
strom_status block_eigs(strom_sdp *s, const double *sv, const std::vector<int32_t> &list, bool want_v,
                        std::vector<double> &w, std::vector<double> &v, const strom::DeviceBuf *work = nullptr) {
  const size_t nl = list.size();
  std::vector<int64_t> od(nl), wo(nl);
  std::vector<int32_t> nd(nl);
  int64_t tn = 0, tn2 = 0;
  int32_t mx = 1;
  for (size_t k = 0; k < nl; ++k) {
    const int32_t n = s->bsize_h[size_t(list[k])];
    nd[k] = n;
    od[k] = tn2;
    wo[k] = tn;
    tn2 += int64_t(n) * n;
    tn += n;
    mx = std::max(mx, n);
  }
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  HIP_TRY(hipSetDevice(s->ctx->device));
  hipStream_t q = s->stream;
  HIP_TRY(hipStreamSynchronize(q));
  const bool big = !fits_lds(s->ctx, mx);  // the multi-workgroup eigensolver, every block padded to mx's size
  const size_t big_doubles = big ? strom::dev::big_work_doubles(strom::dev::big_padded(mx), int(nl)) : 0;
  const size_t bytes = sizeof(int32_t) * nl * 2 + sizeof(int64_t) * nl * 2 + sizeof(double) * size_t(tn) +
                       sizeof(double) * size_t(tn2) * (want_v ? 2 : 1) + sizeof(double) * big_doubles +
                       8 * 256;  // + alignment of 8 regions
  unsigned char *buf = nullptr;
  if (work) {  // the caller's device buffer (no allocation)
    if (bytes > work->bytes)
      return fail(STROM_E_INVAL, "the blocks need " + std::to_string(bytes) + " bytes of work memory, the buffer holds " +
                                     std::to_string(work->bytes));
    buf = work->base;
  } else if (hipMalloc(&buf, bytes) != hipSuccess) {
    return fail(STROM_E_NOMEM, "device memory for the block eigenvalues");
  }
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t o = 0;
  int32_t *d_ids = reinterpret_cast<int32_t *>(buf + o); o = al(o + sizeof(int32_t) * nl);
  int32_t *d_nd = reinterpret_cast<int32_t *>(buf + o); o = al(o + sizeof(int32_t) * nl);
  int64_t *d_od = reinterpret_cast<int64_t *>(buf + o); o = al(o + sizeof(int64_t) * nl);
  int64_t *d_wo = reinterpret_cast<int64_t *>(buf + o); o = al(o + sizeof(int64_t) * nl);
  double *d_w = reinterpret_cast<double *>(buf + o); o = al(o + sizeof(double) * size_t(tn));
  double *d_dense = reinterpret_cast<double *>(buf + o); o = al(o + sizeof(double) * size_t(tn2));
  double *d_v = want_v ? reinterpret_cast<double *>(buf + o) : nullptr;
  if (want_v) o = al(o + sizeof(double) * size_t(tn2));
  double *d_big = reinterpret_cast<double *>(buf + o);
  strom_status st = STROM_OK;
  std::string msg;
  auto chk = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && st == STROM_OK) { st = STROM_E_HIP; msg = std::string(what) + ": " + hipGetErrorString(e); }
  };
  chk(hipMemcpy(d_ids, list.data(), sizeof(int32_t) * nl, hipMemcpyHostToDevice), "upload");
  chk(hipMemcpy(d_nd, nd.data(), sizeof(int32_t) * nl, hipMemcpyHostToDevice), "upload");
  chk(hipMemcpy(d_od, od.data(), sizeof(int64_t) * nl, hipMemcpyHostToDevice), "upload");
  chk(hipMemcpy(d_wo, wo.data(), sizeof(int64_t) * nl, hipMemcpyHostToDevice), "upload");
  chk(hipMemsetAsync(s->ctx->err_flag, 0, sizeof(int32_t), q), "hipMemsetAsync");
  chk(strom::dev::launch_unpack_svec(q, int(nl), d_ids, s->boff, s->bsz, sv, d_od, d_dense), "unpack");
  if (big) {
    strom::dev::BigArgs a;
    a.np = strom::dev::big_padded(mx);
    a.count = int32_t(nl);
    a.nd = d_nd;
    a.od = d_od;
    a.work = d_big;
    a.err = s->ctx->err_flag;
    chk(strom::dev::launch_eig_big_dense(q, a, d_dense, d_wo, d_w, d_v), "eigenvalues");
  } else {
    chk(strom::dev::launch_eig_dense(q, false, int(nl), mx, d_nd, d_od, d_dense, d_wo, d_w, d_v, s->ctx->err_flag),
        "eigenvalues");
  }
  chk(hipStreamSynchronize(q), "hipStreamSynchronize");
  w.resize(size_t(tn));
  chk(hipMemcpy(w.data(), d_w, sizeof(double) * size_t(tn), hipMemcpyDeviceToHost), "download");
  if (want_v) {
    v.resize(size_t(tn2));
    chk(hipMemcpy(v.data(), d_v, sizeof(double) * size_t(tn2), hipMemcpyDeviceToHost), "download");
  }
  if (!work) hipFree(buf);
  if (st != STROM_OK) return fail(st, msg);
  return STROM_OK;
}
}  // namespace

namespace strom {
int sdp_device(const strom_sdp *s) { return s->ctx->device; }

strom_status set_error(strom_status st, const std::string &msg) { return fail(st, msg); }

// The dual bound with its temporary device memory in `work` (nullptr: allocated per call).
strom_status dual_bound_impl(strom_sdp *s, const double *R_beta, double *lb, double *lam_min,
                             const DeviceBuf *work) {
  if (!s || !R_beta || !lb) return fail(STROM_E_INVAL, "bad argument");
  strom_info inf{};
  const strom_status kst = strom_kkt_residuals(s, &inf);  // <b, y> of the current iterate
  if (kst != STROM_OK) return kst;
  {
    std::lock_guard<std::recursive_mutex> dl(device_lock());
    HIP_TRY(hipSetDevice(s->ctx->device));
    // Z = C - A^* y into the X_b work buffer (free between iterations)
    HIP_TRY(strom::dev::launch_slack(s->stream, s->nsvec, s->At_rp, s->At_ci, s->At_v, s->y, s->C, s->Xb));
  }
  std::vector<int32_t> all(size_t(s->nblocks));
  for (int32_t k = 0; k < s->nblocks; ++k) all[size_t(k)] = k;
  std::vector<double> w, v;
  const strom_status est = block_eigs(s, s->Xb, all, false, w, v, work);
  if (est != STROM_OK) return est;
  double bound = inf.dobj;
  int64_t wo = 0;
  for (int32_t k = 0; k < s->nblocks; ++k) {
    const double lmin = w[size_t(wo)];
    if (lam_min) lam_min[k] = lmin;
    bound += R_beta[k] * std::min(0.0, lmin);
    wo += s->bsize_h[size_t(k)];
  }
  *lb = bound;
  return STROM_OK;
}
}  // namespace strom

extern "C" strom_status strom_dual_bound(strom_sdp *s, const double *R_beta, double *lb, double *lam_min) {
  return strom::dual_bound_impl(s, R_beta, lb, lam_min, nullptr);
}

extern "C" strom_status strom_extract(strom_sdp *s, int32_t nlist, const int32_t *blocks, double *lam, double *vtop) {
  if (!s || nlist < 0 || (nlist > 0 && (!blocks || !lam || !vtop))) return fail(STROM_E_INVAL, "bad argument");
  if (nlist == 0) return STROM_OK;
  std::vector<int32_t> list(blocks, blocks + nlist);
  for (int32_t b : list)
    if (b < 0 || b >= s->nblocks) return fail(STROM_E_INVAL, "block index out of range");
  std::vector<double> w, v;
  const strom_status est = block_eigs(s, s->X, list, true, w, v);
  if (est != STROM_OK) return est;
  int64_t wo = 0, vo = 0, out = 0;
  for (int32_t k = 0; k < nlist; ++k) {
    const int32_t n = s->bsize_h[size_t(list[size_t(k)])];
    lam[2 * k] = w[size_t(wo + n - 1)];
    lam[2 * k + 1] = n >= 2 ? w[size_t(wo + n - 2)] : 0.0;
    const double *top = v.data() + vo + int64_t(n - 1) * n;  // eigenvector of the largest eigenvalue
    double scale = top[0];
    if (scale == 0.0) {  // no leading entry to normalize by: unit norm, largest entry positive
      int ia = 0;
      for (int i = 1; i < n; ++i)
        if (std::fabs(top[i]) > std::fabs(top[ia])) ia = i;
      scale = top[ia] < 0 ? -1.0 : 1.0;
    }
    for (int i = 0; i < n; ++i) vtop[out + i] = top[i] / scale;
    wo += n;
    vo += int64_t(n) * n;
    out += n;
  }
  return STROM_OK;
}

// ------------------------------------------------------------------ merged form
struct strom_batch {
  strom_ctx *ctx = nullptr;
  std::vector<strom_sdp *> inst;
  hipStream_t stream = nullptr;  // the context's stream
  int kk = 10, se = 50;          // kkt_every and sigma_every shared by the instances
  int phase = 0;                 // iteration count of every instance modulo kk
  unsigned char *arena = nullptr;
  strom::dev::BatchInst *bi_dev = nullptr, *bi_host = nullptr;  // bi_host: pinned mirror
  strom::dev::SolveArgs *sa_dev = nullptr;
  strom::dev::BatchItem *rows = nullptr, *cols = nullptr, *fwd = nullptr, *bwd = nullptr, *blocks = nullptr;
  int nrows = 0, ncols = 0;
  std::vector<int32_t> fwd_gptr, bwd_gptr;  // merged solve groups (by dependency depth)
  // projection classes: blocks of one size and one default thread count; nt[0] FP64, nt[1] FP32
  struct Cls {
    int n, off, cnt, nt[2];
  };
  std::vector<Cls> cls;
  bool any_f32 = false;  // an instance was set up with the FP32 projection
  size_t solve_lds = 0;
  DevState *states_dev = nullptr, *states_host = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // one round, [sigma rule for some instance at its end]
  hipStream_t capture_stream = nullptr;
  bool graphs = true;
};

namespace {

hipError_t batch_projection(strom_batch *b, hipStream_t q, int cone, bool reorth) {
  for (const auto &c : b->cls) {
    hipError_t e = strom::dev::launch_project_batch(q, false, c.n, c.nt[0], c.cnt, b->blocks + c.off, b->bi_dev, cone,
                                                    reorth);
    if (e != hipSuccess) return e;
    if (b->any_f32 && (e = strom::dev::launch_project_batch(q, true, c.n, c.nt[1], c.cnt, b->blocks + c.off,
                                                            b->bi_dev, cone, reorth)))
      return e;
  }
  return hipSuccess;
}

// One iteration of every running instance (the steps of enqueue_iteration, merged); first: the
// iteration opens a round.
hipError_t batch_iteration(strom_batch *b, hipStream_t q, bool kkt, bool sig, bool first) {
  using namespace strom::dev;
  hipError_t e;
  for (int half = 0; half < 2; ++half) {
    if ((e = launch_rhs_batch(q, b->nrows, b->rows, b->ncols, b->cols, b->bi_dev))) return e;
    if ((e = launch_solve_batch(q, b->fwd_gptr, b->fwd, b->bwd_gptr, b->bwd, b->sa_dev, b->bi_dev, b->solve_lds)))
      return e;
    if (half == 0) {
      if ((e = launch_xb_batch(q, b->ncols, b->cols, b->bi_dev))) return e;
      if ((e = batch_projection(b, q, 0, first))) return e;
    }
  }
  if ((e = launch_xupdate_batch(q, b->ncols, b->cols, b->bi_dev, kkt ? 1 : 0))) return e;
  if (kkt) {
    if (sig && (e = batch_projection(b, q, 1, true))) return e;
    if ((e = launch_kkt_batch(q, b->nrows, b->rows, b->ncols, b->cols, int(b->inst.size()), b->bi_dev, sig ? 1 : 0)))
      return e;
  }
  return hipSuccess;
}

hipError_t batch_capture(strom_batch *b, bool sigma_last, hipGraphExec_t *out) {
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  hipError_t e = hipSuccess;
  if (!b->capture_stream && (e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking))) return e;
  e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
  hipError_t e2 = hipSuccess;
  for (int k = 0; k < b->kk && e == hipSuccess && e2 == hipSuccess; ++k)
    e2 = batch_iteration(b, b->capture_stream, k == b->kk - 1, sigma_last && k == b->kk - 1, k == 0);
  hipGraph_t g = nullptr;
  if (e == hipSuccess) e = hipStreamEndCapture(b->capture_stream, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) hipGraphDestroy(g);
  return e;
}

void batch_drop_graphs(strom_batch *b) {
  for (auto &g : b->graph)
    if (g) {
      hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Flags of every instance for the next launches (a round of `chunk` iterations; chunk < 0:
// every running instance takes the sigma-rule projection, as the autotuner's launches do),
// copied on the batch stream; the pinned host copy is not written again before that stream
// has been synchronized.
hipError_t batch_upload_flags(strom_batch *b, int chunk) {
  for (size_t i = 0; i < b->inst.size(); ++i) {
    const strom_sdp *s = b->inst[i];
    auto &I = b->bi_host[i];
    I.active = s->state == STROM_RUNNING ? 1 : 0;
    I.f32 = s->f32_active ? 1 : 0;
    I.warm = s->q_valid ? 1 : 0;
    I.sig = I.active && (chunk < 0 || (b->se > 0 && (s->iters + chunk) % b->se == 0)) ? 1 : 0;
  }
  return hipMemcpyAsync(b->bi_dev, b->bi_host, sizeof(strom::dev::BatchInst) * b->inst.size(), hipMemcpyHostToDevice,
                        b->stream);
}

}  // namespace

extern "C" strom_status strom_batch_create(strom_ctx *ctx, int32_t count, strom_sdp *const *instances,
                                           strom_batch **out) {
  using strom::dev::BatchInst;
  using strom::dev::BatchItem;
  using strom::dev::SolveArgs;
  if (!ctx || !instances || !out || count <= 0) return fail(STROM_E_INVAL, "bad argument");
  *out = nullptr;
  std::vector<strom_sdp *> v(instances, instances + count);
  for (int32_t i = 0; i < count; ++i) {
    const strom_sdp *s = v[size_t(i)];
    if (!s) return fail(STROM_E_INVAL, "instance " + std::to_string(i) + " is NULL");
    if (s->ctx != ctx) return fail(STROM_E_INVAL, "instance " + std::to_string(i) + " belongs to another context");
    if (s->batch) return fail(STROM_E_STATE, "instance " + std::to_string(i) + " already belongs to a batch");
    if (s->big.count > 0)
      return fail(STROM_E_INVAL, "instance " + std::to_string(i) +
                                     " has blocks beyond one workgroup's LDS; those instances iterate on their own");
    if (s->opts.kkt_every != v[0]->opts.kkt_every || s->opts.sigma_every != v[0]->opts.sigma_every)
      return fail(STROM_E_INVAL, "the instances of a batch need the same kkt_every and sigma_every");
    if (s->iters % s->opts.kkt_every != v[0]->iters % v[0]->opts.kkt_every)
      return fail(STROM_E_INVAL, "the iteration counts of a batch's instances must agree modulo kkt_every");
    for (int32_t j = 0; j < i; ++j)
      if (v[size_t(j)] == s) return fail(STROM_E_INVAL, "instance listed twice");
  }
  auto *b = new strom_batch();
  b->ctx = ctx;
  b->inst = v;
  b->stream = ctx->stream;
  b->kk = v[0]->opts.kkt_every;
  b->se = v[0]->opts.sigma_every;
  b->phase = int(v[0]->iters % b->kk);

  std::vector<BatchInst> bi(static_cast<size_t>(count));
  std::vector<SolveArgs> sa(static_cast<size_t>(count));
  std::vector<BatchItem> rows, cols, fwd, bwd, blocks;
  size_t gf = 0, gb = 0;
  std::map<std::pair<int, int>, std::vector<BatchItem>> by_cls;
  for (int32_t i = 0; i < count; ++i) {
    strom_sdp *s = v[size_t(i)];
    BatchInst &I = bi[size_t(i)];
    I.m = s->m;
    I.nrow_chunks = (s->m + 255) / 256;
    I.n = s->nsvec;
    I.ncol_chunks = int32_t((s->nsvec + 255) / 256);
    I.A_rp = s->A_rp; I.At_rp = s->At_rp; I.boff = s->boff; I.qoff = s->qoff;
    I.A_ci = s->A_ci; I.At_ci = s->At_ci; I.pinv = s->pinv; I.bsz = s->bsz;
    I.A_v = s->A_v; I.At_v = s->At_v; I.b = s->b; I.C = s->C;
    I.X = s->X; I.S = s->S; I.Xb = s->Xb; I.y = s->y; I.w = s->w;
    I.part_rows = s->part_rows; I.part_cols = s->part_cols; I.part_cone = s->part_cone; I.Q = s->Q;
    I.st = s->st;
    I.normb = s->normb;
    I.normC = s->normC;
    sa[size_t(i)] = s->sa;
    for (int32_t c = 0; c < I.nrow_chunks; ++c) rows.push_back({i, c});
    for (int32_t c = 0; c < I.ncol_chunks; ++c) cols.push_back({i, c});
    gf = std::max(gf, s->sch.fwd_gptr.size() - 1);
    gb = std::max(gb, s->sch.bwd_gptr.size() - 1);
    const size_t lds = sizeof(double) * size_t(strom::kSolveThreads * 3 / 2 + s->sa.lds_rows + s->sa.c_cap);
    b->solve_lds = std::max(b->solve_lds, lds);
    b->any_f32 |= s->opts.proj_dtype == STROM_F32;
    // a block keeps the thread count of its own launch: one launch over every block (the
    // largest's count) when the instance has a single projection class, else its size's
    const bool merged = s->cls_n.size() == 1;
    for (int32_t k = 0; k < s->nblocks; ++k) {
      const int nk = s->bsize_h[size_t(k)];
      by_cls[{nk, strom::dev::project_threads(merged ? s->cls_n[0] : nk)}].push_back({i, k});
    }
  }
  // group g of every instance in one launch, its longest tasks first: workgroups start
  // roughly in item order, so the launch does not end on a long task started last
  auto merge = [&](size_t ng, bool forward, std::vector<BatchItem> &items, std::vector<int32_t> &gptr) {
    gptr.assign(1, 0);
    for (size_t g = 0; g < ng; ++g) {
      const size_t first = items.size();
      for (int32_t i = 0; i < count; ++i) {
        const auto &sch = v[size_t(i)]->sch;
        const auto &gp = forward ? sch.fwd_gptr : sch.bwd_gptr;
        const auto &order = forward ? sch.fwd_order : sch.bwd_order;
        if (g + 1 >= gp.size()) continue;
        for (int32_t k = gp[g]; k < gp[g + 1]; ++k) items.push_back({i, order[size_t(k)]});
      }
      auto cost = [&](const BatchItem &it) {
        const auto &sch = v[size_t(it.inst)]->sch;
        return (forward ? sch.fwd_cost : sch.bwd_cost)[size_t(it.idx)];
      };
      std::stable_sort(items.begin() + long(first), items.end(),
                       [&](const BatchItem &a, const BatchItem &b) { return cost(a) > cost(b); });
      gptr.push_back(int32_t(items.size()));
    }
  };
  merge(gf, true, fwd, b->fwd_gptr);
  merge(gb, false, bwd, b->bwd_gptr);
  for (auto it = by_cls.rbegin(); it != by_cls.rend(); ++it) {  // largest blocks first
    const int nt = it->first.second;
    b->cls.push_back({it->first.first, int(blocks.size()), int(it->second.size()), {nt, nt}});
    blocks.insert(blocks.end(), it->second.begin(), it->second.end());
  }
  b->nrows = int(rows.size());
  b->ncols = int(cols.size());

  Arena ar;
  const size_t oBi = ar.reserve<BatchInst>(size_t(count)), oSa = ar.reserve<SolveArgs>(size_t(count)),
               oRows = ar.reserve<BatchItem>(rows.size()), oCols = ar.reserve<BatchItem>(cols.size()),
               oFwd = ar.reserve<BatchItem>(fwd.size()), oBwd = ar.reserve<BatchItem>(bwd.size()),
               oBlk = ar.reserve<BatchItem>(blocks.size()), oSt = ar.reserve<DevState>(size_t(count));
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  auto undo = [&](strom_status st, const std::string &msg) {
    if (b->arena) hipFree(b->arena);
    if (b->bi_host) hipHostFree(b->bi_host);
    if (b->states_host) hipHostFree(b->states_host);
    delete b;
    return fail(st, msg);
  };
  if (hipSetDevice(ctx->device) != hipSuccess) return undo(STROM_E_HIP, "hipSetDevice failed");
  if (hipStreamSynchronize(b->stream) != hipSuccess) return undo(STROM_E_HIP, "stream synchronization failed");
  if (hipMalloc(&b->arena, ar.bytes) != hipSuccess) return undo(STROM_E_NOMEM, "hipMalloc of the batch tables failed");
  if (hipHostMalloc(&b->bi_host, sizeof(BatchInst) * size_t(count), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&b->states_host, sizeof(DevState) * size_t(count), hipHostMallocDefault) != hipSuccess)
    return undo(STROM_E_NOMEM, "hipHostMalloc failed");
  unsigned char *base = b->arena;
  b->bi_dev = reinterpret_cast<BatchInst *>(base + oBi);
  b->sa_dev = reinterpret_cast<SolveArgs *>(base + oSa);
  b->rows = reinterpret_cast<BatchItem *>(base + oRows);
  b->cols = reinterpret_cast<BatchItem *>(base + oCols);
  b->fwd = reinterpret_cast<BatchItem *>(base + oFwd);
  b->bwd = reinterpret_cast<BatchItem *>(base + oBwd);
  b->blocks = reinterpret_cast<BatchItem *>(base + oBlk);
  b->states_dev = reinterpret_cast<DevState *>(base + oSt);
  std::memcpy(b->bi_host, bi.data(), sizeof(BatchInst) * bi.size());
  bool ok = true;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    if (bytes) ok &= hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  up(b->bi_dev, bi.data(), sizeof(BatchInst) * bi.size());
  up(b->sa_dev, sa.data(), sizeof(SolveArgs) * sa.size());
  up(b->rows, rows.data(), sizeof(BatchItem) * rows.size());
  up(b->cols, cols.data(), sizeof(BatchItem) * cols.size());
  up(b->fwd, fwd.data(), sizeof(BatchItem) * fwd.size());
  up(b->bwd, bwd.data(), sizeof(BatchItem) * bwd.size());
  up(b->blocks, blocks.data(), sizeof(BatchItem) * blocks.size());
  if (!ok) return undo(STROM_E_HIP, "upload of the batch tables failed");
  for (strom_sdp *s : v) s->batch = b;
  *out = b;
  return STROM_OK;
}

extern "C" strom_status strom_batch_step(strom_batch *b, int32_t n_iter, strom_info *infos) {
  if (!b || n_iter < 0) return fail(STROM_E_INVAL, "bad argument");
  HIP_TRY(hipSetDevice(b->ctx->device));
  const double t0 = now_s();
  const size_t K = b->inst.size();
  std::vector<char> ran(K, 0);
  int done = 0;
  while (done < n_iter) {
    int64_t room = INT64_MAX;
    bool all_warm = true;
    for (const strom_sdp *s : b->inst)
      if (s->state == STROM_RUNNING) {
        room = std::min(room, s->opts.maxiter - s->iters);
        all_warm &= s->q_valid;
      }
    if (room == INT64_MAX) break;  // every instance retired
    const int chunk = int(std::min<int64_t>(std::min<int64_t>(b->kk - b->phase, n_iter - done), room));
    if (chunk <= 0) break;
    HIP_TRY(batch_upload_flags(b, chunk));
    bool any_sig = false;
    for (size_t i = 0; i < K; ++i) any_sig |= b->bi_host[i].sig != 0;
    bool launched = false;
    if (b->graphs && all_warm && chunk == b->kk) {
      const int sl = any_sig ? 1 : 0;
      if (!b->graph[sl] && batch_capture(b, sl != 0, &b->graph[sl]) != hipSuccess) {
        b->graphs = false;  // capture not available: launch directly from now on
        b->graph[sl] = nullptr;
        (void)hipGetLastError();
      }
      if (b->graph[sl]) {
        HIP_TRY(hipGraphLaunch(b->graph[sl], b->stream));
        launched = true;
      }
    }
    for (int k = 0; !launched && k < chunk; ++k) {
      HIP_TRY(batch_iteration(b, b->stream, k == chunk - 1, any_sig && k == chunk - 1, (b->phase + k) % b->kk == 0));
      if (k == 0 && !all_warm) {  // the first projection has filled every running instance's Q
        for (strom_sdp *s : b->inst)
          if (s->state == STROM_RUNNING) s->q_valid = true;
        HIP_TRY(hipStreamSynchronize(b->stream));
        HIP_TRY(batch_upload_flags(b, chunk));
      }
    }
    b->phase = (b->phase + chunk) % b->kk;
    done += chunk;
    HIP_TRY(strom::dev::launch_gather_states(b->stream, int(K), b->bi_dev, b->states_dev));
    HIP_TRY(hipMemcpyAsync(b->states_host, b->states_dev, sizeof(DevState) * K, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < K; ++i) {
      strom_sdp *s = b->inst[i];
      if (s->state != STROM_RUNNING) continue;
      ran[i] = 1;
      s->iters += chunk;
      s->q_valid = true;
      *s->st_host = b->states_host[i];
      strom::apply_polish_switch(s);
      s->state = classify(s);
    }
  }
  const double dt = now_s() - t0;
  for (size_t i = 0; i < K; ++i) {
    if (ran[i]) b->inst[i]->t_solve += dt;
    if (infos) fill_info(b->inst[i], &infos[i]);
  }
  return STROM_OK;
}

extern "C" strom_status strom_batch_tune(strom_batch *b, int32_t reps, int32_t cap, int32_t *n, int32_t *nt_f64,
                                         int32_t *nt_f32, int32_t *nclass) {
  if (!b || reps < 0 || cap < 0) return fail(STROM_E_INVAL, "bad argument");
  if (reps > 0) {
    bool any = false, has[2] = {false, false};
    for (const strom_sdp *s : b->inst) {
      if (s->state != STROM_RUNNING) continue;
      if (!s->q_valid) return fail(STROM_E_STATE, "tuning needs a completed iteration");
      any = true;
      has[s->f32_active ? 1 : 0] = true;
    }
    if (any) {
      HIP_TRY(hipSetDevice(b->ctx->device));
      HIP_TRY(batch_upload_flags(b, -1));
      hipEvent_t e0 = nullptr, e1 = nullptr;
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      hipError_t err = hipSuccess;
      for (auto &c : b->cls) {
        for (int prec = 0; prec < 2 && err == hipSuccess; ++prec) {
          if (!has[prec]) continue;
          int opt[5];
          const int no = strom::dev::project_thread_options(c.n, prec == 1, opt);
          float best = 0.0f;
          int best_nt = c.nt[prec];
          for (int j = 0; j < no && err == hipSuccess; ++j) {
            auto launch = [&]() {
              return strom::dev::launch_project_batch(b->stream, prec == 1, c.n, opt[j], c.cnt, b->blocks + c.off,
                                                      b->bi_dev, 1, false);
            };
            if ((err = launch())) break;  // untimed first launch
            if ((err = hipEventRecord(e0, b->stream))) break;
            for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch();
            if (err || (err = hipEventRecord(e1, b->stream)) || (err = hipEventSynchronize(e1))) break;
            float ms = 0.0f;
            if ((err = hipEventElapsedTime(&ms, e0, e1))) break;
            if (j == 0 || ms < best) {
              best = ms;
              best_nt = opt[j];
            }
          }
          c.nt[prec] = best_nt;
        }
      }
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      batch_drop_graphs(b);
      if (err != hipSuccess) return fail(STROM_E_HIP, std::string("tuning launch failed: ") + hipGetErrorString(err));
    }
  }
  for (int32_t c = 0; c < cap && c < int32_t(b->cls.size()); ++c) {
    if (n) n[c] = b->cls[size_t(c)].n;
    if (nt_f64) nt_f64[c] = b->cls[size_t(c)].nt[0];
    if (nt_f32) nt_f32[c] = b->cls[size_t(c)].nt[1];
  }
  if (nclass) *nclass = int32_t(b->cls.size());
  return STROM_OK;
}

extern "C" strom_status strom_batch_destroy(strom_batch *b) {
  if (!b) return fail(STROM_E_INVAL, "batch is NULL");
  std::lock_guard<std::recursive_mutex> dl(device_lock());
  hipSetDevice(b->ctx->device);
  hipStreamSynchronize(b->stream);
  batch_drop_graphs(b);
  if (b->capture_stream) hipStreamDestroy(b->capture_stream);
  hipFree(b->arena);
  hipHostFree(b->bi_host);
  hipHostFree(b->states_host);
  for (strom_sdp *s : b->inst) s->batch = nullptr;
  delete b;
  return STROM_OK;
}

extern "C" strom_status strom_submit(strom_ctx *ctx, const strom_problem *P, const strom_opts *opts,
                                     uint64_t *ticket) {
  if (!ctx || !P || !ticket) return fail(STROM_E_INVAL, "NULL argument");
  // the request loop iterates merged batches, which take blocks of the one-workgroup projection
  // only; a problem with larger blocks is set up and iterated on its own (strom_sdp_setup)
  if (P->block_sizes)
    for (int32_t k = 0; k < P->nblocks; ++k)
      if (P->block_sizes[k] > 0 && !fits_lds(ctx, P->block_sizes[k]))
        return fail(STROM_E_INVAL, "block of size " + std::to_string(P->block_sizes[k]) +
                                       " is beyond the one-workgroup projection, which the request loop needs");
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->server) ctx->server = strom::server_start(ctx);
  }
  std::string err;
  strom_status rc = strom::server_submit(ctx->server, P, opts, ticket, err);
  if (rc != STROM_OK) return fail(rc, err);
  return STROM_OK;
}

extern "C" strom_status strom_poll(strom_ctx *ctx, uint64_t ticket, strom_info *out, double *X, double *y,
                                   double *S) {
  if (!ctx) return fail(STROM_E_INVAL, "ctx is NULL");
  if (!ctx->server) return fail(STROM_E_NOTFOUND, "no submitted problems");
  std::string err;
  strom_status rc = strom::server_poll(ctx->server, ticket, out, X, y, S, err);
  if (rc != STROM_OK && rc != STROM_E_AGAIN) return fail(rc, err);
  if (rc == STROM_E_AGAIN) g_err = "in flight";
  return rc;
}
