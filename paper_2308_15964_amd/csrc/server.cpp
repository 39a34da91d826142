// Serving loop of libspx: admission of SPD solve requests by an HBM budget and continuous
// batching over worker lanes (one HIP stream and context each).  Every batch a lane takes
// runs as one persistent-kernel launch over all of its requests' task graphs (Specx
// Sec. 4.1: one engine, several graphs), so the device work of the requests in a batch
// overlaps, and batches of different lanes overlap with each other.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "spx_internal.h"

namespace spx {
namespace {

enum ReqState { WAITING, ADMITTED, RUNNING, DONE };

struct Req {
  spx_request r;
  size_t bytes = 0;
  int tile = 0;
  ReqState state = WAITING;
  spx_result res{};
};

struct Lane {
  spx_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  std::thread th;
};

// One FP64 request of a running batch, watched by the monitor thread: its STORE task
// raises *hflag once X is final in device memory; for host-memory requests the monitor
// then copies X back on its own stream.
struct Watch {
  volatile unsigned int* hflag = nullptr;
  bool copy = false;
  void* dst = nullptr;
  size_t dpitch = 0, spitch = 0, width = 0, height = 0;
  const void* src = nullptr;
  hipEvent_t ev = nullptr;
  std::atomic<int> state{0};  // 0 running, 1 copy issued, 2 X in place
  double t_ready = 0.0;
};

constexpr int kFlagSlots = 1 << 16;  // completion flags in pinned host memory
// Default: mixed-mode requests below this size run in FP64.  Measured on batches of equal
// requests (8 RHS, one lane), mixed over FP64 throughput: 0.26 at N = 2048, 0.58 at 4096,
// 0.90 at 8192, 1.00 at 16384: below that the FP32 updates save less than the refinement
// launches cost.
constexpr int64_t kMixedMinN = 16384;

// Stream-ordered device allocations from the device's default memory pool, so lanes do
// not serialise on the allocator and freed blocks are reused.
void* pool_alloc(size_t bytes, void* stream, void*) {
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, (hipStream_t)stream) != hipSuccess) return nullptr;
  return p;
}
void pool_free(void* p, void* stream, void*) { (void)hipFreeAsync(p, (hipStream_t)stream); }

}  // namespace
}  // namespace spx

using namespace spx;

struct spx_server {
  int device = 0;
  size_t budget = 0;
  spx_server_opts opts{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> waiting;   // arrival order
  std::deque<uint64_t> admitted;  // admission order
  std::vector<Lane> lanes;
  spx_server_stats st{};
  uint64_t running = 0;
  // completion flags (pinned, device-visible) and the monitor that watches them
  unsigned int* flags_h = nullptr;
  unsigned int* flags_d = nullptr;
  std::vector<int> free_slots;  // guarded by mu
  std::mutex mon_mu;
  std::vector<Watch*> watches;  // guarded by mon_mu
  std::atomic<bool> mon_stop{false};
  hipStream_t mon_stream = nullptr;
  std::thread monitor;
  spx_ctx* tuner = nullptr;  // holds the tile tables (copied from the creating context)

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace spx {
namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device bytes a request holds while it runs (what the batched calls and the refinement
// allocate for it, plus device copies of host inputs).
//   FP64: one-shot factor + solve: tiles, 32x32 block inverses, one right-hand-side copy.
//   mixed: kept factor (tiles, block inverses, the tile inverses M_k = L_kk^{-T}, the FP32
//   panel copies) and the two right-hand-side copies of its solves, plus the residual and
//   the refinement buffers.
size_t request_bytes(const spx_request& r, int b) {
  const size_t n = (size_t)r.n, q = (size_t)r.nrhs, nt = (n + b - 1) / b, npad = nt * b;
  const size_t tiles = nt * (nt + 1) / 2 * (size_t)b * b * 8;
  size_t s = align256(tiles) + align256(npad * 32 * 8) + align256(npad * q * 8);
  if (r.mode == SPX_MODE_MIXED)
    s += align256(npad * (size_t)b * 8) + align256(tiles / 2) + 2 * align256(n * q * 8) + align256(npad * q * 8);
  if (r.where == 0) s += align256(n * n * 8) + align256(n * q * 8) + align256(n * q * 8);
  if (r.where == 2) s += align256(n * q * 8);  // the device copy of X
  return s;
}

// Moves waiting requests that fit into the admitted queue (first fit, arrival order).
void admit(spx_server* s) {
  for (auto it = s->waiting.begin(); it != s->waiting.end();) {
    Req& q = s->reqs[*it];
    if (s->st.bytes_in_use + q.bytes <= s->budget) {
      s->st.bytes_in_use += q.bytes;
      s->st.bytes_peak = std::max<uint64_t>(s->st.bytes_peak, s->st.bytes_in_use);
      q.state = ADMITTED;
      q.res.t_admit = s->now();
      s->admitted.push_back(*it);
      it = s->waiting.erase(it);
    } else {
      ++it;
    }
  }
}

struct Work {
  uint64_t ticket;
  spx_request r;
  int tile;
  spx_result res{};
  // device views
  const double* A = nullptr;
  const double* B = nullptr;
  double* X = nullptr;
  int64_t lda = 0, ldb = 0, ldx = 0;
  void* own[3] = {nullptr, nullptr, nullptr};
};

int hip_status(hipError_t e) { return e == hipSuccess ? SPX_OK : SPX_EDEVICE; }

// Runs one batch (all of one mode) on a lane.
void run_batch(spx_server* s, Lane& ln, int lane_id, std::vector<Work>& w) {
  spx_ctx* c = ln.ctx;
  hipStream_t st = ln.stream;
  const int K = (int)w.size();
  const double t_start = s->now();
  for (auto& x : w) {
    x.res.t_start = t_start;
    x.res.batch_size = K;
    x.res.lane = lane_id;
    x.res.tile = x.tile;
    x.res.status = SPX_OK;
  }
  // inputs on the device
  int rc = SPX_OK;
  for (auto& x : w) {
    const size_t n = (size_t)x.r.n, q = (size_t)x.r.nrhs;
    if (x.r.where == 1) {
      x.A = x.r.A;
      x.B = x.r.B;
      x.X = x.r.X;
      x.lda = x.r.lda;
      x.ldb = x.r.ldb;
      x.ldx = x.r.ldx;
      continue;
    }
    if (x.r.where == 2) {  // inputs on the device, X to host memory through a device copy
      x.A = x.r.A;
      x.B = x.r.B;
      x.lda = x.r.lda;
      x.ldb = x.r.ldb;
      x.own[2] = pool_alloc(n * q * 8, st, nullptr);
      if (!x.own[2]) {
        rc = SPX_ENOMEM;
        break;
      }
      x.X = (double*)x.own[2];
      x.ldx = (int64_t)q;
      continue;
    }
    x.own[0] = pool_alloc(n * n * 8, st, nullptr);
    x.own[1] = pool_alloc(n * q * 8, st, nullptr);
    x.own[2] = pool_alloc(n * q * 8, st, nullptr);
    if (!x.own[0] || !x.own[1] || !x.own[2]) {
      rc = SPX_ENOMEM;
      break;
    }
    x.A = (const double*)x.own[0];
    x.B = (const double*)x.own[1];
    x.X = (double*)x.own[2];
    x.lda = (int64_t)n;
    x.ldb = x.ldx = (int64_t)q;
    rc = hip_status(hipMemcpy2DAsync(x.own[0], n * 8, x.r.A, (size_t)x.r.lda * 8, n * 8, n, hipMemcpyHostToDevice, st));
    if (!rc)
      rc = hip_status(
          hipMemcpy2DAsync(x.own[1], q * 8, x.r.B, (size_t)x.r.ldb * 8, q * 8, n, hipMemcpyHostToDevice, st));
    if (rc) break;
  }
  std::vector<int64_t> n(K), lda(K), q(K), ldb(K), ldx(K), info(K, 0);
  std::vector<const double*> A(K), B(K);
  std::vector<double*> X(K);
  for (int i = 0; i < K; ++i) {
    n[i] = w[i].r.n;
    q[i] = w[i].r.nrhs;
    A[i] = w[i].A;
    B[i] = w[i].B;
    X[i] = w[i].X;
    lda[i] = w[i].lda;
    ldb[i] = w[i].ldb;
    ldx[i] = w[i].ldx;
  }
  spx_opts o{};
  o.num_wg = s->opts.num_wg;
  const bool mixed = w[0].r.mode == SPX_MODE_MIXED;
  // FP64 factor + solve of the systems in `sel`, then their backward errors
  auto fp64 = [&](const std::vector<int>& sel) -> int {
    if (sel.empty()) return SPX_OK;
    const int k = (int)sel.size();
    std::vector<int64_t> n2(k), lda2(k), q2(k), ldb2(k), ldx2(k), info2(k);
    std::vector<const double*> A2(k), B2(k);
    std::vector<double*> X2(k);
    for (int j = 0; j < k; ++j) {
      const int i = sel[j];
      n2[j] = n[i], lda2[j] = lda[i], q2[j] = q[i], ldb2[j] = ldb[i], ldx2[j] = ldx[i];
      A2[j] = A[i], B2[j] = B[i], X2[j] = X[i];
    }
    spx_opts o64 = o;
    o64.update_prec = SPX_PREC_FP64;
    int r = spx_posv_batched(c, k, n2.data(), A2.data(), lda2.data(), q2.data(), B2.data(), ldb2.data(), X2.data(),
                             ldx2.data(), &o64, info2.data(), nullptr);
    if (r) return r;
    std::vector<int> ok;
    for (int j = 0; j < k; ++j) {
      w[sel[j]].res.info = info2[j];
      w[sel[j]].res.method_used = 0;
      if (!info2[j]) ok.push_back(j);
    }
    if (ok.empty()) return SPX_OK;
    const int kk = (int)ok.size();
    std::vector<int64_t> n3(kk), lda3(kk), q3(kk), ldb3(kk), ldx3(kk);
    std::vector<const double*> A3(kk), B3(kk), X3(kk);
    std::vector<double> eta(kk);
    for (int t = 0; t < kk; ++t) {
      const int j = ok[t];
      n3[t] = n2[j], lda3[t] = lda2[j], q3[t] = q2[j], ldb3[t] = ldb2[j], ldx3[t] = ldx2[j];
      A3[t] = A2[j], B3[t] = B2[j], X3[t] = X2[j];
    }
    r = spx_backward_error_batched(c, kk, n3.data(), A3.data(), lda3.data(), q3.data(), X3.data(), ldx3.data(),
                                   B3.data(), ldb3.data(), eta.data());
    for (int t = 0; !r && t < kk; ++t) w[sel[ok[t]]].res.eta_max = eta[t];
    return r;
  };
  // per-request completion flags and watches: every request of an FP64 batch, and the
  // requests of a mixed batch that take the FP64 path directly (below mixed_min_n); the
  // others of a mixed batch are final only after the batched refinement
  const int64_t min_n = s->opts.mixed_min_n > 0 ? s->opts.mixed_min_n : kMixedMinN;
  std::vector<std::unique_ptr<Watch>> watch(K);
  std::vector<int> slots;  // slots[t]: the flag slot of request flagged[t]
  std::vector<int> flagged;
  std::vector<unsigned int*> dflags(K, nullptr);
  if (!rc && s->flags_h) {
    for (int i = 0; i < K; ++i)
      if (!mixed || n[i] < min_n) flagged.push_back(i);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (size_t t = 0; t < flagged.size() && !s->free_slots.empty(); ++t) {
        slots.push_back(s->free_slots.back());
        s->free_slots.pop_back();
      }
    }
    flagged.resize(slots.size());
    for (int t = 0; t < (int)slots.size(); ++t) {
      const int i = flagged[t];
      Watch* wt = new Watch();
      watch[i].reset(wt);
      wt->hflag = s->flags_h + slots[t];
      *wt->hflag = 0u;
      dflags[i] = s->flags_d + slots[t];
      const Work& x = w[i];
      if (x.r.where != 1) {
        wt->copy = hipEventCreateWithFlags(&wt->ev, hipEventDisableTiming) == hipSuccess;
        wt->dst = x.r.X;
        wt->dpitch = (size_t)x.r.ldx * 8;
        wt->src = x.X;
        wt->spitch = wt->width = (size_t)x.r.nrhs * 8;
        wt->height = (size_t)x.r.n;
        if (!wt->copy) dflags[i] = nullptr, watch[i].reset();  // no event: copied at the end
      }
    }
    std::atomic_thread_fence(std::memory_order_seq_cst);  // flags cleared before the launch
    std::lock_guard<std::mutex> lk(s->mon_mu);
    for (auto& wt : watch)
      if (wt) s->watches.push_back(wt.get());
  }
  if (!rc && !mixed) {
    std::vector<int> all(K);
    for (int i = 0; i < K; ++i) all[i] = i;
    ctx_set_store_flags(c, dflags.data());
    rc = fp64(all);
    ctx_set_store_flags(c, nullptr);
  } else if (!rc) {
    // Systems below opts.mixed_min_n go straight to FP64 (their updates are too small a
    // share of the work for FP32 to save what the refinement launches cost), first and
    // with their completion flags; then the FP32-update factor and first solve of the
    // others in one launch (factors kept), batched FP64 refinement from that solution,
    // and what does not converge redone in FP64.
    std::vector<int> low, direct, redo;
    for (int i = 0; i < K; ++i) (n[i] >= min_n ? low : direct).push_back(i);
    if (!direct.empty()) {
      std::vector<unsigned int*> fd(direct.size());
      for (size_t j = 0; j < direct.size(); ++j) fd[j] = dflags[direct[j]];
      ctx_set_store_flags(c, fd.data());
      rc = fp64(direct);
      ctx_set_store_flags(c, nullptr);
    }
    o.update_prec = SPX_PREC_FP32;
    const int KL = (int)low.size();
    std::vector<spx_factor*> f(K, nullptr);
    if (!rc && KL > 0) {
      std::vector<int64_t> nl(KL), ldal(KL), ql(KL), ldbl(KL), ldxl(KL), infol(KL);
      std::vector<const double*> Al(KL), Bl(KL);
      std::vector<double*> Xl(KL);
      std::vector<spx_factor*> fl(KL, nullptr);
      for (int j = 0; j < KL; ++j) {
        const int i = low[j];
        nl[j] = n[i], ldal[j] = lda[i], ql[j] = q[i], ldbl[j] = ldb[i], ldxl[j] = ldx[i];
        Al[j] = A[i], Bl[j] = B[i], Xl[j] = X[i];
      }
      rc = spx_posv_batched(c, KL, nl.data(), Al.data(), ldal.data(), ql.data(), Bl.data(), ldbl.data(), Xl.data(),
                            ldxl.data(), &o, infol.data(), fl.data());
      for (int j = 0; j < KL; ++j) f[low[j]] = fl[j];
    }
    std::vector<int> good;
    for (int i : low)
      if (!rc) (f[i] ? good : redo).push_back(i);
    if (!rc && !good.empty()) {
      const int k = (int)good.size();
      std::vector<spx_factor*> f2(k);
      std::vector<int64_t> lda2(k), q2(k), ldb2(k), ldx2(k);
      std::vector<const double*> A2(k), B2(k);
      std::vector<double*> X2(k);
      std::vector<spx_solve_stats> ss(k);
      for (int j = 0; j < k; ++j) {
        const int i = good[j];
        f2[j] = f[i], lda2[j] = lda[i], q2[j] = q[i], ldb2[j] = ldb[i], ldx2[j] = ldx[i];
        A2[j] = A[i], B2[j] = B[i], X2[j] = X[i];
      }
      const double tol = w[good[0]].r.tol > 0 ? w[good[0]].r.tol : 1e-12;
      spx_refine ref{tol, 50, 1, 1, 0};
      rc = spx_potrs_batched(c, k, f2.data(), q2.data(), B2.data(), ldb2.data(), X2.data(), ldx2.data(), A2.data(),
                             lda2.data(), &ref, ss.data());
      for (int j = 0; !rc && j < k; ++j) {
        Work& x = w[good[j]];
        const double tj = x.r.tol > 0 ? x.r.tol : 1e-12;
        x.res.info = 0;
        x.res.iters = ss[j].iters;
        x.res.eta_max = ss[j].eta_max;
        x.res.method_used = 1;
        if (!(ss[j].eta_max <= tj)) redo.push_back(good[j]);
      }
    }
    for (auto* g : f) spx_factor_destroy(g);
    if (!rc && !redo.empty()) {
      std::sort(redo.begin(), redo.end());
      rc = fp64(redo);
    }
  }
  // the launches are done (every STORE released): wait for the monitor to finish with
  // this batch's watches, so its copies are complete before the buffers are freed
  const int rc_k = hip_status(hipStreamSynchronize(st));
  if (!rc) rc = rc_k;
  for (auto& wt : watch) {
    if (!wt) continue;
    const auto tw = std::chrono::steady_clock::now();
    // (after a failed launch a flag may never rise)
    while (wt->state.load() != 2 && !(rc && wt->state.load() == 0) &&
           std::chrono::steady_clock::now() - tw < std::chrono::seconds(10))
      std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  bool copying = false;
  {
    std::lock_guard<std::mutex> lk(s->mon_mu);
    for (auto& wt : watch)
      if (wt) {
        s->watches.erase(std::find(s->watches.begin(), s->watches.end(), wt.get()));
        copying |= wt->state.load() == 1;
      }
  }
  if (copying) (void)hipStreamSynchronize(s->mon_stream);  // a copy still in flight
  // results back to the caller (those the monitor has not copied)
  for (int i = 0; i < K; ++i) {
    Work& x = w[i];
    if (watch[i] && watch[i]->state.load() == 2) x.res.t_ready = watch[i]->t_ready;
    const bool copied = watch[i] && watch[i]->copy && watch[i]->state.load() == 2;
    if (rc || x.r.where == 1 || x.res.info || copied) continue;
    const size_t nn = (size_t)x.r.n, qq = (size_t)x.r.nrhs;
    rc = hip_status(hipMemcpy2DAsync(x.r.X, (size_t)x.r.ldx * 8, x.X, qq * 8, qq * 8, nn, hipMemcpyDeviceToHost, st));
    if (rc) break;
  }
  const int rc_sync = hip_status(hipStreamSynchronize(st));
  if (!rc) rc = rc_sync;
  for (auto& wt : watch)
    if (wt && wt->ev) (void)hipEventDestroy(wt->ev);
  if (!slots.empty()) {
    std::lock_guard<std::mutex> lk(s->mu);
    for (int sl : slots) s->free_slots.push_back(sl);
  }
  for (auto& x : w)
    for (void* p : x.own)
      if (p) pool_free(p, st, nullptr);
  const double t_done = s->now();
  if (rc) std::fprintf(stderr, "spx server: lane %d: a batch of %d requests failed (%d): %s\n", lane_id, K, rc,
                       spx_last_error());
  for (auto& x : w) {
    if (rc) x.res.status = rc;
    x.res.t_done = t_done;
    if (!(x.res.t_ready > 0.0) || x.res.status != SPX_OK) x.res.t_ready = t_done;
  }
}

// Watches the completion flags of the running FP64 batches (every 20 us): a risen flag
// marks the request's X final in device memory; for host memory its copy back is issued
// on the monitor's stream and the request is ready when that copy completes.
void monitor_main(spx_server* s) {
  (void)hipSetDevice(s->device);
  while (!s->mon_stop.load()) {
    {
      std::lock_guard<std::mutex> lk(s->mon_mu);
      for (Watch* w : s->watches) {
        const int st = w->state.load();
        if (st == 0 && *w->hflag != 0u) {
          if (w->copy) {
            const bool ok = hipMemcpy2DAsync(w->dst, w->dpitch, w->src, w->spitch, w->width, w->height,
                                             hipMemcpyDeviceToHost, s->mon_stream) == hipSuccess &&
                            hipEventRecord(w->ev, s->mon_stream) == hipSuccess;
            if (ok) {
              w->state.store(1);
            } else {  // leave the copy to the lane
              w->copy = false;
              w->t_ready = s->now();
              w->state.store(2);
            }
          } else {
            w->t_ready = s->now();
            w->state.store(2);
          }
        } else if (st == 1 && hipEventQuery(w->ev) == hipSuccess) {
          w->t_ready = s->now();
          w->state.store(2);
        }
      }
    }
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

// Runs a batch; if device memory runs out (the budget counts the requests' own arrays, not
// the graph image or what other users of the device hold), runs each half on its own.
void run_batch_split(spx_server* s, Lane& ln, int lane_id, std::vector<Work>& w) {
  run_batch(s, ln, lane_id, w);
  const bool oom = std::all_of(w.begin(), w.end(), [](const Work& x) { return x.res.status == SPX_ENOMEM; });
  if (!oom || w.size() < 2) return;
  std::vector<Work> a(w.begin(), w.begin() + w.size() / 2), b(w.begin() + w.size() / 2, w.end());
  for (auto* part : {&a, &b})
    for (auto& x : *part) {
      x.A = x.B = nullptr;
      x.X = nullptr;
      x.own[0] = x.own[1] = x.own[2] = nullptr;
      x.res.status = SPX_OK;
    }
  run_batch_split(s, ln, lane_id, a);
  run_batch_split(s, ln, lane_id, b);
  std::copy(a.begin(), a.end(), w.begin());
  std::copy(b.begin(), b.end(), w.begin() + a.size());
}

void lane_main(spx_server* s, int id) {
  Lane& ln = s->lanes[id];
  (void)hipSetDevice(s->device);
  for (;;) {
    std::vector<Work> w;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || !s->admitted.empty(); });
      if (s->admitted.empty()) return;  // stopping and nothing admitted
      const spx_request& head = s->reqs[s->admitted.front()].r;
      const int mode = head.mode;
      const double tol = head.tol;
      // a batch holds at most the budget's share of one lane (its workspace is one block)
      const size_t cap = s->budget / s->lanes.size();
      size_t taken = 0;
      for (auto it = s->admitted.begin(); it != s->admitted.end() && (int)w.size() < s->opts.max_batch;) {
        Req& q = s->reqs[*it];
        if (q.r.mode != mode || (mode == SPX_MODE_MIXED && q.r.tol != tol) || (!w.empty() && taken + q.bytes > cap)) {
          ++it;
          continue;
        }
        taken += q.bytes;
        q.state = RUNNING;
        Work x;
        x.ticket = *it;
        x.r = q.r;
        x.tile = q.tile;
        x.res = q.res;
        w.push_back(x);
        it = s->admitted.erase(it);
      }
      s->running += w.size();
      s->st.max_running = std::max<uint64_t>(s->st.max_running, s->running);
      s->st.launches++;
    }
    const double t0 = s->now();
    run_batch_split(s, ln, id, w);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.busy_s += s->now() - t0;
      s->running -= w.size();
      for (auto& x : w) {
        Req& q = s->reqs[x.ticket];
        q.res = x.res;
        q.state = DONE;
        s->st.bytes_in_use -= q.bytes;
        s->st.completed++;
      }
      admit(s);
    }
    s->cv.notify_all();
  }
}

}  // namespace
}  // namespace spx

extern "C" {

int spx_server_create(spx_ctx* ctx, size_t hbm_budget_bytes, const spx_server_opts* opts, spx_server** out) {
  if (!ctx || !out || hbm_budget_bytes == 0) return fail(SPX_EINVAL, "spx_server_create: bad argument");
  *out = nullptr;
  std::unique_ptr<spx_server> s(new spx_server());
  s->device = ctx_device(ctx);
  s->budget = hbm_budget_bytes;
  if (opts) s->opts = *opts;
  if (s->opts.lanes <= 0) s->opts.lanes = 2;
  if (s->opts.lanes > 8) return fail(SPX_EINVAL, "spx_server_create: at most 8 lanes");
  if (s->opts.max_batch <= 0) s->opts.max_batch = 4096;
  s->t0 = std::chrono::steady_clock::now();
  if (hipSetDevice(s->device) != hipSuccess) return fail(SPX_EDEVICE, "spx_server_create: hipSetDevice failed");
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess) {
    uint64_t keep = UINT64_MAX;  // keep freed blocks for reuse instead of returning them
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    uint64_t zero = 0;  // the high-water mark reported by spx_server_get_stats starts here
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrUsedMemHigh, &zero);
  }
  s->lanes.resize(s->opts.lanes);
  for (auto& ln : s->lanes) {
    int rc = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) == hipSuccess ? SPX_OK : SPX_EDEVICE;
    if (!rc) rc = spx_ctx_create(s->device, ln.stream, pool_alloc, pool_free, nullptr, &ln.ctx);
    if (!rc) rc = ctx_copy_tile_tables(ctx, ln.ctx);
    if (rc) {
      for (auto& l2 : s->lanes) {
        if (l2.ctx) spx_ctx_destroy(l2.ctx);
        if (l2.stream) (void)hipStreamDestroy(l2.stream);
      }
      return rc == SPX_EDEVICE ? fail(SPX_EDEVICE, "spx_server_create: lane set-up failed") : rc;
    }
  }
  s->tuner = s->lanes[0].ctx;
  // completion flags: pinned, coherent host memory the kernel writes at system scope
  // (without them, every request of a batch gets the batch's end as t_ready)
  void* fh = nullptr;
  if (hipHostMalloc(&fh, sizeof(unsigned int) * kFlagSlots, hipHostMallocMapped | hipHostMallocCoherent) ==
      hipSuccess) {
    void* fd = nullptr;
    if (hipHostGetDevicePointer(&fd, fh, 0) == hipSuccess &&
        hipStreamCreateWithFlags(&s->mon_stream, hipStreamNonBlocking) == hipSuccess) {
      s->flags_h = (unsigned int*)fh;
      s->flags_d = (unsigned int*)fd;
      s->free_slots.reserve(kFlagSlots);
      for (int i = kFlagSlots - 1; i >= 0; --i) s->free_slots.push_back(i);
    } else {
      (void)hipHostFree(fh);
    }
  }
  spx_server* raw = s.release();
  if (raw->flags_h) raw->monitor = std::thread(monitor_main, raw);
  for (int i = 0; i < (int)raw->lanes.size(); ++i) raw->lanes[i].th = std::thread(lane_main, raw, i);
  *out = raw;
  return SPX_OK;
}

int spx_submit(spx_server* s, const spx_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return fail(SPX_EINVAL, "spx_submit: null argument");
  if (r->n < 1 || r->n > 65536 || r->nrhs < 1 || r->nrhs > 4096 || !r->A || !r->B || !r->X || r->lda < r->n ||
      r->ldb < r->nrhs || r->ldx < r->nrhs || (r->mode != SPX_MODE_FP64 && r->mode != SPX_MODE_MIXED) ||
      r->where < 0 || r->where > 2 || (const double*)r->X == r->B)
    return fail(SPX_EINVAL, "spx_submit: bad request");
  int32_t b = 0;
  const int rc = spx_tile_for(s->tuner, r->mode == SPX_MODE_MIXED ? SPX_PREC_FP32 : SPX_PREC_FP64, r->n, &b);
  if (rc) return rc;
  const size_t bytes = request_bytes(*r, b);
  if (bytes > s->budget) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected++;
    return failf(SPX_ENOMEM, "spx_submit: request needs %zu bytes, budget is %zu", bytes, s->budget);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(SPX_EABORT, "spx_submit: server is shutting down");
    const uint64_t t = s->next_ticket++;
    Req& q = s->reqs[t];
    q.r = *r;
    q.bytes = bytes;
    q.tile = b;
    q.res.tag = r->tag;
    q.res.t_submit = s->now();
    s->waiting.push_back(t);
    s->st.submitted++;
    *ticket = t;
    admit(s);
  }
  s->cv.notify_all();
  return SPX_OK;
}

int spx_poll(spx_server* s, uint64_t ticket, spx_result* out) {
  if (!s || !out) return fail(SPX_EINVAL, "spx_poll: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(SPX_EINVAL, "spx_poll: unknown ticket");
  if (it->second.state != DONE) return SPX_EAGAIN;
  *out = it->second.res;
  s->reqs.erase(it);
  return SPX_OK;
}

double spx_server_now(const spx_server* s) { return s ? s->now() : -1.0; }

int spx_server_get_stats(spx_server* s, spx_server_stats* out) {
  if (!s || !out) return fail(SPX_EINVAL, "spx_server_get_stats: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  hipMemPool_t pool;
  uint64_t high = 0;
  if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess &&
      hipMemPoolGetAttribute(pool, hipMemPoolAttrUsedMemHigh, &high) == hipSuccess)
    out->pool_used_high = high;
  return SPX_OK;
}

void spx_server_destroy(spx_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    const double t = s->now();
    for (uint64_t id : s->waiting) {
      Req& q = s->reqs[id];
      q.state = DONE;
      q.res.status = SPX_EABORT;
      q.res.t_done = t;
    }
    for (uint64_t id : s->admitted) {
      Req& q = s->reqs[id];
      q.state = DONE;
      q.res.status = SPX_EABORT;
      q.res.t_done = t;
    }
    s->waiting.clear();
    s->admitted.clear();
  }
  s->cv.notify_all();
  for (auto& ln : s->lanes)
    if (ln.th.joinable()) ln.th.join();
  s->mon_stop.store(true);
  if (s->monitor.joinable()) s->monitor.join();
  for (auto& ln : s->lanes) {
    spx_ctx_destroy(ln.ctx);
    (void)hipStreamSynchronize(ln.stream);
    (void)hipStreamDestroy(ln.stream);
  }
  if (s->mon_stream) {
    (void)hipStreamSynchronize(s->mon_stream);
    (void)hipStreamDestroy(s->mon_stream);
  }
  if (s->flags_h) (void)hipHostFree(s->flags_h);
  delete s;
}

}  // extern "C"
