// Host runtime of libspx: contexts, device images of task graphs, the factor and solve
// entry points of the C ABI, and run statistics.
//
// A task graph runs as one persistent-kernel launch (Specx Sec. 4.5 push/pop scheduler,
// realised on the GPU).  The static part of a graph's device image (task descriptors,
// CSR successors, in-degrees, part counts, the initial ready queue holding the roots) is
// built once per shape and cached on the context; before each launch a small kernel
// copies it into the per-launch counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "spx_internal.h"

namespace spx {

static thread_local std::string g_err;

int fail(int code, const char* msg) {
  g_err = msg;
  return code;
}

int failf(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

static int hipc(hipError_t e, const char* what) {
  if (e == hipSuccess) return SPX_OK;
  return failf(SPX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SPX_TRY(x)              \
  do {                          \
    int rc_ = (x);              \
    if (rc_ != SPX_OK) return rc_; \
  } while (0)

typedef unsigned long long u64;

// Static + per-launch device image of one task graph.
struct Image {
  uint32_t ntasks = 0, total_parts = 0;
  int nlev = 1;
  uint32_t qbase[kMaxLevels] = {0, 0, 0, 0};
  void* block = nullptr;  // one allocation for every array below
  size_t bytes = 0;
  TaskDesc* tasks = nullptr;
  uint32_t* succ_off = nullptr;
  uint32_t* succ = nullptr;
  uint32_t* indeg = nullptr;
  uint32_t* nparts = nullptr;
  u64* queue0 = nullptr;
  uint32_t* counters0 = nullptr;
  uint32_t* pending = nullptr;
  uint32_t* parts_left = nullptr;
  u64* queue = nullptr;
  uint32_t* counters = nullptr;
};

constexpr uint32_t kNumCounters = (2 * kMaxLevels + 2) * kCounterStride;

}  // namespace spx

using namespace spx;

struct spx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  spx_alloc_fn alloc = nullptr;
  spx_free_fn freef = nullptr;
  void* user = nullptr;
  int num_cu = 0, wg_per_cu = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  spx_stats last{};
  std::map<std::string, Image*> images;
  // small per-launch buffers
  DevMat* dmats = nullptr;
  size_t dmats_cap = 0;
  DevMat* hmats = nullptr;  // pinned staging of the matrix descriptors
  int32_t* dinfo = nullptr;
  int32_t* hinfo = nullptr;  // pinned
  size_t info_cap = 0;
  uint32_t* hcounters = nullptr;  // pinned copy of the counters after a launch
  u64* wg_cycles = nullptr;
  size_t wg_cap = 0;
  u64* trace = nullptr;
  uint32_t* trace_idx = nullptr;
  size_t trace_cap = 0;  // parts
  int64_t trace_len = 0;
  std::vector<u64> host_cycles;
  TaskDesc* dtask = nullptr;  // descriptor of single-task launches
};

struct spx_factor {
  spx_ctx* ctx = nullptr;
  int64_t n = 0, n_pad = 0;
  int32_t b = 0, nt = 0, prec = 0;
  double* tiles = nullptr;
  size_t tile_bytes = 0;
  void* low = nullptr;  // FP32 / BF16 copies of the panel tiles (mixed precision)
  double* dinv = nullptr;  // inverses of the 32x32 diagonal blocks of the diagonal tiles
};

namespace spx {

static void* dev_alloc(spx_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (c->alloc) return c->alloc(bytes, (void*)c->stream, c->user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

static void dev_free(spx_ctx* c, void* p) {
  if (!p) return;
  if (c->freef)
    c->freef(p, (void*)c->stream, c->user);
  else
    (void)hipFree(p);
}

static int valid_tile(int b) { return b == 32 || b == 64 || b == 128 || b == 256 || b == 512; }

static int default_tile(int64_t n) {
  if (n >= 8192) return 512;
  if (n >= 2048) return 256;
  if (n >= 512) return 128;
  if (n >= 128) return 64;
  return 32;
}

// Parts per task for tile size b and right-hand-side count nrhs.
int trsm_rows_of(int b) { return b < 64 ? b : 64; }

uint16_t parts_of(const TaskDesc& d, int b, int nrhs) {
  const int sb = b < 128 ? b : 128, ns = b / sb;
  const int rows = b < 64 ? b : 64;
  switch (d.type) {
    case SPX_T_POTRF: return 1;
    case SPX_T_TRSM: return (uint16_t)(b / trsm_rows_of(b));
    case SPX_T_SYRK: return (uint16_t)(ns * (ns + 1) / 2);
    case SPX_T_GEMM: return (uint16_t)(ns * ns);
    case SPX_T_FTRSM:
    case SPX_T_BTRSM: return (uint16_t)((nrhs + 7) / 8);
    case SPX_T_FGEMM:
    case SPX_T_BGEMM: return (uint16_t)(b / rows);
  }
  return 1;
}

static int level_of(int32_t prio, int policy) {
  if (policy == SPX_Q_FIFO) return 0;
  const int base = prio >> 16;
  int l = 3 - base;
  return l < 0 ? 0 : (l > kMaxLevels - 1 ? kMaxLevels - 1 : l);
}

// Builds (or returns the cached) device image of the factor (solve == false) or solve
// program for nt x nt tiles of size b.
static int get_image(spx_ctx* c, bool solve, int nt, int b, int nrhs, int policy, Image** out) {
  char key[96];
  const int rhs_parts = (nrhs + 7) / 8;
  std::snprintf(key, sizeof key, "%c:%d:%d:%d:%d", solve ? 'S' : 'F', nt, b, solve ? rhs_parts : 0, policy);
  auto it = c->images.find(key);
  if (it != c->images.end()) {
    *out = it->second;
    return SPX_OK;
  }
  std::vector<TaskDesc> tasks;
  std::vector<spx_access> acc;
  if (solve)
    solve_program(nt, tasks, acc);
  else
    cholesky_program(nt, false, tasks, acc);
  std::vector<int32_t> prio(tasks.size());
  for (size_t t = 0; t < tasks.size(); ++t) prio[t] = cholesky_priority(tasks[t], nt);
  Graph g;
  SPX_TRY(build_graph((uint32_t)tasks.size(), acc.data(), acc.size(), prio.data(), g));
  const uint32_t T = g.ntasks;
  std::unique_ptr<Image> im(new Image());
  im->ntasks = T;
  im->nlev = policy == SPX_Q_FIFO ? 1 : kMaxLevels;
  std::vector<uint32_t> nparts(T);
  uint32_t per_level[kMaxLevels] = {0, 0, 0, 0};
  for (uint32_t t = 0; t < T; ++t) {
    tasks[t].nparts = parts_of(tasks[t], b, nrhs);
    tasks[t].level = (uint8_t)level_of(prio[t], policy);
    tasks[t].mat = 0;
    nparts[t] = tasks[t].nparts;
    per_level[tasks[t].level] += nparts[t];
    im->total_parts += nparts[t];
  }
  for (int l = 1; l < kMaxLevels; ++l) im->qbase[l] = im->qbase[l - 1] + per_level[l - 1];
  std::vector<u64> queue0(im->total_parts, ~0ull);
  std::vector<uint32_t> counters0(kNumCounters, 0);
  for (uint32_t t = 0; t < T; ++t) {
    if (g.indeg[t] != 0) continue;
    const int l = tasks[t].level;
    uint32_t& tail = counters0[(kMaxLevels + l) * kCounterStride];
    for (uint32_t p = 0; p < nparts[t]; ++p) queue0[im->qbase[l] + tail + p] = ((u64)t << 16) | p;
    tail += nparts[t];
  }
  std::vector<uint32_t> off32(T + 1);
  for (uint32_t t = 0; t <= T; ++t) off32[t] = (uint32_t)g.off[t];
  // layout
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t o = 0;
  const size_t o_tasks = o; o = align(o + sizeof(TaskDesc) * T);
  const size_t o_off = o; o = align(o + 4 * (size_t)(T + 1));
  const size_t o_succ = o; o = align(o + 4 * (size_t)std::max<size_t>(g.succ.size(), 1));
  const size_t o_indeg = o; o = align(o + 4 * (size_t)T);
  const size_t o_np = o; o = align(o + 4 * (size_t)T);
  const size_t o_q0 = o; o = align(o + 8 * (size_t)im->total_parts);
  const size_t o_c0 = o; o = align(o + 4 * (size_t)kNumCounters);
  const size_t static_bytes = o;
  const size_t o_pend = o; o = align(o + 4 * (size_t)T);
  const size_t o_pl = o; o = align(o + 4 * (size_t)T);
  const size_t o_q = o; o = align(o + 8 * (size_t)im->total_parts);
  const size_t o_c = o; o = align(o + 4 * (size_t)kNumCounters);
  im->bytes = o;
  im->block = dev_alloc(c, o);
  if (!im->block) return fail(SPX_ENOMEM, "device image: allocation failed");
  char* base = (char*)im->block;
  im->tasks = (TaskDesc*)(base + o_tasks);
  im->succ_off = (uint32_t*)(base + o_off);
  im->succ = (uint32_t*)(base + o_succ);
  im->indeg = (uint32_t*)(base + o_indeg);
  im->nparts = (uint32_t*)(base + o_np);
  im->queue0 = (u64*)(base + o_q0);
  im->counters0 = (uint32_t*)(base + o_c0);
  im->pending = (uint32_t*)(base + o_pend);
  im->parts_left = (uint32_t*)(base + o_pl);
  im->queue = (u64*)(base + o_q);
  im->counters = (uint32_t*)(base + o_c);
  std::vector<char> host(static_bytes, 0);
  std::memcpy(host.data() + o_tasks, tasks.data(), sizeof(TaskDesc) * T);
  std::memcpy(host.data() + o_off, off32.data(), 4 * (size_t)(T + 1));
  if (!g.succ.empty()) std::memcpy(host.data() + o_succ, g.succ.data(), 4 * g.succ.size());
  std::memcpy(host.data() + o_indeg, g.indeg.data(), 4 * (size_t)T);
  std::memcpy(host.data() + o_np, nparts.data(), 4 * (size_t)T);
  std::memcpy(host.data() + o_q0, queue0.data(), 8 * (size_t)im->total_parts);
  std::memcpy(host.data() + o_c0, counters0.data(), 4 * (size_t)kNumCounters);
  // synchronous copy: the host vector is freed on return
  int rc = hipc(hipMemcpy(im->block, host.data(), static_bytes, hipMemcpyHostToDevice), "image upload");
  if (rc) {
    dev_free(c, im->block);
    return rc;
  }
  *out = im.get();
  c->images[key] = im.release();
  return SPX_OK;
}

static int ensure_small_buffers(spx_ctx* c, size_t nmats, size_t num_wg, size_t parts, bool trace) {
  if (nmats > c->dmats_cap) {
    dev_free(c, c->dmats);
    dev_free(c, c->dinfo);
    if (c->hmats) (void)hipHostFree(c->hmats);
    if (c->hinfo) (void)hipHostFree(c->hinfo);
    c->dmats = nullptr;
    c->dinfo = nullptr;
    c->hmats = nullptr;
    c->hinfo = nullptr;
    c->dmats_cap = 0;
    const size_t cap = std::max<size_t>(nmats, 16);
    c->dmats = (DevMat*)dev_alloc(c, sizeof(DevMat) * cap);
    c->dinfo = (int32_t*)dev_alloc(c, 4 * cap);
    if (!c->dmats || !c->dinfo) return fail(SPX_ENOMEM, "context buffers: allocation failed");
    SPX_TRY(hipc(hipHostMalloc((void**)&c->hmats, sizeof(DevMat) * cap, 0), "hipHostMalloc"));
    SPX_TRY(hipc(hipHostMalloc((void**)&c->hinfo, 4 * cap, 0), "hipHostMalloc"));
    c->dmats_cap = cap;
  }
  if (!c->hcounters) SPX_TRY(hipc(hipHostMalloc((void**)&c->hcounters, 4 * kNumCounters, 0), "hipHostMalloc"));
  if (num_wg > c->wg_cap) {
    dev_free(c, c->wg_cycles);
    c->wg_cycles = (u64*)dev_alloc(c, 16 * num_wg);
    if (!c->wg_cycles) return fail(SPX_ENOMEM, "context buffers: allocation failed");
    c->wg_cap = num_wg;
  }
  if (trace && parts > c->trace_cap) {
    dev_free(c, c->trace);
    dev_free(c, c->trace_idx);
    c->trace = (u64*)dev_alloc(c, 32 * parts);
    c->trace_idx = (uint32_t*)dev_alloc(c, 256);
    if (!c->trace || !c->trace_idx) return fail(SPX_ENOMEM, "trace buffer: allocation failed");
    c->trace_cap = parts;
  }
  return SPX_OK;
}

// Runs one image over `nmats` matrices (descriptors in c->hmats) and waits for it.
// On return c->hinfo[0..nmats) holds each matrix's info word.
static int run_image(spx_ctx* c, Image* im, int nmats, const spx_opts* o, double pack_ms) {
  const bool trace = o && (o->flags & SPX_F_TRACE);
  int num_wg = (o && o->num_wg > 0) ? o->num_wg : c->num_cu * c->wg_per_cu;
  if (num_wg < 1) num_wg = 1;
  SPX_TRY(ensure_small_buffers(c, nmats, num_wg, im->total_parts, trace));
  SPX_TRY(hipc(hipMemcpyAsync(c->dmats, c->hmats, sizeof(DevMat) * nmats, hipMemcpyHostToDevice, c->stream),
               "descriptor upload"));
  SPX_TRY(launch_sched_init_full(im->pending, im->indeg, im->parts_left, im->nparts, im->ntasks, im->queue,
                                 im->queue0, im->total_parts, im->counters, im->counters0, kNumCounters, c->dinfo,
                                 nmats, trace ? c->trace_idx : nullptr, c->stream));
  SchedArgs a{};
  a.tasks = im->tasks;
  a.succ_off = im->succ_off;
  a.succ = im->succ;
  a.pending = im->pending;
  a.parts_left = im->parts_left;
  a.queue = im->queue;
  a.counters = im->counters;
  for (int l = 0; l < kMaxLevels; ++l) a.qbase[l] = im->qbase[l];
  a.total_parts = im->total_parts;
  a.ntasks = im->ntasks;
  a.nlev = im->nlev;
  a.mats = c->dmats;
  a.trace = trace ? c->trace : nullptr;
  a.trace_idx = trace ? c->trace_idx : nullptr;
  a.wg_cycles = c->wg_cycles;
  a.spin_limit = 100000000ull * 20;  // 20 s of the 100 MHz device clock without progress
  SPX_TRY(hipc(hipEventRecord(c->ev[0], c->stream), "hipEventRecord"));
  SPX_TRY(launch_sched(a, num_wg, c->stream));
  SPX_TRY(hipc(hipEventRecord(c->ev[1], c->stream), "hipEventRecord"));
  SPX_TRY(hipc(hipMemcpyAsync(c->hinfo, c->dinfo, 4 * (size_t)nmats, hipMemcpyDeviceToHost, c->stream), "info"));
  SPX_TRY(hipc(hipMemcpyAsync(c->hcounters, im->counters, 4 * kNumCounters, hipMemcpyDeviceToHost, c->stream),
               "counters"));
  c->host_cycles.resize(2 * (size_t)num_wg);
  SPX_TRY(hipc(hipMemcpyAsync(c->host_cycles.data(), c->wg_cycles, 16 * (size_t)num_wg, hipMemcpyDeviceToHost,
                              c->stream),
               "cycles"));
  SPX_TRY(hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
  float ms = 0.f;
  SPX_TRY(hipc(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]), "hipEventElapsedTime"));
  double busy = 0, idle = 0;
  for (int w = 0; w < num_wg; ++w) {
    busy += (double)c->host_cycles[2 * w];
    idle += (double)c->host_cycles[2 * w + 1];
  }
  c->last.kernel_ms = ms;
  c->last.pack_ms = pack_ms;
  c->last.idle_frac = (busy + idle) > 0 ? idle / (busy + idle) : 0.0;
  c->last.ntasks = im->ntasks;
  c->last.nparts = im->total_parts;
  c->last.num_wg = (uint32_t)num_wg;
  c->trace_len = trace ? im->total_parts : 0;
  const uint32_t status = c->hcounters[(2 * kMaxLevels + 1) * kCounterStride];
  const uint32_t done = c->hcounters[2 * kMaxLevels * kCounterStride];
  if (status & STATUS_TIMEOUT)
    return failf(SPX_ETIMEOUT, "device scheduler made no progress (%u of %u parts done)", done, im->total_parts);
  if (done != im->total_parts)
    return failf(SPX_EDEVICE, "device scheduler ended early (%u of %u parts done)", done, im->total_parts);
  return SPX_OK;
}

}  // namespace spx

extern "C" {

const char* spx_last_error(void) { return g_err.c_str(); }

int spx_ctx_create(int device, void* hip_stream, spx_alloc_fn alloc, spx_free_fn free_fn, void* user, spx_ctx** out) {
  if (!out) return fail(SPX_EINVAL, "spx_ctx_create: null out");
  *out = nullptr;
  int count = 0;
  SPX_TRY(hipc(hipGetDeviceCount(&count), "hipGetDeviceCount"));
  if (device < 0 || device >= count) return fail(SPX_EINVAL, "spx_ctx_create: bad device");
  SPX_TRY(hipc(hipSetDevice(device), "hipSetDevice"));
  std::unique_ptr<spx_ctx> c(new spx_ctx());
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->alloc = alloc;
  c->freef = free_fn;
  c->user = user;
  SPX_TRY(sched_max_wg(device, &c->wg_per_cu, &c->num_cu));
  if (c->wg_per_cu > 2) c->wg_per_cu = 2;
  for (auto& e : c->ev) SPX_TRY(hipc(hipEventCreate(&e), "hipEventCreate"));
  *out = c.release();
  return SPX_OK;
}

void spx_ctx_destroy(spx_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->images) {
    dev_free(c, kv.second->block);
    delete kv.second;
  }
  dev_free(c, c->dmats);
  dev_free(c, c->dinfo);
  dev_free(c, c->wg_cycles);
  dev_free(c, c->trace);
  dev_free(c, c->trace_idx);
  dev_free(c, c->dtask);
  if (c->hmats) (void)hipHostFree(c->hmats);
  if (c->hinfo) (void)hipHostFree(c->hinfo);
  if (c->hcounters) (void)hipHostFree(c->hcounters);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

int spx_potrf_tiled(spx_ctx* c, int64_t n, const double* dA, int64_t lda, const spx_opts* opts, spx_factor** out,
                    int64_t* info) {
  if (!c || !dA || !out || !info) return fail(SPX_EINVAL, "spx_potrf_tiled: null argument");
  *out = nullptr;
  *info = 0;
  if (n < 1 || lda < n) return fail(SPX_EINVAL, "spx_potrf_tiled: need n >= 1 and lda >= n");
  const int b = (opts && opts->tile > 0) ? opts->tile : default_tile(n);
  if (!valid_tile(b)) return fail(SPX_EINVAL, "spx_potrf_tiled: tile must be 32, 64, 128, 256 or 512");
  const int policy = opts ? opts->queue_policy : SPX_Q_PRIORITY;
  if (policy != SPX_Q_PRIORITY && policy != SPX_Q_FIFO) return fail(SPX_EINVAL, "spx_potrf_tiled: bad queue policy");
  const int prec = opts ? opts->update_prec : SPX_PREC_FP64;
  if (prec != SPX_PREC_FP64 && prec != SPX_PREC_FP32 && prec != SPX_PREC_BF16)
    return fail(SPX_EINVAL, "spx_potrf_tiled: bad update precision");
  const int64_t nt = (n + b - 1) / b;
  if (nt > 2048) return fail(SPX_EINVAL, "spx_potrf_tiled: too many tiles");
  SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
  std::unique_ptr<spx_factor> f(new spx_factor());
  f->ctx = c;
  f->n = n;
  f->b = b;
  f->nt = (int32_t)nt;
  f->n_pad = nt * b;
  f->prec = prec;
  f->tile_bytes = (size_t)(nt * (nt + 1) / 2) * (size_t)b * (size_t)b * sizeof(double);
  f->tiles = (double*)dev_alloc(c, f->tile_bytes);
  if (!f->tiles) return fail(SPX_ENOMEM, "spx_potrf_tiled: tile storage allocation failed");
  f->dinv = (double*)dev_alloc(c, (size_t)f->n_pad * 32 * sizeof(double));
  if (!f->dinv) {
    dev_free(c, f->tiles);
    return fail(SPX_ENOMEM, "spx_potrf_tiled: block inverse allocation failed");
  }
  if (prec != SPX_PREC_FP64) {
    f->low = dev_alloc(c, f->tile_bytes / (prec == SPX_PREC_FP32 ? 2 : 4));
    if (!f->low) {
      dev_free(c, f->tiles);
      dev_free(c, f->dinv);
      return fail(SPX_ENOMEM, "spx_potrf_tiled: low-precision copy allocation failed");
    }
  }
  Image* im = nullptr;
  int rc = get_image(c, false, (int)nt, b, 0, policy, &im);
  if (!rc) rc = ensure_small_buffers(c, 1, 1, 0, false);
  if (rc) {
    dev_free(c, f->tiles);
    dev_free(c, f->low);
    dev_free(c, f->dinv);
    return rc;
  }
  DevMat m{};
  m.tiles = f->tiles;
  m.low = f->low;
  m.dinv = f->dinv;
  m.info = c->dinfo;
  m.n_pad = f->n_pad;
  m.nt = (int32_t)nt;
  m.b = b;
  m.prec = prec;
  m.n = (int32_t)n;
  m.trsm_rows = trsm_rows_of(b);
  c->hmats[0] = m;
  rc = hipc(hipEventRecord(c->ev[2], c->stream), "hipEventRecord");
  if (!rc) rc = launch_pack(dA, lda, n, m, c->stream);
  if (!rc) rc = hipc(hipEventRecord(c->ev[3], c->stream), "hipEventRecord");
  if (!rc) rc = run_image(c, im, 1, opts, 0.0);
  if (!rc) {
    float pms = 0.f;
    if (hipEventElapsedTime(&pms, c->ev[2], c->ev[3]) == hipSuccess) c->last.pack_ms = pms;
    c->last.tile = (uint32_t)b;
  }
  if (rc) {
    dev_free(c, f->tiles);
    dev_free(c, f->low);
    dev_free(c, f->dinv);
    return rc;
  }
  if (c->hinfo[0] != INT_MAX) {
    *info = c->hinfo[0];
    dev_free(c, f->tiles);
    dev_free(c, f->low);
    dev_free(c, f->dinv);
    return SPX_OK;
  }
  *out = f.release();
  return SPX_OK;
}

int spx_factor_info(const spx_factor* f, int64_t* n, int32_t* tile, int64_t* n_padded) {
  if (!f) return fail(SPX_EINVAL, "spx_factor_info: null factor");
  if (n) *n = f->n;
  if (tile) *tile = f->b;
  if (n_padded) *n_padded = f->n_pad;
  return SPX_OK;
}

int spx_factor_get_l(spx_ctx* c, const spx_factor* f, double* dL, int64_t ldl) {
  if (!c || !f || !dL || ldl < f->n) return fail(SPX_EINVAL, "spx_factor_get_l: bad argument");
  DevMat m{};
  m.tiles = f->tiles;
  m.nt = f->nt;
  m.b = f->b;
  m.n_pad = f->n_pad;
  SPX_TRY(launch_unpack(m, f->n, dL, ldl, c->stream));
  return hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

void spx_factor_destroy(spx_factor* f) {
  if (!f) return;
  (void)hipStreamSynchronize(f->ctx->stream);
  dev_free(f->ctx, f->tiles);
  dev_free(f->ctx, f->low);
  dev_free(f->ctx, f->dinv);
  delete f;
}

// Runs the solve graph of factor f on the column-major work buffer rhs (n_pad x nrhs).
static int solve_on(spx_ctx* c, const spx_factor* f, int64_t nrhs, double* rhs) {
  Image* im = nullptr;
  SPX_TRY(get_image(c, true, f->nt, f->b, (int)nrhs, SPX_Q_PRIORITY, &im));
  SPX_TRY(ensure_small_buffers(c, 1, 1, 0, false));
  DevMat m{};
  m.tiles = f->tiles;
  m.dinv = f->dinv;
  m.rhs = rhs;
  m.info = c->dinfo;
  m.n_pad = f->n_pad;
  m.nt = f->nt;
  m.b = f->b;
  m.nrhs = (int32_t)nrhs;
  m.prec = PREC_FP64;  // the solve always reads the FP64 factor
  m.n = (int32_t)f->n;
  m.trsm_rows = trsm_rows_of(f->b);
  c->hmats[0] = m;
  return run_image(c, im, 1, nullptr, 0.0);
}

// r = b - A x and the per-column maxima for the backward error; returns eta per column in
// eta (host) and the largest in *eta_max.
static int residual_eta(spx_ctx* c, int64_t n, const double* dA, int64_t lda, int64_t nrhs, const double* dX,
                        int64_t ldx, const double* dB, int64_t ldb, double* R, double* S, std::vector<double>& hs,
                        double* eta, double* eta_max) {
  const size_t sbytes = sizeof(double) * (size_t)(3 * nrhs + 1);
  SPX_TRY(hipc(hipMemsetAsync(S, 0, sbytes, c->stream), "hipMemsetAsync"));
  SPX_TRY(launch_backward_error(n, dA, lda, nrhs, dX, ldx, dB, ldb, R, S, c->stream));
  hs.resize(3 * nrhs + 1);
  SPX_TRY(hipc(hipMemcpyAsync(hs.data(), S, sbytes, hipMemcpyDeviceToHost, c->stream), "stats"));
  SPX_TRY(hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
  const double anorm = hs[3 * nrhs];
  double worst = 0.0;
  for (int64_t q = 0; q < nrhs; ++q) {
    const double e = hs[3 * q] / (anorm * hs[3 * q + 1] + hs[3 * q + 2]);
    if (eta) eta[q] = e;
    if (!(e <= worst)) worst = e;  // NaN propagates
  }
  *eta_max = worst;
  return SPX_OK;
}

int spx_potrs(spx_ctx* c, const spx_factor* f, int64_t nrhs, const double* dB, int64_t ldb, double* dX, int64_t ldx,
              const double* dA, int64_t lda, const spx_refine* refine, spx_solve_stats* stats) {
  if (!c || !f || !dB || !dX) return fail(SPX_EINVAL, "spx_potrs: null argument");
  if (nrhs < 1 || nrhs > 4096 || ldb < nrhs || ldx < nrhs) return fail(SPX_EINVAL, "spx_potrs: bad nrhs / ld");
  if (dX == dB && ldx != ldb) return fail(SPX_EINVAL, "spx_potrs: aliased X and B need equal leading dimensions");
  const int method = refine ? refine->method : 0;
  if (method < 0 || method > 1) return fail(SPX_EINVAL, "spx_potrs: refinement method must be 0 or 1");
  if (method && (!dA || lda < f->n)) return fail(SPX_EINVAL, "spx_potrs: refinement needs the original matrix");
  if (method && dX == dB) return fail(SPX_EINVAL, "spx_potrs: refinement needs X distinct from B");
  SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
  double* rhs = (double*)dev_alloc(c, (size_t)f->n_pad * (size_t)nrhs * sizeof(double));
  double* R = method ? (double*)dev_alloc(c, (size_t)f->n * (size_t)nrhs * sizeof(double)) : nullptr;
  double* S = method ? (double*)dev_alloc(c, sizeof(double) * (size_t)(3 * nrhs + 1)) : nullptr;
  int rc = (!rhs || (method && (!R || !S))) ? fail(SPX_ENOMEM, "spx_potrs: work buffer allocation failed") : SPX_OK;
  if (!rc) rc = launch_rhs_in(dB, ldb, f->n, nrhs, rhs, f->n_pad, c->stream);
  if (!rc) rc = solve_on(c, f, nrhs, rhs);
  if (!rc) rc = launch_rhs_out(rhs, f->n_pad, f->n, nrhs, dX, ldx, 0, c->stream);
  int iters = 0;
  double eta_max = -1.0;
  double solve_ms = c->last.kernel_ms;
  if (!rc && method == 1) {
    // classical iterative refinement: r = b - A x in FP64 with the original matrix,
    // d = solve(L, r), x += d, until the largest normwise backward error <= tol
    std::vector<double> hs;
    const double tol = refine->tol > 0 ? refine->tol : 1e-12;
    const int max_iter = refine->max_iter > 0 ? refine->max_iter : 50;
    double prev = INFINITY;
    int slow = 0;
    for (;;) {
      rc = residual_eta(c, f->n, dA, lda, nrhs, dX, ldx, dB, ldb, R, S, hs, nullptr, &eta_max);
      if (rc || eta_max <= tol || iters >= max_iter) break;
      if (!(eta_max < 0.5 * prev)) {  // stagnation (or NaN): stop after two slow steps
        if (++slow >= 2 || eta_max != eta_max) break;
      } else {
        slow = 0;
      }
      prev = eta_max;
      rc = launch_rhs_in(R, nrhs, f->n, nrhs, rhs, f->n_pad, c->stream);
      if (!rc) rc = solve_on(c, f, nrhs, rhs);
      if (!rc) rc = launch_rhs_out(rhs, f->n_pad, f->n, nrhs, dX, ldx, 1, c->stream);
      if (!rc) solve_ms += c->last.kernel_ms;
      if (rc) break;
      ++iters;
    }
  }
  if (!rc) rc = hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  dev_free(c, rhs);
  dev_free(c, R);
  dev_free(c, S);
  if (rc) return rc;
  c->last.kernel_ms = solve_ms;  // all solve launches of this call
  if (stats) {
    stats->iters = iters;
    stats->method_used = method;
    stats->eta_max = eta_max;
  }
  return SPX_OK;
}

int spx_backward_error(spx_ctx* c, int64_t n, const double* dA, int64_t lda, int64_t nrhs, const double* dX,
                       int64_t ldx, const double* dB, int64_t ldb, double* eta) {
  if (!c || !dA || !dX || !dB || !eta || n < 1 || lda < n || nrhs < 1 || ldx < nrhs || ldb < nrhs)
    return fail(SPX_EINVAL, "spx_backward_error: bad argument");
  SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
  const size_t sbytes = sizeof(double) * (size_t)(3 * nrhs + 1);
  double* R = (double*)dev_alloc(c, sizeof(double) * (size_t)(n * nrhs));
  double* S = (double*)dev_alloc(c, sbytes);
  int rc = (!R || !S) ? fail(SPX_ENOMEM, "spx_backward_error: allocation failed") : SPX_OK;
  if (!rc) rc = hipc(hipMemsetAsync(S, 0, sbytes, c->stream), "hipMemsetAsync");
  if (!rc) rc = launch_backward_error(n, dA, lda, nrhs, dX, ldx, dB, ldb, R, S, c->stream);
  std::vector<double> hs(3 * nrhs + 1);
  if (!rc) rc = hipc(hipMemcpyAsync(hs.data(), S, sbytes, hipMemcpyDeviceToHost, c->stream), "stats");
  if (!rc) rc = hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  dev_free(c, R);
  dev_free(c, S);
  if (rc) return rc;
  const double anorm = hs[3 * nrhs];
  for (int64_t q = 0; q < nrhs; ++q) eta[q] = hs[3 * q] / (anorm * hs[3 * q + 1] + hs[3 * q + 2]);
  return SPX_OK;
}

int spx_run_task(spx_ctx* c, int32_t type, int32_t i, int32_t j, int32_t k, int32_t nt, int32_t b, double* d_tiles,
                 double* d_rhs, int32_t nrhs, int64_t* info) {
  if (!c || !d_tiles || !info) return fail(SPX_EINVAL, "spx_run_task: null argument");
  if (!valid_tile(b) || nt < 1 || nt > 2048) return fail(SPX_EINVAL, "spx_run_task: bad tile size or count");
  if (type < SPX_T_POTRF || type > SPX_T_BGEMM) return fail(SPX_EINVAL, "spx_run_task: bad task type");
  const bool solve = type >= SPX_T_FTRSM;
  if (solve && (!d_rhs || nrhs < 1 || nrhs > 4096)) return fail(SPX_EINVAL, "spx_run_task: solve task needs rhs");
  auto in = [nt](int x) { return x >= 0 && x < nt; };
  bool ok = in(i) && in(j) && in(k);
  switch (type) {
    case SPX_T_POTRF: ok = ok && i == k && j == k; break;
    case SPX_T_TRSM: ok = ok && i > k && j == k; break;
    case SPX_T_SYRK: ok = ok && i > k && j == i; break;
    case SPX_T_GEMM: ok = ok && i > j && j > k; break;
    case SPX_T_FTRSM: case SPX_T_BTRSM: ok = ok && i == k && j == k; break;
    case SPX_T_FGEMM: ok = ok && i > k && j == k; break;
    case SPX_T_BGEMM: ok = ok && i < j && j == k; break;
  }
  if (!ok) return fail(SPX_EINVAL, "spx_run_task: tile indices do not fit the task type");
  SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
  SPX_TRY(ensure_small_buffers(c, 1, 1, 0, false));
  if (!c->dtask) {
    c->dtask = (TaskDesc*)dev_alloc(c, sizeof(TaskDesc));
    if (!c->dtask) return fail(SPX_ENOMEM, "spx_run_task: allocation failed");
  }
  TaskDesc d;
  d.type = (uint8_t)type;
  d.i = (uint16_t)i;
  d.j = (uint16_t)j;
  d.k = (uint16_t)k;
  d.nparts = parts_of(d, b, nrhs);
  // block inverses of the diagonal tile the task reads (written by a POTRF task itself)
  double* dinv = (double*)dev_alloc(c, (size_t)nt * 32 * b * sizeof(double));
  if (!dinv) return fail(SPX_ENOMEM, "spx_run_task: allocation failed");
  const bool reads_diag = type == SPX_T_TRSM || type == SPX_T_FTRSM || type == SPX_T_BTRSM;
  if (reads_diag) {
    const double* lkk = d_tiles + ((size_t)k * (k + 1) / 2 + k) * (size_t)b * b;
    int rc = launch_tile_inverses(lkk, b, dinv + (size_t)k * 32 * b, c->stream);
    if (rc) {
      dev_free(c, dinv);
      return rc;
    }
  }
  DevMat m{};
  m.tiles = d_tiles;
  m.dinv = dinv;
  m.rhs = d_rhs;
  m.info = c->dinfo;
  m.n_pad = (int64_t)nt * b;
  m.nt = nt;
  m.b = b;
  m.nrhs = nrhs;
  m.n = nt * b;
  m.trsm_rows = trsm_rows_of(b);
  c->hmats[0] = m;
  const int32_t healthy = INT_MAX;
  int rc = hipc(hipMemcpyAsync(c->dtask, &d, sizeof d, hipMemcpyHostToDevice, c->stream), "task upload");
  if (!rc) rc = hipc(hipMemcpyAsync(c->dmats, c->hmats, sizeof(DevMat), hipMemcpyHostToDevice, c->stream), "upload");
  if (!rc) rc = hipc(hipMemcpyAsync(c->dinfo, &healthy, 4, hipMemcpyHostToDevice, c->stream), "upload");
  SchedArgs a{};
  a.tasks = c->dtask;
  a.mats = c->dmats;
  if (!rc) rc = launch_one_task(a, d.nparts, c->stream);
  if (!rc) rc = hipc(hipMemcpyAsync(c->hinfo, c->dinfo, 4, hipMemcpyDeviceToHost, c->stream), "info");
  if (!rc) rc = hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  dev_free(c, dinv);
  if (rc) return rc;
  *info = c->hinfo[0] == INT_MAX ? 0 : c->hinfo[0];
  return SPX_OK;
}

int spx_last_stats(const spx_ctx* c, spx_stats* out) {
  if (!c || !out) return fail(SPX_EINVAL, "spx_last_stats: null argument");
  *out = c->last;
  return SPX_OK;
}

int64_t spx_trace(const spx_ctx* c, uint64_t* rec, int64_t cap) {
  if (!c) return fail(SPX_EINVAL, "spx_trace: null context");
  if (c->trace_len <= 0) return 0;
  const int64_t nrec = std::min<int64_t>(cap, c->trace_len);
  if (rec && nrec > 0) {
    if (hipMemcpy(rec, c->trace, 32 * (size_t)nrec, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(SPX_EDEVICE, "spx_trace: copy failed");
  }
  return c->trace_len;
}

}  // extern "C"
