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
#include <cstdlib>
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
  return failf(e == hipErrorOutOfMemory ? SPX_ENOMEM : SPX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
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
  int family = FAM_CHOL;  // the scheduler instantiation that runs its tasks
  uint32_t qbase[kLevelsMax] = {};
  uint32_t qcap[kLevelsMax] = {};
  uint32_t nroots = 0;
  int nshards = 1;
  uint32_t spread_max = 0;  // tasks of at most this many parts deal them over the shards
  void* block = nullptr;  // one allocation for every array below
  size_t bytes = 0;
  TaskDesc* tasks = nullptr;
  uint32_t* succ_off = nullptr;
  uint32_t* succ = nullptr;
  uint32_t* indeg = nullptr;
  uint32_t* nparts = nullptr;
  u64* roots = nullptr;  // (queue slot, item) pairs of the root tasks' parts
  uint32_t* counters0 = nullptr;
  uint32_t* pending = nullptr;
  uint32_t* parts_left = nullptr;
  u64* queue = nullptr;
  uint32_t* counters = nullptr;
  uint32_t* ring = nullptr;  // kXcds x total_parts finished-part entries
  // commutative-write groups (null / 0 without them): see Graph
  uint32_t ngroups = 0, ncroots = 0;
  uint32_t *coff = nullptr, *cent = nullptr, *goff = nullptr, *gtask = nullptr, *gidx = nullptr, *croots = nullptr;
  u64* gstate = nullptr;  // per group: lock bit 63, waiting members' bits 0..62
};


// Task program of one matrix with its dependency graph (built once per shape).
struct Program {
  std::vector<TaskDesc> tasks;
  Graph g;
};

struct ImageHost;

}  // namespace spx

using namespace spx;

struct spx_ctx {
  int device = 0;
  // per-matrix completion flags for the next batched solve (the serving loop sets them)
  unsigned int* const* store_flags = nullptr;
  hipStream_t stream = nullptr;
  spx_alloc_fn alloc = nullptr;
  spx_free_fn freef = nullptr;
  void* user = nullptr;
  int num_cu = 0, wg_per_cu = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  spx_stats last{};
  std::map<std::string, Image*> images;
  std::map<std::string, std::unique_ptr<Program>> programs;
  // images of batched launches: few, large, keyed by the whole shape list (oldest evicted)
  std::vector<std::pair<std::string, Image*>> batch_images;
  // tile table per update precision: (n_max, tile), n_max increasing
  std::vector<std::pair<int64_t, int>> tile_table[3];
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
  int64_t trace_tasks = 0;  // push ticks after the part records
  std::vector<u64> host_cycles;
  TaskDesc* dtask = nullptr;  // descriptor of single-task launches
  uint32_t flags = 0;         // SPX_F_TRACE: trace every launch (spx_ctx_set_flags)
  uint64_t dev_allocs = 0;    // device allocations made so far
  // allocation-free solves: host images by shape, host copies of the counters after a launch
  std::map<std::string, std::shared_ptr<ImageHost>> host_images;
  std::vector<uint32_t> nc_counters;
};

struct spx_factor {
  spx_ctx* ctx = nullptr;
  int64_t n = 0, n_pad = 0;
  int32_t b = 0, nt = 0, prec = 0;
  double* tiles = nullptr;
  size_t tile_bytes = 0;
  void* low = nullptr;  // FP32 / BF16 copies of the panel tiles (mixed precision)
  double* dinv = nullptr;  // inverses of the 32x32 diagonal blocks of the diagonal tiles
  double* minv = nullptr;  // M_k = L_kk^{-T} of every diagonal tile (nt b^2)
  double* dscale = nullptr;  // D^{-1/2} (n_pad) of a factor of the scaled, shifted matrix
  double shift = 0.0;
  bool commute = false;  // made under SPX_F_COMMUTE: its solves use commutative updates too
};

namespace spx {

static void* dev_alloc(spx_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  ++c->dev_allocs;
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

static int get_program(spx_ctx* c, char kind, int nt, const Program** out, int psteps, bool commute) {
  const std::string key = std::string(1, kind) + ":" + std::to_string(nt) + ":" + std::to_string(psteps) +
                          (commute ? ":c" : "");
  auto it = c->programs.find(key);
  if (it != c->programs.end()) {
    *out = it->second.get();
    return SPX_OK;
  }
  std::unique_ptr<Program> pr(new Program());
  std::vector<spx_access> acc;
  switch (kind) {
    case 'F': cholesky_program(nt, false, pr->tasks, acc, true, psteps, commute); break;
    case 'S': solve_program(nt, pr->tasks, acc, commute); break;
    case 'L': io_program(nt, false, pr->tasks, acc, true, psteps); break;
    case 'P': io_program(nt, true, pr->tasks, acc, false, psteps); break;
    case 'K': io_program(nt, true, pr->tasks, acc, true, psteps); break;
    case 'Q': solve_io_program(nt, pr->tasks, acc); break;
    case 'M': gemm_program(nt, pr->tasks, acc, commute); break;
    default: return fail(SPX_EINVAL, "unknown program kind");
  }
  SPX_TRY(build_graph((uint32_t)pr->tasks.size(), acc.data(), acc.size(), nullptr, pr->g));
  rank_priorities(pr->tasks, pr->g);
  *out = pr.get();
  c->programs[key] = std::move(pr);
  return SPX_OK;
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
int trsm_rows_of(int /*b*/) { return 32; }  // the TRSM and inversion kernels take 32-row strips

// Steps of a diagonal factorization: large tiles of a matrix with at least four tile
// columns (whose one-workgroup POTRFs would dominate the critical path) are factored 32
// columns per task, with the rows of each step spread over workgroups.  Matrices of one or
// two tiles are left whole: their steps would only add task hops to a batched launch that
// other matrices already fill.  The rule depends on (nt, b) alone, so a matrix gets the
// same tasks, and the same bits, alone and in a batch.
int potrf_steps_of(int nt, int b) { return b >= 256 && nt >= 4 ? b / 32 : 1; }

uint16_t parts_of(const TaskDesc& d, int b, int nrhs) {
  const int sbase = (d.type == SPX_T_SYRK && d.pad) ? 64 : 128;
  const int sb = b < sbase ? b : sbase, ns = b / sb;
  switch (d.type) {
    case SPX_T_POTRF: {  // step c: the diagonal part, plus one per 32-row block below c + 1
      const int steps = d.pad >> 8, c = d.pad & 0xff, rows = steps - c - 2;
      return (uint16_t)(steps > 1 && c >= 1 && rows > 0 ? 1 + rows : 1);
    }
    case SPX_T_TRSM: return (uint16_t)(b / trsm_rows_of(b));
    case SPX_T_SYRK: return (uint16_t)(ns * (ns + 1) / 2);
    case SPX_T_GEMM: return (uint16_t)(ns * ns);
    case SPX_T_FTRSM:
    case SPX_T_BTRSM: return (uint16_t)((nrhs + 7) / 8 * (d.pad ? b / (b < 64 ? b : 64) : 1));
    case SPX_T_FGEMM:
    case SPX_T_BGEMM: return (uint16_t)(b / (b < 64 ? b : 64));
    case SPX_T_INV: return (uint16_t)(b / trsm_rows_of(b));
    case SPX_T_LOAD: {
      if (d.j) return 1;  // right-hand sides only
      const int ntiles = d.i * (d.i + 1) / 2;
      return (uint16_t)((ntiles <= kLoadTileParts ? ntiles : d.i) + (nrhs > 0 ? 1 : 0));
    }
    case SPX_T_STORE: return 1;
    case SPX_T_MGEMM: {
      const int s = b < 128 ? b : 128;
      return (uint16_t)((b / s) * (b / s));
    }
    case SPX_T_SPIN: return 1;
  }
  return 1;
}

// Priority class (priority >> 16, clamped to 0..63, larger = sooner) -> queue level of an
// image with nlev levels (level 0 is served first).
static int level_of(int32_t prio, int nlev) {
  int cls = prio >> 16;
  cls = cls < 0 ? 0 : (cls > kMaxLevels - 1 ? kMaxLevels - 1 : cls);
  return (kMaxLevels - 1 - cls) * nlev / kMaxLevels;
}

// kind 'F': factor (+ inversions); 'S': substitution alone (with the inverses); 'L': LOAD +
// factor + inversions; 'P': LOAD + factor + in-place substitution + STORE (one-shot
// solves: the inversions would cost more than they save); 'K': LOAD + factor +
// inversions + substitution with the inverses + STORE (factors kept for more solves);
// 'Q': LOAD of the right-hand sides + substitution with the inverses + STORE.
static int get_program(spx_ctx* c, char kind, int nt, const Program** out, int psteps = 1, bool commute = false);

// One matrix's share of an image: its program, descriptor index, tile size and
// right-hand-side count (parts per task depend on both).
struct Piece {
  const Program* p;
  uint32_t mat;
  int b, nrhs;
};

// Host form of a device image: the static arrays (task descriptors, CSR successors,
// in-degrees, part counts, the root items, the initial counters) laid out as one block,
// and the offsets of the per-launch arrays that follow them.
struct ImageHost {
  uint32_t ntasks = 0, total_parts = 0;
  int nlev = 1;
  uint32_t qbase[kLevelsMax] = {};
  uint32_t qcap[kLevelsMax] = {};
  uint32_t nroots = 0;
  int nshards = 1;
  uint32_t spread_max = 0;
  std::vector<char> bytes;       // the static part (static_bytes)
  std::vector<char> comm_bytes;  // the commutative-group arrays, uploaded at o_coff
  size_t o_tasks = 0, o_off = 0, o_succ = 0, o_indeg = 0, o_np = 0, o_q0 = 0, o_c0 = 0, static_bytes = 0;
  size_t o_pend = 0, o_pl = 0, o_q = 0, o_c = 0, o_ring = 0, total_bytes = 0;
  uint32_t ngroups = 0, ncroots = 0;
  size_t o_coff = 0, o_cent = 0, o_goff = 0, o_gtask = 0, o_gidx = 0, o_croots = 0, o_gstate = 0;
};

// Ready-queue shards of the sharded policy for one graph (environment SPX_QUEUE_SHARDS =
// 2, 4 or 8; default 4): the 64 queue words are split into shards x levels (at most kLevelsMax
// levels).  Four shards of sixteen levels measured best on the N = 16384 factor (43.5 ms;
// 8 x 8: 44.8 ms, where a panel task queues behind updates of up to four steps earlier in
// its level; 2 x 32: 45.2 ms, pops contend).
static int queue_shards() {
  static const int s = [] {
    const char* e = std::getenv("SPX_QUEUE_SHARDS");
    const int v = e ? std::atoi(e) : 4;
    return (v == 2 || v == 4 || v == 8) ? v : 4;
  }();
  return s;
}

// Parts a pop may claim at once outside the bulk levels: several where tasks average at
// least two parts (the factor, the solve, the tiled product), where long queues of parts
// otherwise leave workgroups idle behind the compare-and-swaps on one head; one where
// tasks are single parts (chains of small tasks, one-tile batches), where a claim of
// several tasks would run them one after the other while other workgroups wait.
static uint32_t claim_limit(uint32_t total_parts, uint32_t ntasks) {
  return (uint64_t)total_parts >= 2ull * ntasks ? 4u : 1u;
}

// Lays out the concatenation of the pieces' graphs (no edges between pieces) as one image.
static int build_image_host(const std::vector<Piece>& pieces, int policy, ImageHost& im) {
  // one ready queue per level keeps one matrix's tasks in global push order (its critical
  // path runs through the oldest bulk updates); independent matrices need no such order,
  // and sharded queues spread the pops of their many small tasks
  uint64_t T64 = 0, E64 = 0, P64 = 0;
  for (const Piece& pc : pieces) {
    T64 += pc.p->g.ntasks;
    E64 += pc.p->g.succ.size();
    for (const TaskDesc& d : pc.p->tasks) P64 += parts_of(d, pc.b, pc.nrhs);
  }
  // the finer levels of queue_shards() pay where priorities decide the makespan and
  // multi-part claims keep the pops ahead: one graph of multi-part tasks.  Batched images
  // keep 8 shards of 8 levels (their ranks are relative to each matrix, and finer levels
  // put every matrix's first tasks ahead of the later tasks of the matrices already
  // running: 4096 two-tile matrices 20.3 ms with 8 levels, 30.8 ms with 16), and so do
  // graphs of single-part tasks, whose pops need the spread (256 chains of 10 us tasks:
  // 17 us overhead per task with 8 shards, 58 us with 4)
  const bool fine = pieces.size() == 1 && claim_limit((uint32_t)std::min<uint64_t>(P64, UINT32_MAX),
                                                      (uint32_t)std::min<uint64_t>(T64, UINT32_MAX)) > 1;
  const int nshards = policy != SPX_Q_SHARDED && pieces.size() == 1 ? 1 : (fine ? queue_shards() : kShards);
  if (T64 >= (1ull << 32) - 1 || E64 >= (1ull << 32) - 1) return fail(SPX_EINVAL, "task graph too large");
  const uint32_t T = (uint32_t)T64;
  const size_t E = (size_t)E64;
  im.ntasks = T;
  im.nlev = policy == SPX_Q_FIFO ? 1 : (nshards > 1 ? kMaxQueues / nshards : kLevels1);
  std::vector<TaskDesc> tasks(T);
  std::vector<uint32_t> off32(T + 1), succ(std::max<size_t>(E, 1)), indeg(T), nparts(T);
  uint64_t per_level[kLevelsMax] = {};
  uint32_t t0 = 0;
  size_t e0 = 0;
  // commutative groups of all pieces, renumbered
  uint64_t G64 = 0, C64 = 0;
  for (const Piece& pc : pieces) {
    G64 += pc.p->g.ngroups;
    C64 += pc.p->g.cent.size();
  }
  if (G64 >= (1ull << 26)) return fail(SPX_EINVAL, "too many commutative groups");
  const bool comm = G64 > 0;
  std::vector<uint32_t> coff(comm ? T + 1 : 0, 0), cent, goff(comm ? G64 + 1 : 0, 0), gtask, gidx, croots;
  cent.reserve(C64);
  gtask.reserve(C64);
  gidx.reserve(C64);
  uint32_t g0 = 0;
  for (const Piece& pc : pieces) {
    const Program& pr = *pc.p;
    if (comm) {
      for (uint32_t t = 0; t < pr.g.ntasks; ++t) {
        const uint32_t n = pr.g.ngroups ? pr.g.coff[t + 1] - pr.g.coff[t] : 0;
        coff[t0 + t + 1] = coff[t0 + t] + n;
        for (uint32_t i = 0; i < n; ++i) cent.push_back(pr.g.cent[pr.g.coff[t] + i] + (g0 << 6));
      }
      for (uint32_t k = 0; k < pr.g.ngroups; ++k) {
        goff[g0 + k + 1] = goff[g0 + k] + (pr.g.goff[k + 1] - pr.g.goff[k]);
        for (uint32_t m = pr.g.goff[k]; m < pr.g.goff[k + 1]; ++m) {
          gtask.push_back(t0 + pr.g.gtask[m]);
          gidx.push_back(pr.g.gidx[m]);
        }
      }
      g0 += pr.g.ngroups;
    }
    for (uint32_t t = 0; t < pr.g.ntasks; ++t) {
      TaskDesc d = pr.tasks[t];
      d.nparts = parts_of(d, pc.b, pc.nrhs);
      d.level = (uint8_t)level_of(pr.g.prio[t], im.nlev);
      d.mat = pc.mat;
      tasks[t0 + t] = d;
      nparts[t0 + t] = d.nparts;
      indeg[t0 + t] = pr.g.indeg[t];
      off32[t0 + t] = (uint32_t)(e0 + pr.g.off[t]);
      per_level[d.level] += d.nparts;
    }
    // each task's successors by decreasing priority: those made ready by one completion are
    // pushed in that order, so within a queue level the most urgent one comes out first
    for (uint32_t t = 0; t < pr.g.ntasks; ++t) {
      const uint64_t a = pr.g.off[t], z = pr.g.off[t + 1];
      for (uint64_t e = a; e < z; ++e) succ[e0 + e] = t0 + pr.g.succ[e];
      std::stable_sort(succ.begin() + (e0 + a), succ.begin() + (e0 + z), [&](uint32_t x, uint32_t y) {
        return pr.g.prio[x - t0] > pr.g.prio[y - t0];
      });
    }
    t0 += pr.g.ntasks;
    e0 += pr.g.succ.size();
  }
  off32[T] = (uint32_t)E;
  uint64_t total = 0;
  for (int l = 0; l < kLevelsMax; ++l) total += per_level[l];
  if (total * kShards >= (1ull << 32) - 1) return fail(SPX_EINVAL, "task graph too large");
  im.total_parts = (uint32_t)total;
  for (int l = 0; l < kLevelsMax; ++l) im.qcap[l] = (uint32_t)per_level[l];
  for (int l = 1; l < kLevelsMax; ++l) im.qbase[l] = im.qbase[l - 1] + im.qcap[l - 1];
  // root parts are dealt round-robin over the shards of their level, the largest pieces
  // first (task count times b^3, about their work): ranks are relative to each piece's own
  // graph, so across independent matrices this queue order is what starts the longest
  // ones first (and leaves the short ones for the end of the launch)
  std::vector<uint32_t> porder(pieces.size()), pstart(pieces.size() + 1, 0);
  for (size_t i = 0; i < pieces.size(); ++i) {
    porder[i] = (uint32_t)i;
    pstart[i + 1] = pstart[i] + pieces[i].p->g.ntasks;
  }
  std::stable_sort(porder.begin(), porder.end(), [&](uint32_t x, uint32_t y) {
    const auto w = [&](uint32_t i) { return (double)pieces[i].p->g.ntasks * pieces[i].b * pieces[i].b * pieces[i].b; };
    return w(x) > w(y);
  });
  std::vector<u64> roots;
  std::vector<uint32_t> counters0(kNumCounters, 0);
  uint32_t deal = 0;
  for (uint32_t pi : porder)
  for (uint32_t t = pstart[pi]; t < pstart[pi + 1]; ++t) {
    if (indeg[t] != 0) continue;
    if (comm && coff[t + 1] > coff[t]) {  // takes its locks at the start of the launch
      croots.push_back(t);
      continue;
    }
    const int l = tasks[t].level;
    for (uint32_t p = 0; p < nparts[t]; ++p) {
      const int sh = (int)(deal++ % nshards);
      uint32_t& tail = counters0[ctr_queue_idx(l * nshards + sh) + 1];  // the high half of the word
      roots.push_back((u64)im.qbase[l] * kShards + (u64)sh * im.qcap[l] + tail);
      roots.push_back(((u64)t << 16) | p);
      ++tail;
    }
  }
  im.nroots = (uint32_t)(roots.size() / 2);
  im.nshards = nshards;
  // one graph: its small tasks deal their parts over the shards (latency-bound chains such
  // as the substitutions start all parts of a task at once); a batched launch keeps every
  // task's parts on one queue head, where thousands of independent small tasks already
  // spread over the shards (dealt there, FP32 batched factor: 16.6 -> 21.8 ms, workgroups
  // idle 22 -> 41 %, lost claim races on queues holding single parts)
  im.spread_max = pieces.size() == 1 ? 8u : 0u;
  if (roots.empty()) roots.assign(2, 0);
  // layout
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t o = 0;
  im.o_tasks = o; o = align(o + sizeof(TaskDesc) * T);
  im.o_off = o; o = align(o + 4 * (size_t)(T + 1));
  im.o_succ = o; o = align(o + 4 * succ.size());
  im.o_indeg = o; o = align(o + 4 * (size_t)T);
  im.o_np = o; o = align(o + 4 * (size_t)T);
  im.o_q0 = o; o = align(o + 8 * roots.size());
  im.o_c0 = o; o = align(o + 4 * (size_t)kNumCounters);
  im.static_bytes = o;
  im.o_pend = o; o = align(o + 4 * (size_t)T);
  im.o_pl = o; o = align(o + 4 * (size_t)T);
  im.o_q = o; o = align(o + 8 * (size_t)im.total_parts * kShards);
  im.o_c = o; o = align(o + 4 * (size_t)kNumCounters);
  im.o_ring = o; o = align(o + 4 * (size_t)kXcds * im.total_parts);
  im.ngroups = (uint32_t)G64;
  im.ncroots = (uint32_t)croots.size();
  if (comm) {
    im.o_gstate = o; o = align(o + 8 * (size_t)G64);
  }
  im.total_bytes = o;
  if (comm) {  // static arrays after the per-launch ones, to keep the earlier offsets
    im.o_coff = o; o = align(o + 4 * coff.size());
    im.o_cent = o; o = align(o + 4 * std::max<size_t>(cent.size(), 1));
    im.o_goff = o; o = align(o + 4 * goff.size());
    im.o_gtask = o; o = align(o + 4 * std::max<size_t>(gtask.size(), 1));
    im.o_gidx = o; o = align(o + 4 * std::max<size_t>(gidx.size(), 1));
    im.o_croots = o; o = align(o + 4 * std::max<size_t>(croots.size(), 1));
    im.total_bytes = o;
  }
  im.bytes.assign(im.static_bytes, 0);
  char* h = im.bytes.data();
  std::memcpy(h + im.o_tasks, tasks.data(), sizeof(TaskDesc) * T);
  std::memcpy(h + im.o_off, off32.data(), 4 * (size_t)(T + 1));
  std::memcpy(h + im.o_succ, succ.data(), 4 * succ.size());
  std::memcpy(h + im.o_indeg, indeg.data(), 4 * (size_t)T);
  std::memcpy(h + im.o_np, nparts.data(), 4 * (size_t)T);
  std::memcpy(h + im.o_q0, roots.data(), 8 * roots.size());
  std::memcpy(h + im.o_c0, counters0.data(), 4 * (size_t)kNumCounters);
  if (comm) {
    im.comm_bytes.assign(im.total_bytes - im.o_coff, 0);
    char* c = im.comm_bytes.data() - im.o_coff;  // addressed by image offsets
    std::memcpy(c + im.o_coff, coff.data(), 4 * coff.size());
    std::memcpy(c + im.o_cent, cent.data(), 4 * cent.size());
    std::memcpy(c + im.o_goff, goff.data(), 4 * goff.size());
    std::memcpy(c + im.o_gtask, gtask.data(), 4 * gtask.size());
    std::memcpy(c + im.o_gidx, gidx.data(), 4 * gidx.size());
    std::memcpy(c + im.o_croots, croots.data(), 4 * croots.size());
  }
  return SPX_OK;
}

// Points the arrays of `im` into the device block `base` laid out as `h` says.
static void bind_image(const ImageHost& h, char* base, Image* im) {
  im->ntasks = h.ntasks;
  im->total_parts = h.total_parts;
  im->nlev = h.nlev;
  for (int l = 0; l < kLevelsMax; ++l) {
    im->qbase[l] = h.qbase[l];
    im->qcap[l] = h.qcap[l];
  }
  im->nroots = h.nroots;
  im->nshards = h.nshards;
  im->spread_max = h.spread_max;
  im->bytes = h.total_bytes;
  im->tasks = (TaskDesc*)(base + h.o_tasks);
  im->succ_off = (uint32_t*)(base + h.o_off);
  im->succ = (uint32_t*)(base + h.o_succ);
  im->indeg = (uint32_t*)(base + h.o_indeg);
  im->nparts = (uint32_t*)(base + h.o_np);
  im->roots = (u64*)(base + h.o_q0);
  im->counters0 = (uint32_t*)(base + h.o_c0);
  im->pending = (uint32_t*)(base + h.o_pend);
  im->parts_left = (uint32_t*)(base + h.o_pl);
  im->queue = (u64*)(base + h.o_q);
  im->counters = (uint32_t*)(base + h.o_c);
  im->ring = (uint32_t*)(base + h.o_ring);
  im->ngroups = h.ngroups;
  im->ncroots = h.ncroots;
  if (h.ngroups) {
    im->gstate = (u64*)(base + h.o_gstate);
    im->coff = (uint32_t*)(base + h.o_coff);
    im->cent = (uint32_t*)(base + h.o_cent);
    im->goff = (uint32_t*)(base + h.o_goff);
    im->gtask = (uint32_t*)(base + h.o_gtask);
    im->gidx = (uint32_t*)(base + h.o_gidx);
    im->croots = (uint32_t*)(base + h.o_croots);
  }
}

// Uploads the concatenation of the pieces' graphs (no edges between pieces) as one
// device image.
static int make_image(spx_ctx* c, const std::vector<Piece>& pieces, int policy, Image** out) {
  ImageHost h;
  SPX_TRY(build_image_host(pieces, policy, h));
  std::unique_ptr<Image> im(new Image());
  im->block = dev_alloc(c, h.total_bytes);
  if (!im->block) return fail(SPX_ENOMEM, "device image: allocation failed");
  bind_image(h, (char*)im->block, im.get());
  // synchronous copy: the host vector is freed on return
  int rc = hipc(hipMemcpy(im->block, h.bytes.data(), h.static_bytes, hipMemcpyHostToDevice), "image upload");
  if (!rc && h.ngroups)
    rc = hipc(hipMemcpy((char*)im->block + h.o_coff, h.comm_bytes.data(), h.comm_bytes.size(), hipMemcpyHostToDevice),
              "image upload");
  if (rc) {
    dev_free(c, im->block);
    return rc;
  }
  *out = im.release();
  return SPX_OK;
}

// Builds (or returns the cached) device image of the factor (solve == false) or solve
// program for nt x nt tiles of size b.
static int get_image(spx_ctx* c, bool solve, int nt, int b, int nrhs, int policy, Image** out,
                     bool commute = false) {
  char key[96];
  const int rhs_parts = (nrhs + 7) / 8;
  std::snprintf(key, sizeof key, "%c:%d:%d:%d:%d:%d", solve ? 'S' : 'F', nt, b, solve ? rhs_parts : 0, policy,
                commute ? 1 : 0);
  auto it = c->images.find(key);
  if (it != c->images.end()) {
    *out = it->second;
    return SPX_OK;
  }
  const Program* pr = nullptr;
  SPX_TRY(get_program(c, solve ? 'S' : 'F', nt, &pr, solve ? 1 : potrf_steps_of(nt, b), commute));
  Image* im = nullptr;
  SPX_TRY(make_image(c, {Piece{pr, 0, b, nrhs}}, policy, &im));
  c->images[key] = im;
  *out = im;
  return SPX_OK;
}

static int ensure_small_buffers(spx_ctx* c, size_t nmats, size_t num_wg, size_t parts, bool trace, size_t tasks = 0) {
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
  // four words per part, then one push tick per task
  if (trace && 4 * parts + tasks > 4 * c->trace_cap) {
    dev_free(c, c->trace);
    dev_free(c, c->trace_idx);
    c->trace = (u64*)dev_alloc(c, 32 * parts + 8 * tasks);
    c->trace_idx = (uint32_t*)dev_alloc(c, 256);
    if (!c->trace || !c->trace_idx) return fail(SPX_ENOMEM, "trace buffer: allocation failed");
    c->trace_cap = parts + (tasks + 3) / 4;
  }
  return SPX_OK;
}

// Runs one image over `nmats` matrices (descriptors in c->hmats) and waits for it.
// On return c->hinfo[0..nmats) holds each matrix's info word.
static int run_image(spx_ctx* c, Image* im, int nmats, const spx_opts* o, double pack_ms) {
  const bool trace = (o && (o->flags & SPX_F_TRACE)) || (c->flags & SPX_F_TRACE);
  int num_wg = (o && o->num_wg > 0) ? o->num_wg : c->num_cu * c->wg_per_cu;
  if (num_wg < 1) num_wg = 1;
  SPX_TRY(ensure_small_buffers(c, nmats, num_wg, im->total_parts, trace, im->ntasks));
  SPX_TRY(hipc(hipMemcpyAsync(c->dmats, c->hmats, sizeof(DevMat) * nmats, hipMemcpyHostToDevice, c->stream),
               "descriptor upload"));
  SPX_TRY(launch_sched_init_full(im->pending, im->indeg, im->parts_left, im->nparts, im->ntasks, im->queue,
                                 im->total_parts * kShards, im->roots, im->nroots, im->counters, im->counters0,
                                 kNumCounters, im->ring, kXcds * im->total_parts, im->gstate, im->ngroups, c->dinfo,
                                 nmats, trace ? c->trace_idx : nullptr, c->stream));
  SchedArgs a{};
  a.tasks = im->tasks;
  a.succ_off = im->succ_off;
  a.succ = im->succ;
  a.pending = im->pending;
  a.parts_left = im->parts_left;
  a.queue = im->queue;
  a.counters = im->counters;
  a.ring = im->ring;
  a.ring_cap = im->total_parts;
  a.coff = im->coff;
  a.cent = im->cent;
  a.goff = im->goff;
  a.gtask = im->gtask;
  a.gidx = im->gidx;
  a.gstate = im->gstate;
  a.croots = im->croots;
  a.ncroots = im->ncroots;
  for (int l = 0; l < kLevelsMax; ++l) {
    a.qbase[l] = im->qbase[l];
    a.qcap[l] = im->qcap[l];
  }
  a.total_parts = im->total_parts;
  a.ntasks = im->ntasks;
  a.max_claim = claim_limit(im->total_parts, im->ntasks);
  a.spread_max = im->spread_max;
  a.nlev = im->nlev;
  a.nshards = im->nshards;
  a.mats = c->dmats;
  a.trace = trace ? c->trace : nullptr;
  a.trace_idx = trace ? c->trace_idx : nullptr;
  a.trace_push = trace ? c->trace + 4 * (size_t)im->total_parts : nullptr;
  a.wg_cycles = c->wg_cycles;
  a.spin_limit = 100000000ull * 20;  // 20 s of the 100 MHz device clock without progress
  SPX_TRY(hipc(hipEventRecord(c->ev[0], c->stream), "hipEventRecord"));
  SPX_TRY(launch_sched(a, num_wg, c->stream, im->family));
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
  c->trace_tasks = trace ? im->ntasks : 0;
  const uint32_t status = c->hcounters[kStatusIdx];
  uint64_t done = 0;  // parts taken from the queues; a normal exit means all of them ran
  for (int q = 0; q < kMaxQueues; ++q) done += c->hcounters[ctr_queue_idx(q)];
  if (status & STATUS_TIMEOUT)
    return failf(SPX_ETIMEOUT, "device scheduler made no progress (%llu of %u parts started)",
                 (unsigned long long)done, im->total_parts);
  if (done != im->total_parts)
    return failf(SPX_EDEVICE, "device scheduler ended early (%llu of %u parts started)", (unsigned long long)done,
                 im->total_parts);
  return SPX_OK;
}

static int tile_for_n(const spx_ctx* c, int prec, int64_t n) {
  const auto& t = c->tile_table[prec];
  if (t.empty()) return default_tile(n);
  for (const auto& e : t)
    if (n <= e.first) return e.second;
  return default_tile(n);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Cached image of a batched launch (a few, keyed by the whole shape list; oldest evicted).
static int get_batch_image(spx_ctx* c, const std::string& key, const std::vector<Piece>& pieces, int policy,
                           Image** out) {
  for (auto& kv : c->batch_images)
    if (kv.first == key) {
      *out = kv.second;
      return SPX_OK;
    }
  Image* im = nullptr;
  SPX_TRY(make_image(c, pieces, policy, &im));
  if (c->batch_images.size() >= 4) {
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, c->batch_images.front().second->block);
    delete c->batch_images.front().second;
    c->batch_images.erase(c->batch_images.begin());
  }
  c->batch_images.emplace_back(key, im);
  *out = im;
  return SPX_OK;
}

// One launch solving L_m L_m^T Y = B_m for the matrices in idx (factor f[m]); STORE
// writes Y to X_m, or adds it when accumulate is set.
static int batched_solve(spx_ctx* c, const std::vector<int>& idx, const spx_factor* const* f, const int64_t* q,
                         const double* const* B, const int64_t* ldb, double* const* X, const int64_t* ldx,
                         bool accumulate) {
  const int K = (int)idx.size();
  if (K == 0) return SPX_OK;
  std::vector<size_t> off(K);
  size_t ws = 0;
  std::string key = "Q";
  std::vector<Piece> pieces(K);
  for (int j = 0; j < K; ++j) {
    const spx_factor* g = f[idx[j]];
    off[j] = ws;
    ws = align256(ws + 2 * (size_t)g->n_pad * (size_t)q[idx[j]] * sizeof(double));
    const Program* pr = nullptr;
    SPX_TRY(get_program(c, 'Q', g->nt, &pr));
    pieces[j] = Piece{pr, (uint32_t)j, g->b, (int)q[idx[j]]};
    key += "," + std::to_string(g->nt) + "/" + std::to_string(g->b) + "/" + std::to_string((q[idx[j]] + 7) / 8);
  }
  Image* im = nullptr;
  SPX_TRY(get_batch_image(c, key, pieces, SPX_Q_SHARDED, &im));
  SPX_TRY(ensure_small_buffers(c, K, 1, 0, false));
  char* block = (char*)dev_alloc(c, ws);
  if (!block) return fail(SPX_ENOMEM, "batched solve: workspace allocation failed");
  for (int j = 0; j < K; ++j) {
    const int m = idx[j];
    const spx_factor* g = f[m];
    DevMat d{};
    d.tiles = g->tiles;
    d.dinv = g->dinv;
    d.minv = g->minv;
    d.rhs = (double*)(block + off[j]);
    d.rhs2 = d.rhs + (size_t)g->n_pad * (size_t)q[m];
    d.info = c->dinfo + j;
    d.n_pad = g->n_pad;
    d.nt = g->nt;
    d.b = g->b;
    d.nrhs = (int32_t)q[m];
    d.prec = PREC_FP64;
    d.n = (int32_t)g->n;
    d.trsm_rows = trsm_rows_of(g->b);
    d.B = B[m];
    d.ldb = ldb[m];
    d.X = X[m];
    d.ldx = ldx[m];
    d.store_acc = accumulate ? 1 : 0;
    c->hmats[j] = d;
  }
  int rc = run_image(c, im, K, nullptr, 0.0);
  dev_free(c, block);
  return rc;
}

// Normwise backward errors of the systems in idx (one launch): R_m = B_m - A_m X_m is
// written to R[m] (n x q row-major) and eta[m] receives the largest column error.
static int batched_eta(spx_ctx* c, const std::vector<int>& idx, const int64_t* n, const double* const* A,
                       const int64_t* lda, const int64_t* q, const double* const* X, const int64_t* ldx,
                       const double* const* B, const int64_t* ldb, double* const* R, double* eta) {
  const int K = (int)idx.size();
  if (K == 0) return SPX_OK;
  std::vector<ResDesc> rd(K);
  std::vector<uint32_t> prefix(K + 1, 0);
  std::vector<size_t> soff(K);
  size_t nstat = 0;
  for (int j = 0; j < K; ++j) {
    const int m = idx[j];
    soff[j] = nstat;
    nstat += 3 * (size_t)q[m] + 1;
    prefix[j + 1] = prefix[j] + (uint32_t)((n[m] + 63) / 64);
  }
  const size_t rd_bytes = align256(sizeof(ResDesc) * K), pf_bytes = align256(4 * (size_t)(K + 1));
  char* block = (char*)dev_alloc(c, rd_bytes + pf_bytes + nstat * sizeof(double));
  if (!block) return fail(SPX_ENOMEM, "batched residual: allocation failed");
  double* S = (double*)(block + rd_bytes + pf_bytes);
  for (int j = 0; j < K; ++j) {
    const int m = idx[j];
    rd[j] = ResDesc{n[m], lda[m], q[m], ldx[m], ldb[m], A[m], X[m], B[m], R[m], S + soff[j]};
  }
  std::vector<double> hs(nstat);
  int rc = hipc(hipMemcpyAsync(block, rd.data(), sizeof(ResDesc) * K, hipMemcpyHostToDevice, c->stream), "upload");
  if (!rc)
    rc = hipc(hipMemcpyAsync(block + rd_bytes, prefix.data(), 4 * (size_t)(K + 1), hipMemcpyHostToDevice, c->stream),
              "upload");
  if (!rc) rc = hipc(hipMemsetAsync(S, 0, nstat * sizeof(double), c->stream), "hipMemsetAsync");
  if (!rc)
    rc = launch_backward_error_batched((const ResDesc*)block, (const uint32_t*)(block + rd_bytes), K, prefix[K],
                                       c->stream);
  if (!rc) rc = hipc(hipMemcpyAsync(hs.data(), S, nstat * sizeof(double), hipMemcpyDeviceToHost, c->stream), "stats");
  if (!rc) rc = hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  dev_free(c, block);
  if (rc) return rc;
  for (int j = 0; j < K; ++j) {
    const int m = idx[j];
    const double* h = hs.data() + soff[j];
    const double anorm = h[3 * q[m]];
    double worst = 0.0;
    for (int64_t k = 0; k < q[m]; ++k) {
      const double e = h[3 * k] / (anorm * h[3 * k + 1] + h[3 * k + 2]);
      if (!(e <= worst)) worst = e;
    }
    eta[m] = worst;
  }
  return SPX_OK;
}

void ctx_set_store_flags(spx_ctx* c, unsigned int* const* flags) { c->store_flags = flags; }

int ctx_device(const spx_ctx* c) { return c->device; }

int ctx_copy_tile_tables(const spx_ctx* from, spx_ctx* to) {
  for (int p = 0; p < 3; ++p) to->tile_table[p] = from->tile_table[p];
  return SPX_OK;
}

// Batched factorisation (and with solve: substitution and STORE) of `count` matrices in
// one launch.  fout (factor-only calls): receives one handle per healthy matrix.
static int batched(spx_ctx* c, int count, const int64_t* n, const double* const* dA, const int64_t* lda,
                   const int64_t* nrhs, const double* const* dB, const int64_t* ldb, double* const* dX,
                   const int64_t* ldx, const spx_opts* o, bool solve, spx_factor** fout, int64_t* info) {
  const char* who = solve ? "spx_posv_batched" : "spx_potrf_batched";
  if (!c || !n || !dA || !lda || !info || (solve && (!nrhs || !dB || !ldb || !dX || !ldx)) || (!solve && !fout))
    return failf(SPX_EINVAL, "%s: null argument", who);
  const bool keep = fout != nullptr;  // per-matrix factor storage, handed to the caller
  if (count < 1 || count > (1 << 20)) return failf(SPX_EINVAL, "%s: count must be in [1, 2^20]", who);
  const int prec = o ? o->update_prec : SPX_PREC_FP64;
  if (prec != SPX_PREC_FP64 && prec != SPX_PREC_FP32 && prec != SPX_PREC_BF16)
    return failf(SPX_EINVAL, "%s: bad update precision", who);
  const int policy = o ? o->queue_policy : SPX_Q_SHARDED;
  if (policy != SPX_Q_PRIORITY && policy != SPX_Q_FIFO && policy != SPX_Q_SHARDED) return failf(SPX_EINVAL, "%s: bad queue policy", who);
  if (o && o->tile > 0 && !valid_tile(o->tile)) return failf(SPX_EINVAL, "%s: bad tile size", who);
  if (o && (o->flags & SPX_F_SCALED)) return failf(SPX_EINVAL, "%s: scaled factors are single-matrix only", who);
  if (o && (o->flags & SPX_F_COMMUTE)) return failf(SPX_EINVAL, "%s: commutative updates are single-matrix only", who);
  std::vector<int> bs(count), nts(count), qs(count, 0);
  for (int m = 0; m < count; ++m) {
    if (n[m] < 1 || lda[m] < n[m] || !dA[m]) return failf(SPX_EINVAL, "%s: matrix %d: bad n, lda or pointer", who, m);
    if (solve) {
      if (nrhs[m] < 1 || nrhs[m] > 4096 || ldb[m] < nrhs[m] || ldx[m] < nrhs[m] || !dB[m] || !dX[m])
        return failf(SPX_EINVAL, "%s: matrix %d: bad right-hand sides", who, m);
      if ((const double*)dX[m] == dB[m]) return failf(SPX_EINVAL, "%s: matrix %d: X aliases B", who, m);
      qs[m] = (int)nrhs[m];
    }
    bs[m] = (o && o->tile > 0) ? o->tile : tile_for_n(c, prec, n[m]);
    const int64_t nt = (n[m] + bs[m] - 1) / bs[m];
    if (nt > 2048) return failf(SPX_EINVAL, "%s: matrix %d: too many tiles", who, m);
    nts[m] = (int)nt;
  }
  SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
  // storage: one workspace for the whole batch (posv) or one factor per matrix (potrf)
  std::vector<size_t> off_t(count), off_d(count), off_r(count), off_l(count);
  size_t ws = 0;
  for (int m = 0; m < count; ++m) {
    const size_t b = bs[m], nt = nts[m], npad = nt * b;
    const size_t tb = nt * (nt + 1) / 2 * b * b * sizeof(double);
    if (!keep) {  // one-shot solve: in-place substitution, no tile inverses, one rhs copy
      off_t[m] = ws; ws = align256(ws + tb);
      off_d[m] = ws; ws = align256(ws + npad * 32 * sizeof(double));
    }
    off_r[m] = ws; ws = align256(ws + (keep ? 2 : 1) * npad * (size_t)qs[m] * sizeof(double));
    off_l[m] = ws; ws = align256(ws + ((prec == SPX_PREC_FP64 || keep) ? 0 : tb / (prec == SPX_PREC_FP32 ? 2 : 4)));
  }
  char* block = nullptr;
  std::vector<std::unique_ptr<spx_factor>> fs;
  auto release = [&]() {
    if (block) dev_free(c, block);
    for (auto& f : fs)
      if (f) {
        dev_free(c, f->tiles);
        dev_free(c, f->low);
        dev_free(c, f->dinv);
        dev_free(c, f->minv);
        f.reset();
      }
  };
  if (solve) {
    block = (char*)dev_alloc(c, ws);
    if (!block) return failf(SPX_ENOMEM, "%s: workspace allocation failed (%zu bytes)", who, ws);
  }
  if (keep) {
    fs.resize(count);
    for (int m = 0; m < count; ++m) {
      std::unique_ptr<spx_factor> f(new spx_factor());
      f->ctx = c;
      f->n = n[m];
      f->b = bs[m];
      f->nt = nts[m];
      f->n_pad = (int64_t)nts[m] * bs[m];
      f->prec = prec;
      f->tile_bytes = (size_t)nts[m] * (nts[m] + 1) / 2 * (size_t)bs[m] * bs[m] * sizeof(double);
      f->tiles = (double*)dev_alloc(c, f->tile_bytes);
      f->dinv = (double*)dev_alloc(c, (size_t)f->n_pad * 32 * sizeof(double));
      f->minv = (double*)dev_alloc(c, (size_t)f->n_pad * (size_t)bs[m] * sizeof(double));
      if (prec != SPX_PREC_FP64) f->low = dev_alloc(c, f->tile_bytes / (prec == SPX_PREC_FP32 ? 2 : 4));
      const bool ok = f->tiles && f->dinv && f->minv && (prec == SPX_PREC_FP64 || f->low);
      fs[m] = std::move(f);
      if (!ok) {
        release();
        return failf(SPX_ENOMEM, "%s: factor storage allocation failed", who);
      }
    }
  }
  // image: concatenated per-matrix programs
  const char kind = solve ? (keep ? 'K' : 'P') : 'L';
  std::string key(1, kind);
  key += ":" + std::to_string(policy);
  std::vector<Piece> pieces(count);
  for (int m = 0; m < count; ++m) {
    const Program* pr = nullptr;
    int rc = get_program(c, kind, nts[m], &pr, potrf_steps_of(nts[m], bs[m]));
    if (rc) {
      release();
      return rc;
    }
    pieces[m] = Piece{pr, (uint32_t)m, bs[m], qs[m]};
    key += "," + std::to_string(nts[m]) + "/" + std::to_string(bs[m]) + "/" + std::to_string((qs[m] + 7) / 8);
  }
  Image* im = nullptr;
  int rc = get_batch_image(c, key, pieces, policy, &im);
  if (!rc) rc = ensure_small_buffers(c, count, 1, 0, false);
  if (rc) {
    release();
    return rc;
  }
  for (int m = 0; m < count; ++m) {
    DevMat d{};
    if (keep) {
      d.tiles = fs[m]->tiles;
      d.dinv = fs[m]->dinv;
      d.minv = fs[m]->minv;
      d.low = fs[m]->low;
    } else {
      d.tiles = (double*)(block + off_t[m]);
      d.dinv = (double*)(block + off_d[m]);
      d.low = prec == SPX_PREC_FP64 ? nullptr : (void*)(block + off_l[m]);
    }
    if (solve) {
      d.rhs = (double*)(block + off_r[m]);
      if (keep) d.rhs2 = d.rhs + (size_t)nts[m] * bs[m] * (size_t)qs[m];
      d.B = dB[m];
      d.X = dX[m];
      d.ldb = ldb[m];
      d.ldx = ldx[m];
      d.done_flag = c->store_flags ? c->store_flags[m] : nullptr;
    }
    d.info = c->dinfo + m;
    d.n_pad = (int64_t)nts[m] * bs[m];
    d.nt = nts[m];
    d.b = bs[m];
    d.nrhs = qs[m];
    d.prec = prec;
    d.n = (int32_t)n[m];
    d.trsm_rows = trsm_rows_of(bs[m]);
    // a one-shot solve of a one-tile matrix reads only the tile's live lower part (POTRF
    // and the substitutions stop at the last live row and never read above the
    // diagonal), so its LOAD packs only the 64x64 blocks there
    d.load_live = kind == 'P' && nts[m] == 1 ? 1 : 0;
    d.A = dA[m];
    d.lda = lda[m];
    c->hmats[m] = d;
  }
  rc = run_image(c, im, count, o, 0.0);
  if (!rc) c->last.tile = (o && o->tile > 0) ? (uint32_t)o->tile : 0u;
  if (rc) {
    (void)hipStreamSynchronize(c->stream);
    release();
    return rc;
  }
  for (int m = 0; m < count; ++m) {
    info[m] = c->hinfo[m] == INT_MAX ? 0 : c->hinfo[m];
    if (keep) {
      if (info[m] == 0) {
        fout[m] = fs[m].release();
      } else {
        fout[m] = nullptr;
        dev_free(c, fs[m]->tiles);
        dev_free(c, fs[m]->low);
        dev_free(c, fs[m]->dinv);
        dev_free(c, fs[m]->minv);
        fs[m].reset();
      }
    }
  }
  if (block) dev_free(c, block);
  return SPX_OK;
}

}  // namespace spx

extern "C" {

const char* spx_last_error(void) { return g_err.c_str(); }

int spx_posv_batched(spx_ctx* c, int32_t count, const int64_t* n, const double* const* dA, const int64_t* lda,
                     const int64_t* nrhs, const double* const* dB, const int64_t* ldb, double* const* dX,
                     const int64_t* ldx, const spx_opts* opts, int64_t* info, spx_factor** keep) {
  if (keep && count > 0)
    for (int m = 0; m < count; ++m) keep[m] = nullptr;
  try {
    return batched(c, count, n, dA, lda, nrhs, dB, ldb, dX, ldx, opts, true, keep, info);
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_posv_batched: out of host memory");
  }
}

int spx_potrf_batched(spx_ctx* c, int32_t count, const int64_t* n, const double* const* dA, const int64_t* lda,
                      const spx_opts* opts, spx_factor** out, int64_t* info) {
  if (out && count > 0)
    for (int m = 0; m < count; ++m) out[m] = nullptr;
  try {
    return batched(c, count, n, dA, lda, nullptr, nullptr, nullptr, nullptr, nullptr, opts, false, out, info);
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_potrf_batched: out of host memory");
  }
}

int spx_potrs_batched(spx_ctx* c, int32_t count, spx_factor* const* f, const int64_t* nrhs, const double* const* dB,
                      const int64_t* ldb, double* const* dX, const int64_t* ldx, const double* const* dA,
                      const int64_t* lda, const spx_refine* refine, spx_solve_stats* stats) {
  if (!c || !f || !nrhs || !dB || !ldb || !dX || !ldx || count < 1 || count > (1 << 20))
    return fail(SPX_EINVAL, "spx_potrs_batched: bad argument");
  const int method = refine ? refine->method : 0;
  if (method < 0 || method > 1) return fail(SPX_EINVAL, "spx_potrs_batched: refinement method must be 0 or 1");
  const bool want_eta = dA != nullptr;
  if (method && !want_eta) return fail(SPX_EINVAL, "spx_potrs_batched: refinement needs the original matrices");
  if (want_eta && !lda) return fail(SPX_EINVAL, "spx_potrs_batched: lda missing");
  for (int m = 0; m < count; ++m) {
    if (!f[m] || !dB[m] || !dX[m] || nrhs[m] < 1 || nrhs[m] > 4096 || ldb[m] < nrhs[m] || ldx[m] < nrhs[m] ||
        (const double*)dX[m] == dB[m] || (want_eta && (!dA[m] || lda[m] < f[m]->n)))
      return failf(SPX_EINVAL, "spx_potrs_batched: system %d: bad argument", m);
  }
  try {
    SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
    std::vector<int> all(count);
    for (int m = 0; m < count; ++m) all[m] = m;
    double ms = 0.0;
    if (!(refine && refine->x_init && method)) {
      SPX_TRY(batched_solve(c, all, f, nrhs, dB, ldb, dX, ldx, false));
      ms += c->last.kernel_ms;
    }
    std::vector<int> iters(count, 0);
    std::vector<double> eta(count, -1.0);
    if (want_eta) {
      std::vector<int64_t> n(count), q1(count);
      size_t rtot = 0;
      std::vector<size_t> roff(count);
      for (int m = 0; m < count; ++m) {
        n[m] = f[m]->n;
        roff[m] = rtot;
        rtot = align256(rtot + (size_t)n[m] * (size_t)nrhs[m] * sizeof(double));
      }
      char* rblock = (char*)dev_alloc(c, rtot);
      if (!rblock) return fail(SPX_ENOMEM, "spx_potrs_batched: residual allocation failed");
      std::vector<double*> R(count);
      std::vector<const double*> Rc(count);
      for (int m = 0; m < count; ++m) {
        R[m] = (double*)(rblock + roff[m]);
        Rc[m] = R[m];
        q1[m] = nrhs[m];
      }
      const double tol = (refine && refine->tol > 0) ? refine->tol : 1e-12;
      const int max_iter = (refine && refine->max_iter > 0) ? refine->max_iter : 50;
      std::vector<double> prev(count, INFINITY);
      std::vector<int> slow(count, 0);
      std::vector<int> active = all;
      int rc = SPX_OK;
      for (;;) {
        rc = batched_eta(c, active, n.data(), dA, lda, nrhs, (const double* const*)dX, ldx, dB, ldb, R.data(),
                         eta.data());
        if (rc || !method) break;
        std::vector<int> next;
        for (int m : active) {
          if (eta[m] <= tol || iters[m] >= max_iter) continue;
          if (!(eta[m] < 0.5 * prev[m])) {  // stagnation (or NaN): stop after two slow steps
            if (++slow[m] >= 2 || eta[m] != eta[m]) continue;
          } else {
            slow[m] = 0;
          }
          prev[m] = eta[m];
          next.push_back(m);
        }
        if (next.empty()) break;
        rc = batched_solve(c, next, f, nrhs, Rc.data(), q1.data(), dX, ldx, true);
        if (rc) break;
        ms += c->last.kernel_ms;
        for (int m : next) ++iters[m];
        active.swap(next);
      }
      dev_free(c, rblock);
      if (rc) return rc;
    }
    c->last.kernel_ms = ms;
    if (stats)
      for (int m = 0; m < count; ++m) stats[m] = spx_solve_stats{iters[m], method, eta[m]};
    return SPX_OK;
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_potrs_batched: out of host memory");
  }
}

int spx_backward_error_batched(spx_ctx* c, int32_t count, const int64_t* n, const double* const* dA,
                               const int64_t* lda, const int64_t* nrhs, const double* const* dX, const int64_t* ldx,
                               const double* const* dB, const int64_t* ldb, double* eta_max) {
  if (!c || !n || !dA || !lda || !nrhs || !dX || !ldx || !dB || !ldb || !eta_max || count < 1 || count > (1 << 20))
    return fail(SPX_EINVAL, "spx_backward_error_batched: bad argument");
  for (int m = 0; m < count; ++m)
    if (n[m] < 1 || lda[m] < n[m] || nrhs[m] < 1 || ldx[m] < nrhs[m] || ldb[m] < nrhs[m] || !dA[m] || !dX[m] ||
        !dB[m])
      return failf(SPX_EINVAL, "spx_backward_error_batched: system %d: bad argument", m);
  try {
    SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
    size_t rtot = 0;
    std::vector<size_t> roff(count);
    for (int m = 0; m < count; ++m) {
      roff[m] = rtot;
      rtot = align256(rtot + (size_t)n[m] * (size_t)nrhs[m] * sizeof(double));
    }
    char* rblock = (char*)dev_alloc(c, rtot);
    if (!rblock) return fail(SPX_ENOMEM, "spx_backward_error_batched: allocation failed");
    std::vector<double*> R(count);
    std::vector<int> all(count);
    for (int m = 0; m < count; ++m) {
      R[m] = (double*)(rblock + roff[m]);
      all[m] = m;
    }
    int rc = batched_eta(c, all, n, dA, lda, nrhs, dX, ldx, dB, ldb, R.data(), eta_max);
    dev_free(c, rblock);
    return rc;
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_backward_error_batched: out of host memory");
  }
}

int spx_set_tile_table(spx_ctx* c, int32_t prec, int32_t count, const int64_t* n_max, const int32_t* tile) {
  if (!c || prec < 0 || prec > 2 || count < 0 || (count > 0 && (!n_max || !tile)))
    return fail(SPX_EINVAL, "spx_set_tile_table: bad argument");
  std::vector<std::pair<int64_t, int>> t;
  for (int i = 0; i < count; ++i) {
    if (!valid_tile(tile[i]) || n_max[i] < 1 || (i > 0 && n_max[i] <= n_max[i - 1]))
      return fail(SPX_EINVAL, "spx_set_tile_table: tiles must be valid and n_max increasing");
    t.emplace_back(n_max[i], tile[i]);
  }
  c->tile_table[prec] = t;
  return SPX_OK;
}

int spx_tile_for(const spx_ctx* c, int32_t prec, int64_t n, int32_t* tile) {
  if (!c || !tile || prec < 0 || prec > 2 || n < 1) return fail(SPX_EINVAL, "spx_tile_for: bad argument");
  *tile = tile_for_n(c, prec, n);
  return SPX_OK;
}

int spx_autotune_batched(spx_ctx* c, int32_t prec, int32_t nsizes, const int64_t* sizes, int32_t nrhs,
                         int32_t copies, int32_t reps, int32_t* best_tile, double* ms) {
  static const int cand[5] = {32, 64, 128, 256, 512};
  if (!c || !sizes || !best_tile || prec < 0 || prec > 2 || nsizes < 1 || nrhs < 1 || nrhs > 4096 || copies < 1 ||
      reps < 1)
    return fail(SPX_EINVAL, "spx_autotune_batched: bad argument");
  for (int i = 0; i < nsizes; ++i)
    if (sizes[i] < 1 || sizes[i] > 65536 || (i > 0 && sizes[i] <= sizes[i - 1]))
      return fail(SPX_EINVAL, "spx_autotune_batched: sizes must be increasing, in [1, 65536]");
  SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
  std::vector<int64_t> nmax(nsizes);
  std::vector<int32_t> best(nsizes);
  for (int i = 0; i < nsizes; ++i) {
    const int64_t sz = sizes[i];
    int64_t p2 = 32;
    while (p2 < sz) p2 *= 2;
    double* A = (double*)dev_alloc(c, (size_t)(sz * sz) * sizeof(double));
    double* B = (double*)dev_alloc(c, (size_t)(sz * nrhs) * sizeof(double));
    double* X = (double*)dev_alloc(c, (size_t)(sz * nrhs) * copies * sizeof(double));
    int rc = (!A || !B || !X) ? fail(SPX_ENOMEM, "spx_autotune_batched: allocation failed") : SPX_OK;
    if (!rc) rc = launch_spd_fill(A, sz, (uint32_t)i, c->stream);
    if (!rc) rc = hipc(hipMemsetAsync(B, 0, (size_t)(sz * nrhs) * sizeof(double), c->stream), "hipMemsetAsync");
    std::vector<int64_t> nv(copies, sz), ldv(copies, sz), qv(copies, nrhs), ldq(copies, nrhs), info(copies);
    std::vector<const double*> av(copies, A), bv(copies, B);
    std::vector<double*> xv(copies);
    for (int m = 0; m < copies; ++m) xv[m] = X + (size_t)m * sz * nrhs;
    double best_ms = INFINITY;
    int best_b = default_tile(sz);
    for (int ci = 0; ci < 5 && !rc; ++ci) {
      const int b = cand[ci];
      if (ms) ms[i * 5 + ci] = 0.0;
      if (b > p2) continue;
      spx_opts o{};
      o.tile = b;
      o.update_prec = prec;
      double t = INFINITY;
      for (int r = 0; r <= reps && !rc; ++r) {
        rc = batched(c, copies, nv.data(), av.data(), ldv.data(), qv.data(), bv.data(), ldq.data(), xv.data(),
                     ldq.data(), &o, true, nullptr, info.data());
        if (!rc && r > 0) t = std::min(t, c->last.kernel_ms);
      }
      if (rc) break;
      if (ms) ms[i * 5 + ci] = t;
      if (t < best_ms) {
        best_ms = t;
        best_b = b;
      }
    }
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, A);
    dev_free(c, B);
    dev_free(c, X);
    if (rc) return rc;
    nmax[i] = sz;
    best[i] = best_b;
    best_tile[i] = best_b;
  }
  return spx_set_tile_table(c, prec, nsizes, nmax.data(), best.data());
}


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
  SPX_TRY(scratch_init(device));  // the allocation-free solve's array on this device
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
  for (auto& kv : c->batch_images) {
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
  const int policy = opts ? opts->queue_policy : SPX_Q_SHARDED;
  if (policy != SPX_Q_PRIORITY && policy != SPX_Q_FIFO && policy != SPX_Q_SHARDED) return fail(SPX_EINVAL, "spx_potrf_tiled: bad queue policy");
  const int prec = opts ? opts->update_prec : SPX_PREC_FP64;
  if (prec != SPX_PREC_FP64 && prec != SPX_PREC_FP32 && prec != SPX_PREC_BF16)
    return fail(SPX_EINVAL, "spx_potrf_tiled: bad update precision");
  const int64_t nt = (n + b - 1) / b;
  if (nt > 2048) return fail(SPX_EINVAL, "spx_potrf_tiled: too many tiles");
  const bool scaled = opts && (opts->flags & SPX_F_SCALED);
  if (scaled && !(opts->shift >= 0.0)) return fail(SPX_EINVAL, "spx_potrf_tiled: shift must be >= 0");
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
  f->minv = (double*)dev_alloc(c, (size_t)f->n_pad * (size_t)b * sizeof(double));
  if (!f->dinv || !f->minv) {
    dev_free(c, f->tiles);
    dev_free(c, f->dinv);
    dev_free(c, f->minv);
    return fail(SPX_ENOMEM, "spx_potrf_tiled: block inverse allocation failed");
  }
  if (prec != SPX_PREC_FP64) {
    f->low = dev_alloc(c, f->tile_bytes / (prec == SPX_PREC_FP32 ? 2 : 4));
    if (!f->low) {
      dev_free(c, f->tiles);
      dev_free(c, f->dinv);
      dev_free(c, f->minv);
      return fail(SPX_ENOMEM, "spx_potrf_tiled: low-precision copy allocation failed");
    }
  }
  auto drop = [&]() {
    dev_free(c, f->tiles);
    dev_free(c, f->low);
    dev_free(c, f->dinv);
    dev_free(c, f->minv);
    dev_free(c, f->dscale);
  };
  Image* im = nullptr;
  f->commute = opts && (opts->flags & SPX_F_COMMUTE);
  int rc = get_image(c, false, (int)nt, b, 0, policy, &im, f->commute);
  if (!rc) rc = ensure_small_buffers(c, 1, 1, 0, false);
  if (!rc && scaled) {
    f->shift = opts->shift;
    f->dscale = (double*)dev_alloc(c, (size_t)f->n_pad * sizeof(double));
    rc = f->dscale ? launch_diag_scale(dA, lda, n, f->dscale, f->n_pad, c->stream)
                   : fail(SPX_ENOMEM, "spx_potrf_tiled: scale allocation failed");
  }
  if (rc) {
    drop();
    return rc;
  }
  DevMat m{};
  m.tiles = f->tiles;
  m.low = f->low;
  m.dinv = f->dinv;
  m.minv = f->minv;
  m.info = c->dinfo;
  m.n_pad = f->n_pad;
  m.nt = (int32_t)nt;
  m.b = b;
  m.prec = prec;
  m.n = (int32_t)n;
  m.trsm_rows = trsm_rows_of(b);
  m.dscale = f->dscale;
  m.shift = f->shift;
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
    drop();
    return rc;
  }
  if (c->hinfo[0] != INT_MAX) {
    *info = c->hinfo[0];
    drop();
    return SPX_OK;
  }
  *out = f.release();
  return SPX_OK;
}

int spx_gemm_tiled(spx_ctx* c, int64_t n, const double* dA, int64_t lda, const double* dB, int64_t ldb, double* dC,
                   int64_t ldc, const spx_opts* opts) {
  if (!c || !dA || !dB || !dC) return fail(SPX_EINVAL, "spx_gemm_tiled: null argument");
  if (n < 1 || lda < n || ldb < n || ldc < n) return fail(SPX_EINVAL, "spx_gemm_tiled: need n >= 1 and ld >= n");
  const int b = (opts && opts->tile > 0) ? opts->tile : default_tile(n);
  if (!valid_tile(b)) return fail(SPX_EINVAL, "spx_gemm_tiled: tile must be 32, 64, 128, 256 or 512");
  // default: sharded queues (nt^2 independent chains, no critical path to keep in order)
  const int policy = opts ? opts->queue_policy : SPX_Q_SHARDED;
  if (policy != SPX_Q_PRIORITY && policy != SPX_Q_FIFO && policy != SPX_Q_SHARDED) return fail(SPX_EINVAL, "spx_gemm_tiled: bad queue policy");
  if (opts && opts->update_prec != SPX_PREC_FP64) return fail(SPX_EINVAL, "spx_gemm_tiled: FP64 only");
  const int64_t nt = (n + b - 1) / b;
  if (nt > 160) return fail(SPX_EINVAL, "spx_gemm_tiled: too many tiles (at most 160 per side)");
  try {
    SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
    const size_t tile_bytes = (size_t)(nt * nt) * (size_t)b * (size_t)b * sizeof(double);
    char* block = (char*)dev_alloc(c, 3 * tile_bytes);
    if (!block) return fail(SPX_ENOMEM, "spx_gemm_tiled: tile storage allocation failed");
    double* ta = (double*)block;
    double* tbt = (double*)(block + tile_bytes);
    double* tc = (double*)(block + 2 * tile_bytes);
    char key[96];
    const bool commute = opts && (opts->flags & SPX_F_COMMUTE);
    std::snprintf(key, sizeof key, "M:%d:%d:%d:%d", (int)nt, b, policy, commute ? 1 : 0);
    Image* im = nullptr;
    int rc = SPX_OK;
    auto it = c->images.find(key);
    if (it != c->images.end()) {
      im = it->second;
    } else {
      const Program* pr = nullptr;
      rc = get_program(c, 'M', (int)nt, &pr, 1, commute);
      if (!rc) rc = make_image(c, {Piece{pr, 0, b, 0}}, policy, &im);
      if (!rc) {
        im->family = FAM_GEMM;
        c->images[key] = im;
      }
    }
    if (!rc) rc = ensure_small_buffers(c, 1, 1, 0, false);
    if (!rc) rc = hipc(hipEventRecord(c->ev[2], c->stream), "hipEventRecord");
    if (!rc) rc = launch_pack_full(dA, lda, n, ta, b, (int)nt, 0, c->stream);
    if (!rc) rc = launch_pack_full(dB, ldb, n, tbt, b, (int)nt, 1, c->stream);
    if (!rc) rc = launch_pack_full(dC, ldc, n, tc, b, (int)nt, 0, c->stream);
    if (!rc) rc = hipc(hipEventRecord(c->ev[3], c->stream), "hipEventRecord");
    if (!rc) {
      DevMat m{};
      m.tiles = tc;
      m.ga = ta;
      m.gbt = tbt;
      m.info = c->dinfo;
      m.n_pad = nt * b;
      m.nt = (int32_t)nt;
      m.b = b;
      m.n = (int32_t)n;
      c->hmats[0] = m;
      rc = run_image(c, im, 1, opts, 0.0);
    }
    if (!rc) {
      float pms = 0.f;
      if (hipEventElapsedTime(&pms, c->ev[2], c->ev[3]) == hipSuccess) c->last.pack_ms = pms;
      c->last.tile = (uint32_t)b;
      rc = launch_unpack_full(tc, b, (int)nt, n, dC, ldc, c->stream);
    }
    if (!rc) rc = hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, block);
    return rc;
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_gemm_tiled: out of host memory");
  }
}

int spx_run_graph(spx_ctx* c, const spx_graph* g, uint64_t spin_ticks, const spx_opts* opts) {
  if (!c || !g) return fail(SPX_EINVAL, "spx_run_graph: null argument");
  if (spin_ticks > 1000000000ull) return fail(SPX_EINVAL, "spx_run_graph: spin_ticks above 10^9");
  if (g->g.ntasks == 0) return fail(SPX_EINVAL, "spx_run_graph: empty graph");
  const int policy = opts ? opts->queue_policy : SPX_Q_SHARDED;
  if (policy != SPX_Q_PRIORITY && policy != SPX_Q_FIFO && policy != SPX_Q_SHARDED) return fail(SPX_EINVAL, "spx_run_graph: bad queue policy");
  try {
    SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
    // every task a spin task; the graph's priorities spread over the queue levels (the
    // largest ones first), ties served in push order
    Program pr;
    pr.g = g->g;
    pr.tasks.assign(g->g.ntasks, TaskDesc());
    int32_t pmin = INT32_MAX, pmax = INT32_MIN;
    for (int32_t p : g->g.prio) {
      pmin = std::min(pmin, p);
      pmax = std::max(pmax, p);
    }
    for (uint32_t t = 0; t < g->g.ntasks; ++t) {
      pr.tasks[t].type = SPX_T_SPIN;
      // priority -> base 0..kMaxLevels-1 for level_of: equal priorities share the first level
      const int64_t span = (int64_t)pmax - pmin;
      const int top = kMaxLevels - 1;
      const int base = span > 0 ? (int)(top * ((int64_t)g->g.prio[t] - pmin) / span) : top;
      pr.g.prio[t] = base << 16;
    }
    Image* im = nullptr;
    SPX_TRY(make_image(c, {Piece{&pr, 0, 32, 0}}, policy, &im));
    std::unique_ptr<Image> own(im);
    im->family = FAM_SPIN;
    int rc = ensure_small_buffers(c, 1, 1, 0, false);
    if (!rc) {
      DevMat m{};
      m.info = c->dinfo;
      m.spin_ticks = spin_ticks;
      c->hmats[0] = m;
      rc = run_image(c, im, 1, opts, 0.0);
    }
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, im->block);
    return rc;
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_run_graph: out of host memory");
  }
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
  dev_free(f->ctx, f->minv);
  dev_free(f->ctx, f->dscale);
  delete f;
}

// Runs the solve graph of factor f on the column-major work buffer rhs (n_pad x nrhs;
// rhs2: a second one of the same shape that the diagonal solves write).
static int solve_on(spx_ctx* c, const spx_factor* f, int64_t nrhs, double* rhs, double* rhs2) {
  Image* im = nullptr;
  SPX_TRY(get_image(c, true, f->nt, f->b, (int)nrhs, SPX_Q_SHARDED, &im, f->commute));
  SPX_TRY(ensure_small_buffers(c, 1, 1, 0, false));
  DevMat m{};
  m.tiles = f->tiles;
  m.dinv = f->dinv;
  m.minv = f->minv;
  m.rhs = rhs;
  m.rhs2 = rhs2;
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

// Y = M^{-1} R for the n x nrhs row-major R (ld ldr) into Y (ld ldy; accumulate: Y +=),
// M = L L^T, or D^{1/2} L L^T D^{1/2} for a scaled factor; rhs: 2 x n_pad x nrhs work.
static int apply_inverse(spx_ctx* c, const spx_factor* f, int64_t nrhs, const double* R, int64_t ldr, double* Y,
                         int64_t ldy, int accumulate, double* rhs, double* ms) {
  SPX_TRY(launch_rhs_in(R, ldr, f->n, nrhs, rhs, f->n_pad, f->dscale, c->stream));
  SPX_TRY(solve_on(c, f, nrhs, rhs, rhs + (size_t)f->n_pad * (size_t)nrhs));
  *ms += c->last.kernel_ms;
  return launch_rhs_out(rhs, f->n_pad, f->n, nrhs, Y, ldy, accumulate, f->dscale, c->stream);
}

// Column sums of U .* V (n x q row-major), reduced on the host in a fixed order.
static int dot_cols(spx_ctx* c, int64_t n, int64_t q, const double* U, const double* V, double* partial,
                    std::vector<double>& hp, double* out) {
  int nthr = 0;
  SPX_TRY(launch_dot_cols(n, q, U, V, partial, &nthr, c->stream));
  hp.resize(nthr);
  SPX_TRY(hipc(hipMemcpyAsync(hp.data(), partial, sizeof(double) * nthr, hipMemcpyDeviceToHost, c->stream), "dot"));
  SPX_TRY(hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize"));
  for (int64_t k = 0; k < q; ++k) out[k] = 0.0;
  for (int g = 0; g < nthr; ++g) out[g % q] += hp[g];
  return SPX_OK;
}

int spx_potrs(spx_ctx* c, const spx_factor* f, int64_t nrhs, const double* dB, int64_t ldb, double* dX, int64_t ldx,
              const double* dA, int64_t lda, const spx_refine* refine, spx_solve_stats* stats) {
  if (!c || !f || !dB || !dX) return fail(SPX_EINVAL, "spx_potrs: null argument");
  if (nrhs < 1 || nrhs > 4096 || ldb < nrhs || ldx < nrhs) return fail(SPX_EINVAL, "spx_potrs: bad nrhs / ld");
  if (dX == dB && ldx != ldb) return fail(SPX_EINVAL, "spx_potrs: aliased X and B need equal leading dimensions");
  const int method = refine ? refine->method : 0;
  if (method < 0 || method > 2) return fail(SPX_EINVAL, "spx_potrs: refinement method must be 0, 1 or 2");
  if (method && (!dA || lda < f->n)) return fail(SPX_EINVAL, "spx_potrs: refinement needs the original matrix");
  if (method && dX == dB) return fail(SPX_EINVAL, "spx_potrs: refinement needs X distinct from B");
  SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
  const int64_t n = f->n, q = nrhs;
  const size_t vec = (size_t)n * (size_t)q * sizeof(double);
  std::vector<void*> bufs;
  auto get = [&](size_t bytes) {
    void* p = dev_alloc(c, bytes);
    bufs.push_back(p);
    return (double*)p;
  };
  double* rhs = get(2 * (size_t)f->n_pad * (size_t)q * sizeof(double));
  double* R = method ? get(vec) : nullptr;
  double* S = method ? get(sizeof(double) * (size_t)(3 * q + 1)) : nullptr;
  double *Z = nullptr, *P = nullptr, *NQ = nullptr, *zero = nullptr, *part = nullptr, *alpha = nullptr;
  double* X = dX;  // PCG works on a dense n x q copy when X has a wider leading dimension
  int64_t ldw = ldx;
  if (method == 2) {
    if (ldx != q) {
      X = get(vec);
      ldw = q;
    }
    Z = get(vec);
    P = get(vec);
    NQ = get(vec);
    zero = get(vec);
    part = get(sizeof(double) * 256 * 256);
    alpha = get(sizeof(double) * (size_t)q);
  }
  int rc = SPX_OK;
  for (void* p : bufs)
    if (!p) rc = fail(SPX_ENOMEM, "spx_potrs: work buffer allocation failed");
  double solve_ms = 0.0;
  const bool x_init = refine && refine->x_init && method;
  if (!rc && x_init && X != dX)
    rc = hipc(hipMemcpy2DAsync(X, (size_t)ldw * 8, dX, (size_t)ldx * 8, (size_t)q * 8, (size_t)n, hipMemcpyDeviceToDevice,
                               c->stream),
              "copy");
  if (!rc && !x_init) rc = apply_inverse(c, f, q, dB, ldb, X, ldw, 0, rhs, &solve_ms);
  int iters = 0;
  double eta_max = -1.0;
  const double tol = (refine && refine->tol > 0) ? refine->tol : 1e-12;
  const int max_iter = (refine && refine->max_iter > 0) ? refine->max_iter : 50;
  std::vector<double> hs;
  if (!rc && method == 1) {
    // classical iterative refinement: r = b - A x in FP64 with the original matrix,
    // d = M^{-1} r, x += d, until the largest normwise backward error <= tol
    double prev = INFINITY;
    int slow = 0;
    for (;;) {
      rc = residual_eta(c, n, dA, lda, q, dX, ldx, dB, ldb, R, S, hs, nullptr, &eta_max);
      if (rc || eta_max <= tol || iters >= max_iter) break;
      if (!(eta_max < 0.5 * prev)) {  // stagnation (or NaN): stop after two slow steps
        if (++slow >= 2 || eta_max != eta_max) break;
      } else {
        slow = 0;
      }
      prev = eta_max;
      rc = apply_inverse(c, f, q, R, q, dX, ldx, 1, rhs, &solve_ms);
      if (rc) break;
      ++iters;
    }
  } else if (!rc && method == 2) {
    // preconditioned conjugate gradients on A x = b, one recurrence per column, started
    // from x0 = M^{-1} b; the true residual replaces the recurrence every iteration
    std::vector<double> rho(q), pq(q), rz(q), a(q), hp;
    double best = INFINITY;
    int since_best = 0;
    rc = hipc(hipMemsetAsync(zero, 0, vec, c->stream), "hipMemsetAsync");
    if (!rc) rc = residual_eta(c, n, dA, lda, q, X, ldw, dB, ldb, R, S, hs, nullptr, &eta_max);
    if (!rc && !(eta_max <= tol)) {
      rc = apply_inverse(c, f, q, R, q, Z, q, 0, rhs, &solve_ms);
      if (!rc) rc = hipc(hipMemcpyAsync(P, Z, vec, hipMemcpyDeviceToDevice, c->stream), "copy");
      if (!rc) rc = dot_cols(c, n, q, R, Z, part, hp, rho.data());
      while (!rc && iters < max_iter) {
        // NQ = 0 - A P
        double unused = 0.0;
        rc = residual_eta(c, n, dA, lda, q, P, q, zero, q, NQ, S, hs, nullptr, &unused);
        if (!rc) rc = dot_cols(c, n, q, P, NQ, part, hp, pq.data());
        if (rc) break;
        for (int64_t k = 0; k < q; ++k) a[k] = (pq[k] != 0.0 && rho[k] != 0.0) ? rho[k] / -pq[k] : 0.0;
        rc = hipc(hipMemcpyAsync(alpha, a.data(), sizeof(double) * q, hipMemcpyHostToDevice, c->stream), "alpha");
        if (!rc) rc = launch_axpy_cols(n, q, alpha, P, X, 0, c->stream);  // x += alpha p
        if (rc) break;
        ++iters;
        rc = residual_eta(c, n, dA, lda, q, X, ldw, dB, ldb, R, S, hs, nullptr, &eta_max);
        if (rc || eta_max <= tol) break;
        if (eta_max < best) {
          best = eta_max;
          since_best = 0;
        } else if (++since_best >= 10 || eta_max != eta_max) {
          break;
        }
        rc = apply_inverse(c, f, q, R, q, Z, q, 0, rhs, &solve_ms);
        if (!rc) rc = dot_cols(c, n, q, R, Z, part, hp, rz.data());
        if (rc) break;
        for (int64_t k = 0; k < q; ++k) {
          a[k] = rho[k] != 0.0 ? rz[k] / rho[k] : 0.0;
          rho[k] = rz[k];
        }
        rc = hipc(hipMemcpyAsync(alpha, a.data(), sizeof(double) * q, hipMemcpyHostToDevice, c->stream), "beta");
        if (!rc) rc = launch_axpy_cols(n, q, alpha, Z, P, 1, c->stream);  // p = z + beta p
      }
    }
    if (!rc && X != dX)
      rc = hipc(hipMemcpy2DAsync(dX, (size_t)ldx * 8, X, (size_t)q * 8, (size_t)q * 8, (size_t)n, hipMemcpyDeviceToDevice,
                                 c->stream),
                "copy");
  }
  if (!rc) rc = hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  (void)hipStreamSynchronize(c->stream);
  for (void* p : bufs) dev_free(c, p);
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
  d.nparts = parts_of(d, b, nrhs);  // pad = 0: the in-place substitution kernels
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
  int rc = hipc(hipMemcpyAsync(c->dmats, c->hmats, sizeof(DevMat), hipMemcpyHostToDevice, c->stream), "upload");
  if (!rc) rc = hipc(hipMemcpyAsync(c->dinfo, &healthy, 4, hipMemcpyHostToDevice, c->stream), "upload");
  SchedArgs a{};
  a.tasks = c->dtask;
  a.mats = c->dmats;
  if (!rc) rc = hipc(hipMemcpyAsync(c->dtask, &d, sizeof d, hipMemcpyHostToDevice, c->stream), "task upload");
  if (!rc) rc = launch_one_task(a, d.nparts, c->stream);
  if (!rc) rc = hipc(hipMemcpyAsync(c->hinfo, c->dinfo, 4, hipMemcpyDeviceToHost, c->stream), "info");
  if (!rc) rc = hipc(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  dev_free(c, dinv);
  if (rc) return rc;
  *info = c->hinfo[0] == INT_MAX ? 0 : c->hinfo[0];
  return SPX_OK;
}

int spx_ctx_set_flags(spx_ctx* c, uint32_t flags) {
  if (!c || (flags & ~(uint32_t)SPX_F_TRACE)) return fail(SPX_EINVAL, "spx_ctx_set_flags: bad argument");
  c->flags = flags;
  return SPX_OK;
}

int spx_last_stats(const spx_ctx* c, spx_stats* out) {
  if (!c || !out) return fail(SPX_EINVAL, "spx_last_stats: null argument");
  *out = c->last;
  out->device_allocs = c->dev_allocs;
  return SPX_OK;
}

int spx_potrs_noalloc(spx_ctx* c, const spx_factor* f, int64_t nrhs, const double* dB, int64_t ldb, double* dX,
                      int64_t ldx) {
  if (!c || !f || !dB || !dX) return fail(SPX_EINVAL, "spx_potrs_noalloc: null argument");
  if (nrhs < 1 || nrhs > 4096 || ldb < nrhs || ldx < nrhs) return fail(SPX_EINVAL, "spx_potrs_noalloc: bad nrhs / ld");
  if (dX == dB && ldx != ldb) return fail(SPX_EINVAL, "spx_potrs_noalloc: aliased X and B need equal leading dimensions");
  try {
    SPX_TRY(hipc(hipSetDevice(c->device), "hipSetDevice"));
    void* sp = nullptr;
    SPX_TRY(scratch_get(c->device, &sp));
    // the host image of the solve graph (host memory only), cached by shape
    char key[96];
    std::snprintf(key, sizeof key, "S:%d:%d:%d:%d", f->nt, f->b, (int)((nrhs + 7) / 8), f->commute ? 1 : 0);
    std::shared_ptr<ImageHost>& h = c->host_images[key];
    if (!h) {
      const Program* pr = nullptr;
      SPX_TRY(get_program(c, 'S', f->nt, &pr, 1, f->commute));
      std::shared_ptr<ImageHost> nh(new ImageHost());
      SPX_TRY(build_image_host({Piece{pr, 0, f->b, (int)nrhs}}, SPX_Q_SHARDED, *nh));
      h = nh;
    }
    // scratch layout: image (static + per-launch arrays), matrix descriptor, info word,
    // the two right-hand-side copies
    const size_t o_mat = align256(h->total_bytes);
    const size_t o_info = o_mat + align256(sizeof(DevMat));
    const size_t o_rhs = o_info + 256;
    const size_t rhs_bytes = 2 * (size_t)f->n_pad * (size_t)nrhs * sizeof(double);
    const size_t need = o_rhs + align256(rhs_bytes);
    if (need > kScratchBytes)
      return failf(SPX_EINVAL, "spx_potrs_noalloc: this solve needs %zu bytes of scratch, the limit is %zu", need,
                   (size_t)kScratchBytes);
    char* base = (char*)sp;
    Image im;
    bind_image(*h, base, &im);
    DevMat m{};
    m.tiles = f->tiles;
    m.dinv = f->dinv;
    m.minv = f->minv;
    m.rhs = (double*)(base + o_rhs);
    m.rhs2 = m.rhs + (size_t)f->n_pad * (size_t)nrhs;
    m.info = (int32_t*)(base + o_info);
    m.n_pad = f->n_pad;
    m.nt = f->nt;
    m.b = f->b;
    m.nrhs = (int32_t)nrhs;
    m.prec = PREC_FP64;
    m.n = (int32_t)f->n;
    m.trsm_rows = trsm_rows_of(f->b);
    hipStream_t st = c->stream;
    SPX_TRY(hipc(hipMemcpyAsync(base, h->bytes.data(), h->static_bytes, hipMemcpyHostToDevice, st), "image upload"));
    if (h->ngroups)
      SPX_TRY(hipc(hipMemcpyAsync(base + h->o_coff, h->comm_bytes.data(), h->comm_bytes.size(),
                                  hipMemcpyHostToDevice, st),
                   "image upload"));
    SPX_TRY(hipc(hipMemcpyAsync(base + o_mat, &m, sizeof m, hipMemcpyHostToDevice, st), "descriptor upload"));
    SPX_TRY(launch_rhs_in(dB, ldb, f->n, nrhs, m.rhs, f->n_pad, f->dscale, st));
    SPX_TRY(launch_sched_init_full(im.pending, im.indeg, im.parts_left, im.nparts, im.ntasks, im.queue,
                                   im.total_parts * kShards, im.roots, im.nroots, im.counters, im.counters0,
                                   kNumCounters, im.ring, kXcds * im.total_parts, im.gstate, im.ngroups, m.info, 1,
                                   nullptr, st));
    SchedArgs a{};
    a.tasks = im.tasks;
    a.succ_off = im.succ_off;
    a.succ = im.succ;
    a.pending = im.pending;
    a.parts_left = im.parts_left;
    a.queue = im.queue;
    a.counters = im.counters;
    a.ring = im.ring;
    a.ring_cap = im.total_parts;
    a.coff = im.coff;
    a.cent = im.cent;
    a.goff = im.goff;
    a.gtask = im.gtask;
    a.gidx = im.gidx;
    a.gstate = im.gstate;
    a.croots = im.croots;
    a.ncroots = im.ncroots;
    for (int l = 0; l < kLevelsMax; ++l) {
      a.qbase[l] = im.qbase[l];
      a.qcap[l] = im.qcap[l];
    }
    a.total_parts = im.total_parts;
    a.ntasks = im.ntasks;
    a.max_claim = claim_limit(im.total_parts, im.ntasks);
    a.spread_max = im.spread_max;
    a.nlev = im.nlev;
    a.nshards = im.nshards;
    a.mats = (const DevMat*)(base + o_mat);
    a.spin_limit = 100000000ull * 20;
    int num_wg = c->num_cu * c->wg_per_cu;
    if (num_wg < 1) num_wg = 1;
    SPX_TRY(hipc(hipEventRecord(c->ev[0], st), "hipEventRecord"));
    SPX_TRY(launch_sched(a, num_wg, st));
    SPX_TRY(hipc(hipEventRecord(c->ev[1], st), "hipEventRecord"));
    SPX_TRY(launch_rhs_out(m.rhs, f->n_pad, f->n, nrhs, dX, ldx, 0, f->dscale, st));
    c->nc_counters.resize(kNumCounters);
    SPX_TRY(hipc(hipMemcpyAsync(c->nc_counters.data(), im.counters, 4 * kNumCounters, hipMemcpyDeviceToHost, st),
                 "counters"));
    SPX_TRY(hipc(hipStreamSynchronize(st), "hipStreamSynchronize"));
    float ms = 0.f;
    SPX_TRY(hipc(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]), "hipEventElapsedTime"));
    c->last = spx_stats{};
    c->last.kernel_ms = ms;
    c->last.ntasks = im.ntasks;
    c->last.nparts = im.total_parts;
    c->last.num_wg = (uint32_t)num_wg;
    c->last.tile = (uint32_t)f->b;
    c->trace_len = 0;
    uint64_t done = 0;
    for (int q = 0; q < kMaxQueues; ++q) done += c->nc_counters[ctr_queue_idx(q)];
    if (c->nc_counters[kStatusIdx] & STATUS_TIMEOUT)
      return failf(SPX_ETIMEOUT, "device scheduler made no progress (%llu of %u parts started)",
                   (unsigned long long)done, im.total_parts);
    if (done != im.total_parts)
      return failf(SPX_EDEVICE, "device scheduler ended early (%llu of %u parts started)", (unsigned long long)done,
                   im.total_parts);
    return SPX_OK;
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_potrs_noalloc: out of host memory");
  }
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

int64_t spx_trace_push(const spx_ctx* c, uint64_t* ticks, int64_t cap) {
  if (!c) return fail(SPX_EINVAL, "spx_trace_push: null context");
  if (c->trace_len <= 0 || c->trace_tasks <= 0) return 0;
  const int64_t n = std::min<int64_t>(cap, c->trace_tasks);
  if (ticks && n > 0) {
    if (hipMemcpy(ticks, c->trace + 4 * c->trace_len, 8 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(SPX_EDEVICE, "spx_trace_push: copy failed");
  }
  return c->trace_tasks;
}

}  // extern "C"
