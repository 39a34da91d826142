// Internal declarations shared by the host runtime and the HIP kernels of libspx.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "spx.h"

namespace spx {

// Records a message for spx_last_error() and returns `code`.
int fail(int code, const char* msg);
int failf(int code, const char* fmt, ...);

// Immediate-dependency graph in CSR form (successors), with in-degrees and priorities.
// Commutative-write groups: a run of at most kGroupMax consecutive commutative writes of
// one datum; its members may run in any order, one at a time.
constexpr int kGroupMax = 63;
struct Graph {
  uint32_t ntasks = 0;
  std::vector<uint64_t> off;  // ntasks + 1
  std::vector<uint32_t> succ;
  std::vector<uint32_t> indeg;
  std::vector<int32_t> prio;
  // commutative writes (empty when the graph has none): task t's groups are
  // cent[coff[t] .. coff[t+1]) = (group << 6) | slot, by increasing group (the order the
  // task takes their locks in); group g's members are gtask/gidx[goff[g] .. goff[g+1])
  // (slot s = member goff[g] + s; gidx = the entry's index within its task's list)
  uint32_t ngroups = 0;
  std::vector<uint32_t> coff, cent, goff, gtask, gidx;
};

// Device task descriptor (16 bytes).  `level` is the ready-queue level (0 = served
// first); `nparts` the number of workgroup-sized pieces the task is cut into; `pad` = 1
// marks the solve tasks that use the tile inverse M_k (row-split, out of place) and the
// SYRK(k+1, k+1, k) that the next diagonal factorization waits on (64x64 parts).
struct TaskDesc {
  uint8_t type = 0;
  uint8_t level = 0;
  uint16_t nparts = 1;
  uint16_t i = 0, j = 0, k = 0;
  uint16_t pad = 0;
  uint32_t mat = 0;
};
static_assert(sizeof(TaskDesc) == 16, "TaskDesc must stay 16 bytes");

int build_graph(uint32_t ntasks, const spx_access* acc, uint64_t nacc, const int32_t* priority, Graph& g);
// potrf_steps > 1: each POTRF(k) becomes that many chained step tasks (TaskDesc.pad =
// step | (potrf_steps << 8)); the device splits the diagonal factorization at 32 columns
// per step, so potrf_steps must be b / 32.
// commute (every program): the updates are commutative writes.
void cholesky_program(int nt, bool with_solve, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc,
                      bool with_inverse = false, int potrf_steps = 1, bool commute = false);
void solve_program(int nt, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc, bool commute = false);
// The tiled matrix product C += A B (k outermost, then i, then j).
void gemm_program(int nt, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc, bool commute = false);
// Sets g.prio to the upward-rank priorities of the program's tasks.
void rank_priorities(const std::vector<TaskDesc>& tasks, Graph& g);
// LOAD, the factor program (and with_solve: the substitution), STORE (with_solve only);
// with_inverse: the inversion tasks and the inverse-based substitution.
void io_program(int nt, bool with_solve, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc,
                bool with_inverse, int potrf_steps = 1, bool commute = false);
// LOAD of the right-hand sides only (TaskDesc.j = 1), the substitution, STORE.
void solve_io_program(int nt, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc, bool commute = false);

// ---------------------------------------------------------------------------------------
// Device-side descriptors (plain data, copied to the GPU).
// ---------------------------------------------------------------------------------------

enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2 };

// One matrix being factored / solved.  Tile (i,j), i >= j, of the lower triangle is
// stored contiguously, column-major, at tiles + (i(i+1)/2 + j) b^2.
struct DevMat {
  double* tiles;
  void* low;        // low-precision copies of the off-diagonal tiles (same packing), or null
  double* rhs;      // right-hand side / solution, column-major n_pad x nrhs (ld = n_pad)
  double* rhs2;     // second copy written by the diagonal solves (same layout)
  double* dinv;     // inverses of the 32x32 diagonal blocks of each diagonal tile (32 b per tile)
  double* minv;     // M_k = L_kk^{-T} per diagonal tile (b x b, column-major, upper triangular)
  int32_t* info;    // 0x7fffffff while healthy; else the 1-based failing column
  int64_t n_pad;
  int32_t nt, b, nrhs, prec;
  int32_t n, trsm_rows;
  int32_t store_acc;  // STORE adds the solution to X instead of overwriting it
  int32_t load_live;  // LOAD packs only the live lower 64x64 blocks of the matrix's one tile
                      // (a one-shot solve: nothing reads the upper triangle or the padding)
  // caller's dense arrays, used by the LOAD / STORE tasks of batched and served graphs
  const double* dscale;  // packing: A(i,j) d_i d_j (+ shift on the diagonal), or null
  double shift;
  const double* A;  // n x n row-major, lower triangle read
  const double* B;  // n x nrhs row-major
  double* X;        // n x nrhs row-major
  int64_t lda, ldb, ldx;
  // tiled matrix product: A tiles and B^T tiles (all nt x nt, tile (i,j) at (i nt + j) b^2,
  // column-major); C tiles in `tiles` with the same layout
  const double* ga;
  const double* gbt;
  unsigned long long spin_ticks;  // SPX_T_SPIN: device clock ticks each task waits
  // set to 1 (system scope) when the matrix's STORE has been released: its X is final in
  // device memory (host-visible flag of the serving loop), or null
  unsigned int* done_flag;
};

// A LOAD task has one part per lower tile while they fit the 16-bit part index.
constexpr int kLoadTileParts = 65534;
constexpr int kMaxQueues = 64;      // ready queues per image: levels x shards (one per lane of a wave)
constexpr int kMaxLevels = 64;      // priority classes (priority >> 16)
constexpr int kLevels1 = 16;        // queue levels with one shard
constexpr int kLevelsMax = 32;      // most levels any policy uses (2 shards x 32 levels)
constexpr int kShards = 8;          // ready queues per priority level (one per XCD-sized group of workgroups)
constexpr int kCounterStride = 32;  // 128-byte spacing of hot counters (uint32 units)
// Counter layout: one 64-bit word per queue q = level x shards + shard (head in the low
// half, tail in the high half, so one load reads both and one compare-and-swap claims
// against both), then the status word.
constexpr uint32_t ctr_queue_idx(int q) { return (uint32_t)q * kCounterStride; }
constexpr uint32_t kStatusIdx = (uint32_t)kMaxQueues * kCounterStride;
// Per XCD x (kXcds of them): the tail and head of its ring of finished, not yet released
// parts, and the lock of its release rounds, each on its own line.
constexpr int kXcds = 8;
constexpr uint32_t ctr_ring_tail_idx(int x) { return kStatusIdx + (uint32_t)(1 + 3 * x) * kCounterStride; }
constexpr uint32_t ctr_ring_head_idx(int x) { return kStatusIdx + (uint32_t)(2 + 3 * x) * kCounterStride; }
constexpr uint32_t ctr_ring_lock_idx(int x) { return kStatusIdx + (uint32_t)(3 + 3 * x) * kCounterStride; }
constexpr uint32_t kNumCounters = kStatusIdx + (uint32_t)(1 + 3 * kXcds) * kCounterStride;

// Everything the persistent scheduler kernel needs for one launch.
struct SchedArgs {
  const TaskDesc* tasks;
  const uint32_t* succ_off;  // ntasks + 1
  const uint32_t* succ;
  uint32_t* pending;         // remaining predecessors per task
  uint32_t* parts_left;      // parts not yet finished per task
  unsigned long long* queue; // item = task << 16 | part; queue (l, s) holds qcap[l] slots
                             // at qbase[l] * kShards + s * qcap[l]
  uint32_t* counters;        // ctr_queue_idx / kStatusIdx / ctr_ring_*_idx
  uint32_t* ring;            // per XCD x: ring_cap task ids at x * ring_cap (finished parts awaiting release)
  uint32_t ring_cap;
  // commutative-write groups (coff null without them; layout as in Graph): a task with
  // commutative accesses takes its groups' locks, in group order, once it is ready, and
  // is pushed when it holds all of them
  const uint32_t* coff;
  const uint32_t* cent;
  const uint32_t* goff;
  const uint32_t* gtask;
  const uint32_t* gidx;
  unsigned long long* gstate;  // per group: lock bit 63, waiting members' bits 0..62
  const uint32_t* croots;      // root tasks with commutative accesses (take their locks at the start)
  uint32_t ncroots;
  uint32_t qbase[kLevelsMax];
  uint32_t qcap[kLevelsMax];
  uint32_t total_parts;
  uint32_t max_claim;  // parts one pop may claim outside the bulk levels (1 or 4)
  uint32_t spread_max;  // a task of at most this many parts deals them over the shards (0: none)
  uint32_t ntasks;
  int32_t nlev;     // levels in use (nlev x nshards <= kMaxQueues)
  int32_t nshards;  // queues in use per level (1..kShards); the image's roots use the same count
  const DevMat* mats;
  unsigned long long* trace;  // 4 x uint64 per part, or null
  uint32_t* trace_idx;
  unsigned long long* trace_push;  // per task: the tick its last predecessor pushed it, or null
  unsigned long long* wg_cycles;  // per workgroup: busy, idle (wall clock ticks)
  unsigned long long spin_limit;  // ticks without progress before giving up
};

enum { STATUS_TIMEOUT = 1u };

// Host-side launchers (spx_kernels.hip).
int launch_pack(const double* dA, int64_t lda, int64_t n, const DevMat& m, void* stream);
int launch_unpack(const DevMat& m, int64_t n, double* dL, int64_t ldl, void* stream);
// Dense row-major n x n (ld) <-> all nt x nt tiles of size b (tile (i,j) at (i nt + j) b^2,
// column-major), zero padding; trans: the tiles of the transpose.
int launch_pack_full(const double* src, int64_t ld, int64_t n, double* tiles, int b, int nt, int trans, void* stream);
int launch_unpack_full(const double* tiles, int b, int nt, int64_t n, double* dst, int64_t ld, void* stream);
// scale (nullable): row r is multiplied by scale[r] on the way in / out.
int launch_rhs_in(const double* dB, int64_t ldb, int64_t n, int64_t nrhs, double* rhs, int64_t n_pad,
                  const double* scale, void* stream);
int launch_rhs_out(const double* rhs, int64_t n_pad, int64_t n, int64_t nrhs, double* dX, int64_t ldx, int accumulate,
                   const double* scale, void* stream);
// d[i] = 1 / sqrt(A(i,i)) for i < n, 1 for n <= i < n_pad.
int launch_diag_scale(const double* dA, int64_t lda, int64_t n, double* d, int64_t n_pad, void* stream);
// Column sums of U .* V (n x q row-major, ld q), deterministic: partial[g] for g < nthreads
// (nthreads returned, a multiple of q); the host adds partial[c], partial[c + q], ... in order.
int launch_dot_cols(int64_t n, int64_t q, const double* U, const double* V, double* partial, int* nthreads,
                    void* stream);
// mode 0: Y += alpha_c X;  mode 1: Y = X + alpha_c Y  (n x q row-major, alpha: q on the device).
int launch_axpy_cols(int64_t n, int64_t q, const double* alpha, const double* X, double* Y, int mode, void* stream);
// roots: nroots pairs (queue slot, item) written after the queue is cleared.
int launch_sched_init_full(uint32_t* pending, const uint32_t* indeg, uint32_t* parts_left, const uint32_t* nparts,
                           uint32_t ntasks, unsigned long long* queue, uint32_t queue_len,
                           const unsigned long long* roots, uint32_t nroots, uint32_t* counters,
                           const uint32_t* counters0, uint32_t ncounters, uint32_t* ring, uint32_t ring_len,
                           unsigned long long* gstate, uint32_t ngroups, int32_t* info, int ninfo,
                           uint32_t* trace_idx, void* stream);
// Task families of the scheduler kernel (one instantiation each): FAM_CHOL runs every
// task of the Cholesky, solve, batched and served graphs; FAM_GEMM the tiled product's;
// FAM_SPIN the empty tasks of spx_run_graph.
enum { FAM_CHOL = 0, FAM_GEMM = 1, FAM_SPIN = 2 };
int launch_sched(const SchedArgs& a, int num_wg, void* stream, int family = FAM_CHOL);
int launch_one_task(const SchedArgs& a, int nparts, void* stream);
int launch_tile_inverses(const double* l, int b, double* dinv, void* stream);
uint16_t parts_of(const TaskDesc& d, int b, int nrhs);
int sched_max_wg(int device, int* per_cu, int* num_cu);
int launch_spd_fill(double* A, int64_t n, uint32_t seed, void* stream);
// Residuals of many systems in one launch: row block blk of matrix m for prefix[m] <=
// blk < prefix[m+1] (prefix: count + 1 entries, device).
struct ResDesc {
  int64_t n, lda, nrhs, ldx, ldb;
  const double* A;
  const double* X;
  const double* B;
  double* R;      // n x nrhs row-major
  double* stats;  // 3 nrhs + 1, cleared by the caller
};
int launch_backward_error_batched(const ResDesc* d, const uint32_t* prefix, int count, uint32_t nblocks, void* stream);
int launch_backward_error(int64_t n, const double* dA, int64_t lda, int64_t nrhs, const double* dX, int64_t ldx,
                          const double* dB, int64_t ldb, double* dR, double* dstats, void* stream);

// Scratch array of the allocation-free entry point (a file-scope device array in
// spx_kernels.hip, one copy per GPU).  scratch_init looks up the calling thread's current
// device's copy (once per device; `device` must be current); scratch_get returns it.
constexpr size_t kScratchBytes = 32ull << 20;
int scratch_init(int device);
int scratch_get(int device, void** ptr);

// Context internals the serving loop needs.
int ctx_device(const spx_ctx* c);
// Per-matrix completion flags (device-visible pointers, one per matrix, entries may be
// null) for the next batched solve on the context; null clears them.
void ctx_set_store_flags(spx_ctx* c, unsigned int* const* flags);
int ctx_copy_tile_tables(const spx_ctx* from, spx_ctx* to);

}  // namespace spx

struct spx_graph {
  spx::Graph g;
  std::vector<spx::TaskDesc> tasks;
};
