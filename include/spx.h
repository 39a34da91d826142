/*
 * spx.h - C ABI of libspx: tile-DAG Cholesky factorisation and solve on one MI355X.
 *
 * Method (Specx, arXiv 2308.15964):
 *   Sec. 2.1 / Sec. 4.1  sequential task flow: tasks are inserted in program order with
 *                        read (SpRead) or read-write (SpWrite) accesses to data; the
 *                        dependencies follow from that order, and any parallel execution
 *                        must give the sequential result.
 *   Sec. 4.1             priorities the scheduler may use; the user keeps data alive until
 *                        the tasks using it are done; a task viewer can wait on a task.
 *   Sec. 4.5             scheduler with push (a task became ready) and pop (an idle worker
 *                        asks for work, possibly getting none).
 *   Sec. 4.7             per-datum ordered task lists whose progress releases successors.
 *   Sec. 4.8             DOT export of the task graph, traces and idle time.
 *   Sec. 5.2             tiled Cholesky as POTRF / TRSM / SYRK / GEMM tasks in FP64.
 *
 * Conventions for every call:
 *   - Return value: SPX_OK (0); a positive value only where stated (LAPACK-style info);
 *     a negative SPX_E* code on error.  No C++ exception crosses the ABI.  After an error,
 *     spx_last_error() returns a message for the calling thread.
 *   - "device pointer" = memory of the context's GPU (e.g. from torch); "host pointer" =
 *     ordinary or pinned host memory.  Every buffer passed in is owned by the caller, who
 *     keeps it alive and unmodified until the call returns (or, for spx_submit, until
 *     spx_poll reports the request done).  Handles (graph, factor, server, context) are
 *     owned by the library and freed only by their destroy call.
 *   - Dense matrices are row-major with a leading dimension (elements between rows);
 *     only the lower triangle (row >= column) of a symmetric input is read.
 *   - Every GPU call is issued on the context's stream.
 */
#ifndef SPX_H
#define SPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SPX_OK = 0,
  SPX_EINVAL = -1,   /* null/invalid argument, unsupported size or option */
  SPX_ENOMEM = -2,   /* allocation failed, or a request can never fit the budget */
  SPX_EDEVICE = -3,  /* a HIP call failed */
  SPX_EAGAIN = -4,   /* not finished yet (spx_poll) / no capacity right now */
  SPX_EABORT = -5,   /* the run was aborted by the host */
  SPX_ETIMEOUT = -6  /* the device scheduler saw no progress within its spin limit */
};

/* Access modes (Sec. 4.1): SpRead, SpWrite (read or write) and SpCommutativeWrite
 * (Sec. 4.1, Sec. 4.7): a read-modify-write whose order among the commutative writes of
 * the same datum inserted one after another does not matter.  Such a run (cut into groups
 * of at most 63 consecutive commutative writes) needs the datum's state before it, the
 * next other access needs all of it, and its members run one at a time in any order: the
 * device scheduler takes a lock per group when a member becomes ready and hands it to the
 * next ready member when the holder finishes. */
enum { SPX_ACC_R = 1, SPX_ACC_RW = 2, SPX_ACC_CW = 3 };

/* One declared access: task index (insertion order), mode, datum id.  Accesses are given
 * grouped by task in insertion order; a task may name a datum twice (the same mode twice
 * counts once; two different modes count as SPX_ACC_RW). */
typedef struct {
  uint32_t task;
  uint32_t mode;
  uint64_t datum;
} spx_access;

typedef struct spx_ctx spx_ctx;
typedef struct spx_graph spx_graph;
typedef struct spx_factor spx_factor;
typedef struct spx_server spx_server;

const char* spx_last_error(void);

/* ---------------------------------------------------------------------------------------
 * Context: device, stream and (optionally) the caller's allocator.
 *   device: HIP device ordinal.  hip_stream: a hipStream_t (NULL = the null stream).
 *   alloc/free: nullable; if given, every device allocation of the library goes through
 *   them (e.g. torch's caching allocator) with the context's stream and `user`.
 *   Errors: SPX_EINVAL (bad device), SPX_EDEVICE.
 * ------------------------------------------------------------------------------------ */
typedef void* (*spx_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*spx_free_fn)(void* ptr, void* stream, void* user);
int spx_ctx_create(int device, void* hip_stream, spx_alloc_fn alloc, spx_free_fn free_fn, void* user,
                   spx_ctx** out);
void spx_ctx_destroy(spx_ctx* ctx);

/* ---------------------------------------------------------------------------------------
 * Graph building (Sec. 2.1, Sec. 4.1, Sec. 4.7).  Host only, integer only.
 *   spx_graph_build: infers the immediate-dependency edges of ntasks tasks from their
 *   accesses: a read depends on the datum's last writer (RAW); a write depends on every
 *   read since the last write (WAR), or on the last writer if there was none (WAW); a
 *   commutative write depends on what a write would at the start of its group, and the
 *   access after a group on all of its members ("last writer" then means every member).
 *   Edges are deduplicated and always point from an earlier to a later task, so the graph
 *   is acyclic.  priority (nullable, ntasks entries): larger runs sooner (Sec. 4.1).
 *   Errors: SPX_EINVAL (task index >= ntasks, bad mode, accesses not grouped by task in
 *   increasing order), SPX_ENOMEM.
 * ------------------------------------------------------------------------------------ */
int spx_graph_build(uint32_t ntasks, const spx_access* acc, uint64_t nacc, const int32_t* priority,
                    spx_graph** out);
int spx_graph_info(const spx_graph* g, uint32_t* ntasks, uint64_t* nedges);
/* Edges sorted by (src, dst); cap = capacity of src/dst.  SPX_EINVAL if cap < nedges. */
int spx_graph_edges(const spx_graph* g, uint32_t* src, uint32_t* dst, uint64_t cap);
int spx_graph_indegree(const spx_graph* g, uint32_t* indeg, uint32_t cap);
/* Writes the graph in graphviz DOT form (Sec. 4.8) to `path`.  SPX_EINVAL if unwritable. */
int spx_graph_to_dot(const spx_graph* g, const char* path);
void spx_graph_destroy(spx_graph* g);


/* The task program the factorisation (and, with with_solve bit 0, the block forward and
 * backward substitution) inserts for nt x nt tiles, built with spx_graph_build: right-
 * looking, lower triangle; for k: POTRF(k); TRSM(i,k) i>k; SYRK(i,k) and GEMM(i,j,k)
 * k<j<i.  with_solve bit 1 adds the LOAD task in front (and, with bit 0, STORE at the end)
 * as the batched calls run it; bit 2 appends INV(k) for every k after the factor tasks and
 * makes the substitution use M_k with a second right-hand-side copy (as the library runs
 * every graph whose factor is kept; one-shot batched solves use the in-place program).  Datum ids: tile (i,j) -> i*nt + j,
 * right-hand-side block k -> nt*nt + k, M_k -> nt*nt + nt + k.  task_types (nullable,
 * ntasks entries) receives SPX_T_* codes. */
enum { SPX_T_POTRF = 0, SPX_T_TRSM, SPX_T_SYRK, SPX_T_GEMM, SPX_T_FTRSM, SPX_T_FGEMM, SPX_T_BTRSM, SPX_T_BGEMM,
       SPX_T_LOAD, SPX_T_STORE, SPX_T_INV, SPX_T_MGEMM, SPX_T_SPIN };
/* SPX_T_LOAD / SPX_T_STORE appear only in the graphs of the batched and served calls: the
 * first task of each matrix copies its dense input (and right-hand sides) into tile
 * storage, writing every tile; the last one reads the solution blocks and writes X.
 * SPX_T_INV(k), appended after the factor tasks of the graphs the library runs (with_solve
 * bit 2 here), reads the factored diagonal tile L_kk and writes M_k = L_kk^{-T}; the
 * diagonal solves FTRSM(k) / BTRSM(k) then read M_k instead of L_kk.  Bits 8-15 of
 * with_solve (0 or 1: whole tasks; at most 64): each POTRF(k) becomes that many chained
 * step tasks on tile (k,k), as the library runs the diagonal tiles of 256 and 512 in
 * matrices of at least four tile columns (b/32 steps).  Bit 3: the updates (SYRK and GEMM
 * on their tile, FGEMM and BGEMM on their right-hand-side block) are commutative writes,
 * as SPX_F_COMMUTE runs them. */
int spx_cholesky_graph(int32_t nt, int32_t with_solve, spx_graph** out, int32_t* task_types, uint32_t cap);

/* The tiled matrix product of Sec. 5.2 (the GEMM application) for nt x nt tiles: one task
 * SPX_T_MGEMM(i, j, k) per tile triple, C_ij <- C_ij + A_ik B_kj, declaring SpRead on A_ik
 * and B_kj and SpWrite on C_ij, inserted with k outermost (then i, then j).  Datum ids:
 * A_ik -> i*nt + k, B_kj -> nt^2 + k*nt + j, C_ij -> 2 nt^2 + i*nt + j.  The graph is nt^2
 * independent chains of nt - 1 write-after-write edges.  nt | SPX_GEMM_COMMUTE: the
 * updates of C_ij are commutative writes instead (no edges; groups of at most 63 updates
 * of a tile, run one at a time in any order), as SPX_F_COMMUTE runs them.  task_types as
 * for spx_cholesky_graph.  Errors: SPX_EINVAL (nt outside [1, 512]), SPX_ENOMEM. */
enum { SPX_GEMM_COMMUTE = 1 << 16 };
int spx_gemm_graph(int32_t nt, spx_graph** out, int32_t* task_types, uint32_t cap);

/* ---------------------------------------------------------------------------------------
 * Factorisation (Sec. 5.2).
 *   tile: tile size b (32, 64, 128, 256 or 512; 0 = chosen from n).  n is padded to a
 *     multiple of b with an identity diagonal (exact: the padding adds only exact zeros).
 *   update_prec: SPX_PREC_FP64 (all tasks FP64), SPX_PREC_FP32 or SPX_PREC_BF16 (SYRK and
 *     GEMM read FP32 / BF16 copies of the panel tiles and accumulate in FP32 on the matrix
 *     cores; POTRF and TRSM stay FP64; the factor is stored in FP64).
 *   queue_policy: the ready queues.  Tasks carry upward-rank priorities (the longest
 *     chain of work from the task to the end of the graph): the panel chain first, then
 *     the updates by how soon their tile is consumed.  SPX_Q_SHARDED (the default, 0):
 *     sixteen priority levels, each split into 4 queues (shards), one per pair of XCDs; a
 *     task is pushed into the shard of the XCD that released its last predecessor (the
 *     j-th successor of one finished task into the j-th shard after it, and in a launch of
 *     one graph the parts of a task of at most 8 parts, or a substitution task of at most
 *     16, dealt over the shards), and a
 *     workgroup serves the highest non-empty level, its own shard first, so pops spread
 *     over 4 queue heads per level (environment SPX_QUEUE_SHARDS = 2, 4 or 8 trades
 *     shards for levels: 32, 16 or 8 levels).  This split, and pops that claim up to 4
 *     parts from a long queue, apply to one graph whose tasks average at least two parts;
 *     batched launches and graphs of single-part tasks use 8 shards of 8 levels and
 *     single claims.
 *     SPX_Q_PRIORITY: sixteen
 *     levels, one queue each (exact push order within a level; every pop contends for one
 *     queue head, which limits pops to about one per microsecond).  SPX_Q_FIFO: one queue
 *     in push order.  Results are bitwise identical under every policy.
 *   num_wg: persistent workgroups (0 = fill the GPU).
 *   flags: SPX_F_TRACE records per-task device timestamps (spx_trace).
 *     SPX_F_SCALED factors D^{-1/2} A D^{-1/2} + shift I instead of A (D = diag(A)):
 *     a stabilised low-precision factor that spx_potrs uses as a preconditioner (the
 *     factor keeps D^{-1/2} and applies it around every solve).  spx_factor_get_l then
 *     returns the factor of the scaled, shifted matrix.  Single-matrix calls only.
 *     SPX_F_COMMUTE declares the updates as commutative writes (Sec. 4.1): SYRK and GEMM
 *     on their tile in the factor, FGEMM and BGEMM on their right-hand-side block in the
 *     solve (spx_potrs with a factor made under the flag), MGEMM on C_ij in
 *     spx_gemm_tiled.  The updates of a tile then run in the order they become ready, one
 *     at a time, instead of in insertion order: the result changes by rounding from
 *     launch to launch (no longer bitwise reproducible) and stays within the same error
 *     bounds.  Single-matrix calls only.
 * ------------------------------------------------------------------------------------ */
enum { SPX_PREC_FP64 = 0, SPX_PREC_FP32 = 1, SPX_PREC_BF16 = 2 };
enum { SPX_Q_SHARDED = 0, SPX_Q_PRIORITY = 1, SPX_Q_FIFO = 2 };
enum { SPX_F_TRACE = 1u, SPX_F_SCALED = 2u, SPX_F_COMMUTE = 4u };
typedef struct {
  int32_t tile;
  int32_t update_prec;
  int32_t queue_policy;
  int32_t num_wg;
  uint32_t flags;
  int32_t pad;
  double shift; /* with SPX_F_SCALED only */
} spx_opts;

/* Factors the n x n SPD matrix dA (device pointer, row-major, leading dimension lda >= n,
 * lower triangle read, never written).  The factor is kept in library-owned tile storage
 * on the device; *out receives its handle.  *info: 0, or the 1-based global column whose
 * leading minor is not positive definite (the factor is then discarded and *out is NULL).
 * opts nullable (defaults).  The call returns after the device has finished.
 * Errors: SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE, SPX_ETIMEOUT. */
int spx_potrf_tiled(spx_ctx* ctx, int64_t n, const double* dA, int64_t lda, const spx_opts* opts,
                    spx_factor** out, int64_t* info);

/* Size, tile and padded size of a factor. */
int spx_factor_info(const spx_factor* f, int64_t* n, int32_t* tile, int64_t* n_padded);
/* Writes L (n x n, row-major, device pointer, leading dimension ldl >= n) with zeros above
 * the diagonal. */
int spx_factor_get_l(spx_ctx* ctx, const spx_factor* f, double* dL, int64_t ldl);
void spx_factor_destroy(spx_factor* f);

/* C <- C + A B for n x n matrices (Sec. 5.2, the GEMM application), run as the task graph of
 * spx_gemm_graph by the device scheduler in one persistent launch, in FP64.  dA, dB, dC:
 * device pointers, row-major with leading dimensions lda, ldb, ldc >= n; A and B are only
 * read; C is read and overwritten and may not overlap A or B.  The matrices are copied into
 * library tile storage for the call (A and C as b x b column-major tiles, B as the tiles of
 * B^T; n padded to a multiple of b with zeros, which add exact zeros) and C back out.
 * opts (nullable; NULL means sharded queues and the defaults below): tile (32..512; 0 =
 * chosen from n), queue_policy (SPX_Q_SHARDED suits this graph: nt^2 independent chains,
 * whose pops would otherwise serialise on one queue head), num_wg, flags (SPX_F_TRACE);
 * update_prec must be SPX_PREC_FP64.  Each task's b x b update runs as
 * 128 x 128 parts on the matrix cores; every C_ij takes its k terms in increasing k, so the
 * result does not depend on the schedule.  spx_last_stats reports the launch (pack_ms: the
 * three packs).  Errors: SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE, SPX_ETIMEOUT. */
int spx_gemm_tiled(spx_ctx* ctx, int64_t n, const double* dA, int64_t lda, const double* dB, int64_t ldb, double* dC,
                   int64_t ldc, const spx_opts* opts);

/* Runs a graph built by spx_graph_build on the device scheduler with every task an empty
 * task (SPX_T_SPIN) that keeps its workgroup busy for spin_ticks ticks of the device's
 * 100 MHz wall clock: the device form of the runtime-overhead study of Sec. 5.1 (a task
 * body that only waits a duration D, so the launch time minus the waiting measures what
 * the runtime adds per task).  The graph's edges and priorities are used as for any
 * launch; each task is one part (one workgroup).  opts (nullable; NULL means sharded
 * queues): queue_policy, num_wg, flags (SPX_F_TRACE); the other fields are ignored.  spx_last_stats reports the launch.
 * spin_ticks <= 10^9 (10 s).  Errors: SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE, SPX_ETIMEOUT. */
int spx_run_graph(spx_ctx* ctx, const spx_graph* g, uint64_t spin_ticks, const spx_opts* opts);

/* ---------------------------------------------------------------------------------------
 * Solve A X = B with the factor (Sec. 5.2 task style: block forward and backward
 * substitution run as a task graph by the same device scheduler).
 *   dB, dX: device pointers, n x nrhs row-major with leading dimensions ldb, ldx >= nrhs;
 *   dB is not written; dX may equal dB only if ldx == ldb.
 *   refine (nullable): iterative refinement in FP64 against the original matrix until the
 *   largest normwise backward error of the columns is <= tol, or max_iter corrections:
 *   method 0 = none, 1 = classical refinement (r = b - A x in FP64 with the original
 *   matrix, x += solve(L, r)), stopping early after two steps that fail to halve the
 *   error; 2 = preconditioned conjugate gradients in FP64 on A with the factor as the
 *   preconditioner (every column its own recurrence; the true residual b - A x is
 *   recomputed each iteration; stops after 10 iterations without a new best error).  A
 *   factor made with SPX_F_SCALED is applied as D^{-1/2} (L L^T)^{-1} D^{-1/2}.  Refinement needs the original matrix: pass it in dA (device, row-major, lda);
 *   the caller keeps it alive and unmodified during the call; dX must not alias dB.
 *   tol <= 0 means 1e-12, max_iter <= 0 means 50.
 *   stats (nullable) receives the number of corrections and the final largest backward
 *   error (-1 when not refining).
 * Errors: SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE, SPX_ETIMEOUT. */
typedef struct {
  double tol;
  int32_t max_iter;
  int32_t method;
  int32_t x_init; /* nonzero: dX already holds a first solution (skip the initial solve) */
  int32_t pad;
} spx_refine;
typedef struct {
  int32_t iters;
  int32_t method_used;
  double eta_max;
} spx_solve_stats;
int spx_potrs(spx_ctx* ctx, const spx_factor* f, int64_t nrhs, const double* dB, int64_t ldb, double* dX,
              int64_t ldx, const double* dA, int64_t lda, const spx_refine* refine, spx_solve_stats* stats);

/* Allocation-free solve, for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * X = A^{-1} B through the factor f, with the same task graph, kernels and results (bit for
 * bit) as spx_potrs without refinement.  It calls no hipMalloc, hipFree or allocating
 * library routine: the graph image, the matrix descriptor, the info word and the two
 * right-hand-side work copies live in a static device array of the library, 32 MiB per
 * GPU (kept until the process ends), whose address is looked up once per device by
 * spx_ctx_create.  dB, dX, ldb, ldx as for spx_potrs (dX may equal dB only if ldx == ldb).
 * Every call on one GPU uses that GPU's one array and leaves its contents behind (each
 * call rewrites what it reads), so calls that overlap on one GPU (other host threads, other
 * contexts or streams) race: the caller serialises them.
 * Errors: SPX_EINVAL (bad arguments, or a solve that needs more than the 32 MiB: about
 * 2 n nrhs doubles plus the graph image), SPX_EDEVICE, SPX_ETIMEOUT. */
int spx_potrs_noalloc(spx_ctx* ctx, const spx_factor* f, int64_t nrhs, const double* dB, int64_t ldb, double* dX,
                      int64_t ldx);

/* Normwise backward errors eta_q = ||b_q - A x_q||_inf / (||A||_inf ||x_q||_inf +
 * ||b_q||_inf), computed on the device in FP64 (row-major device pointers as above);
 * eta: host array of nrhs doubles. */
int spx_backward_error(spx_ctx* ctx, int64_t n, const double* dA, int64_t lda, int64_t nrhs, const double* dX,
                       int64_t ldx, const double* dB, int64_t ldb, double* eta);

/* ---------------------------------------------------------------------------------------
 * One task of the Cholesky / solve program (task types SPX_T_*, tile indices i, j, k as
 * spx_cholesky_graph inserts them) run on caller-owned device storage, all of its parts
 * in parallel: for tests of the tile kernels.
 *   d_tiles: the lower tiles of an nt x nt tile matrix, tile (i,j), i >= j, b x b column-
 *   major at d_tiles + (i(i+1)/2 + j) b^2 (device pointer).  d_rhs (nullable unless the
 *   task is a solve task): nt*b x nrhs column-major.  *info: 0 or the 1-based global
 *   column of a failed pivot (POTRF).  Errors: SPX_EINVAL (bad type, index or tile size).
 * ------------------------------------------------------------------------------------ */
int spx_run_task(spx_ctx* ctx, int32_t type, int32_t i, int32_t j, int32_t k, int32_t nt, int32_t b,
                 double* d_tiles, double* d_rhs, int32_t nrhs, int64_t* info);

/* ---------------------------------------------------------------------------------------
 * Batched factorisation and solve: many independent matrices in ONE persistent launch
 * (Sec. 4.1: one engine runs several task graphs).  Each matrix contributes its own task
 * graph (LOAD, the factor program, for spx_posv_batched the block substitution, STORE);
 * the graphs are concatenated into one device image with no edges between matrices, so
 * workgroups move freely between matrices while every matrix keeps its own dependency
 * order.  Results are bitwise identical to spx_potrf_tiled / spx_potrs on each matrix with
 * the same tile size.
 *   count: number of matrices (1..1<<20).  n, lda, nrhs, ldb, ldx: host arrays of count
 *   entries.  dA, dB, dX: host arrays of count device pointers (row-major, as for the
 *   single-matrix calls; dA and dB are read only; dX may not alias dB).
 *   opts: tile > 0 forces one tile size for every matrix; tile <= 0 takes each matrix's
 *   tile from the context's tile table for opts->update_prec (spx_set_tile_table or
 *   spx_autotune_batched), else from a size rule.  update_prec as for spx_potrf_tiled
 *   (no refinement here: the FP32 / BF16 runs report the backward error they reach).
 *   info: host array of count entries: 0, or the 1-based failing column of that matrix
 *   (its X is then not written).  A failure of one matrix does not stop the others.
 *   spx_potrf_batched returns one factor handle per matrix in out (NULL where info > 0),
 *   usable with spx_potrs and spx_factor_get_l; spx_posv_batched returns them in keep when
 *   keep is not NULL (count entries), else keeps none (one workspace for the batch).
 * Errors: SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE, SPX_ETIMEOUT. */
int spx_posv_batched(spx_ctx* ctx, int32_t count, const int64_t* n, const double* const* dA, const int64_t* lda,
                     const int64_t* nrhs, const double* const* dB, const int64_t* ldb, double* const* dX,
                     const int64_t* ldx, const spx_opts* opts, int64_t* info, spx_factor** keep);
int spx_potrf_batched(spx_ctx* ctx, int32_t count, const int64_t* n, const double* const* dA, const int64_t* lda,
                      const spx_opts* opts, spx_factor** out, int64_t* info);

/* Batched solves with existing factors (one launch per sweep over all systems): X_m =
 * A_m^{-1} B_m through f[m].  refine (nullable) as for spx_potrs: with method 1 every
 * refinement step is one batched residual launch over the systems not yet converged and
 * one batched solve launch adding the corrections.  dA/lda (nullable unless refining):
 * the original matrices; when given, stats[m].eta_max receives the final backward error
 * of system m (else -1).  stats: count entries or NULL.  X_m must not alias B_m. */
int spx_potrs_batched(spx_ctx* ctx, int32_t count, spx_factor* const* f, const int64_t* nrhs,
                      const double* const* dB, const int64_t* ldb, double* const* dX, const int64_t* ldx,
                      const double* const* dA, const int64_t* lda, const spx_refine* refine,
                      spx_solve_stats* stats);
/* Largest normwise backward error of each system (one launch): eta_max host array. */
int spx_backward_error_batched(spx_ctx* ctx, int32_t count, const int64_t* n, const double* const* dA,
                               const int64_t* lda, const int64_t* nrhs, const double* const* dX,
                               const int64_t* ldx, const double* const* dB, const int64_t* ldb,
                               double* eta_max);

/* Tile table of the context for update precision prec: a matrix of size n takes the tile
 * of the first entry with n <= n_max[i] (n_max increasing); above the last entry, and
 * with no table, a size rule applies (32 below 128, 64 below 512, 128 below 2048, 256
 * below 8192, else 512).
 * count 0 clears the table (the size rule applies again).  tile[i] in {32,...,512}. */
int spx_set_tile_table(spx_ctx* ctx, int32_t prec, int32_t count, const int64_t* n_max, const int32_t* tile);
/* Tile the context would use for a matrix of size n at precision prec. */
int spx_tile_for(const spx_ctx* ctx, int32_t prec, int64_t n, int32_t* tile);

/* Autotuner: for each probe size sizes[i] (increasing), times spx_posv_batched on `copies`
 * synthetic diagonally dominant SPD matrices of that size with nrhs right-hand sides, for
 * every candidate tile in {32, 64, 128, 256, 512} not above the size rounded up to a power
 * of two, and keeps the fastest (best kernel time of `reps` launches after one warm-up).
 * best_tile: count entries; ms (nullable): nsizes x 5 kernel times in candidate order (0
 * for a skipped candidate).  The result becomes the context's tile table for prec, with
 * n_max = sizes; the caller may persist it and restore it with spx_set_tile_table. */
int spx_autotune_batched(spx_ctx* ctx, int32_t prec, int32_t nsizes, const int64_t* sizes, int32_t nrhs,
                         int32_t copies, int32_t reps, int32_t* best_tile, double* ms);

/* ---------------------------------------------------------------------------------------
 * Serving: SPD solve requests of mixed sizes, admitted by an HBM budget and run with
 * continuous batching.  The server owns `lanes` worker threads, each with its own HIP
 * stream and context.  Admission is first-fit over the queue of waiting requests in
 * arrival order (a request that does not fit yet does not block smaller ones behind it)
 * against the byte budget (factor tiles, block inverses, low-precision copies, right-hand
 * side work arrays, and device copies of host inputs).  An idle lane takes every admitted
 * request of one mode (and, for mixed, one tolerance; up to max_batch) and runs them as ONE
 * batched launch (mixed: one factor launch, then one residual and one solve launch per
 * refinement sweep over the systems not yet converged); requests that
 * arrive meanwhile are admitted as memory frees up and start on the next idle lane, so
 * their work overlaps on the device with the batches already running.
 *   mode SPX_MODE_FP64: FP64 factor + solve (spx_posv_batched), then the backward error.
 *   mode SPX_MODE_MIXED: FP32-update factor (spx_potrf_batched), then FP64 classical
 *   iterative refinement to tol (spx_potrs_batched method 1); a request whose low-precision
 *   factor breaks down or whose refinement does not reach tol is redone in FP64
 *   (method_used = 0 reports the fallback).  Requests with n < opts.mixed_min_n run the
 *   FP64 path directly (method_used = 0): there the updates are too small a share of the
 *   work for FP32 to save what a refinement step costs.
 * The result of a request does not depend on what else is in the same batch or lane: a
 * batched member runs the same kernels in the same dependency order as when alone.
 *   A, B, X: n x n, n x nrhs, n x nrhs row-major with leading dimensions lda, ldb, ldx;
 *   where = 0: host memory (copied in and out by the lane; pinned memory copies faster),
 *   where = 1: device memory of the context's GPU, where = 2: A and B in device memory, X
 *   in host memory (solved into a device copy, then copied back).  The caller keeps them alive and A, B
 *   unmodified until spx_poll returns SPX_OK for the ticket (or the server is destroyed).
 *   tol <= 0 means 1e-12.  tag: returned in the result.
 * spx_submit never blocks: it records the request and returns a ticket; SPX_ENOMEM if the
 * request can never fit the budget; SPX_EINVAL for bad arguments.
 * spx_poll: SPX_OK with *out filled (the ticket is then released), SPX_EAGAIN if not
 * done, SPX_EINVAL for an unknown ticket.  out->status: SPX_OK, SPX_EDEVICE, ... for the
 * request itself; out->info > 0: not positive definite at that column.
 * Times (seconds on the server's steady clock, spx_server_now): submit, admission, start
 * of the launch that ran it, batch finished (t_done: X written back and every diagnostic
 * of the batch done; spx_poll answers from then on), and t_ready: this request's X was
 * final in the caller's memory.  In FP64 mode each request's STORE task, once released,
 * raises a host-visible flag; a monitor thread of the server sees it while the batch is
 * still running and, for host memory, copies X back at once, so t_ready is per request
 * (t_ready <= t_done).  In mixed mode X is final only after the batched refinement:
 * t_ready = t_done.
 * spx_server_destroy: requests not yet started end with status SPX_EABORT; running
 * batches finish first. */
enum { SPX_MODE_FP64 = 0, SPX_MODE_MIXED = 1 };
typedef struct {
  int64_t n, nrhs;
  const double* A;
  const double* B;
  double* X;
  int64_t lda, ldb, ldx;
  int32_t mode;
  int32_t where;
  double tol;
  uint64_t tag;
} spx_request;
typedef struct {
  int32_t status;
  int32_t iters;
  int32_t method_used;
  int32_t tile;
  int64_t info;
  double eta_max;
  double t_submit, t_admit, t_start, t_done;
  uint64_t tag;
  int32_t batch_size;
  int32_t lane;
  double t_ready;
} spx_result;
typedef struct {
  int32_t lanes;      /* worker lanes (streams); <= 0: 2 */
  int32_t max_batch;  /* requests per launch; <= 0: 4096 */
  int32_t num_wg;     /* workgroups per launch; <= 0: fill the GPU */
  int32_t mixed_min_n; /* mixed-mode requests with n below this run in FP64; <= 0: 16384 */
} spx_server_opts;
typedef struct {
  uint64_t submitted, completed, rejected, launches;
  uint64_t bytes_in_use, bytes_peak; /* admitted request bytes (the budget's accounting) */
  uint64_t max_running;  /* most requests running at once over all lanes */
  double busy_s;         /* summed lane busy time */
  uint64_t pool_used_high; /* high-water mark of the device memory pool the lanes allocate
                              from (bytes in use), since the server was created */
} spx_server_stats;
int spx_server_create(spx_ctx* ctx, size_t hbm_budget_bytes, const spx_server_opts* opts, spx_server** out);
int spx_submit(spx_server* s, const spx_request* req, uint64_t* ticket);
int spx_poll(spx_server* s, uint64_t ticket, spx_result* out);
double spx_server_now(const spx_server* s);
int spx_server_get_stats(spx_server* s, spx_server_stats* out);
void spx_server_destroy(spx_server* s);

/* ---------------------------------------------------------------------------------------
 * Run statistics of the last factor or solve launch on the context (Sec. 4.8 idle time).
 * ------------------------------------------------------------------------------------ */
typedef struct {
  double kernel_ms;     /* persistent kernel duration (HIP events on the context stream) */
  double pack_ms;       /* dense -> tile packing */
  double idle_frac;     /* sum of workgroup cycles spent waiting for work / sum of cycles */
  uint32_t ntasks, nparts, num_wg, tile;
  uint64_t device_allocs; /* device allocations the context has made so far (all calls) */
} spx_stats;
int spx_last_stats(const spx_ctx* ctx, spx_stats* out);
/* Context-wide launch flags: SPX_F_TRACE makes every later launch on the context (factor,
 * solve, batched) record its per-part trace, as the flag in spx_opts does for one call.
 * 0 turns it off.  Errors: SPX_EINVAL for other bits. */
int spx_ctx_set_flags(spx_ctx* ctx, uint32_t flags);
/* Per-part trace of the last launch made with SPX_F_TRACE: for part p, rec[4p..4p+3] =
 * {task, part | (workgroup << 16) | (task type << 32), start tick, end tick} (device wall
 * clock, 100 MHz).
 * Returns the record count (or < 0); writes at most cap records. */
int64_t spx_trace(const spx_ctx* ctx, uint64_t* rec, int64_t cap);
/* Push ticks of the same launch: ticks[t] = the device clock when task t's last
 * predecessor pushed it into a ready queue (0 for the graph's roots, pushed before the
 * launch).  With spx_trace it splits a task's wait into the scheduler's completion
 * handling (end of the last predecessor to push) and the queueing (push to first start).
 * Returns the task count (or < 0); writes at most cap ticks. */
int64_t spx_trace_push(const spx_ctx* ctx, uint64_t* ticks, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif /* SPX_H */
