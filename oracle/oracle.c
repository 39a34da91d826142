/*
 * Oracle for the tile-DAG Cholesky path.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product (the HIP library and its Python binding) links, loads or calls this file.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Plain, slow, sequential FP64 C.  Built with -ffp-contract=off so every product and
 * every difference is rounded on its own (no FMA), no BLAS, IEEE sqrt and division.
 *
 * What it follows (Specx, arXiv 2308.15964):
 *  - Sec. 2.1 (task-based parallelization, STF): one thread inserts tasks in program
 *    order with their data accesses; the runtime infers the dependencies from that
 *    order and the parallel run must give exactly the sequential result.
 *  - Sec. 4.1 (task insertion): access modes SpRead (read only), SpWrite (read or
 *    write) and SpCommutativeWrite (a write whose order among the commutative writes
 *    inserted one after another does not matter); a datum is identified by its address
 *    (here: an integer id).
 *  - Sec. 4.7 (internal implementation): per-datum ordered list of the tasks that use
 *    it; a finished task releases the next tasks of each list.
 *  - Sec. 5.2 (numerical applications, Cholesky): the factorisation is split into
 *    tiles and runs as POTRF / TRSM / SYRK / GEMM tasks in FP64.
 *
 * The DAG here is the plain pairwise definition (not the per-datum builder the product
 * uses).  On each datum, a maximal run of consecutive commutative writes is cut into
 * groups of at most 63 (the first 63, the next 63, ...); two commutative writes of one
 * group have no edge (they may run in any order, one at a time).  Otherwise commutative
 * writes count as writes, and for tasks a < b in insertion order, edge (a,b) exists iff
 * some datum d is used by both, at least one of them writes it, and
 *     RAW: a writes d, b only reads d, and every task strictly between them that writes
 *          d is a commutative write of a's group;
 *     WAR: a only reads d, b writes d, and every task strictly between them that writes
 *          d is a commutative write of b's group;
 *     WAW: both write d (not two members of one group), and every task strictly between
 *          them is a commutative write of a's group or of b's group.
 * Without commutative writes these are the plain rules: nothing that writes between a
 * read and a write, nothing at all between two writes.
 * The Cholesky variant is the right-looking tile algorithm on the lower triangle.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_R 1u  /* SpRead  */
#define ORC_RW 2u /* SpWrite (read or write) */
#define ORC_CW 3u /* SpCommutativeWrite */
#define ORC_GROUP_MAX 63

typedef struct {
  uint32_t task;
  uint32_t mode;
  uint64_t datum;
} orc_access;

/* ------------------------------------------------------------------------------------
 * DAG by the pairwise definition
 * ---------------------------------------------------------------------------------- */

typedef struct {
  uint64_t datum;
  uint32_t task;
  uint32_t mode;
  int64_t group; /* commutative writes: the group's number on this datum; else -1 */
} orc_use;

static int cmp_use(const void* x, const void* y) {
  const orc_use* a = (const orc_use*)x;
  const orc_use* b = (const orc_use*)y;
  if (a->datum != b->datum) return a->datum < b->datum ? -1 : 1;
  if (a->task != b->task) return a->task < b->task ? -1 : 1;
  return 0;
}

typedef struct {
  uint32_t src, dst, kind; /* kind: 0 RAW, 1 WAR, 2 WAW */
} orc_edge;

static int cmp_edge(const void* x, const void* y) {
  const orc_edge* a = (const orc_edge*)x;
  const orc_edge* b = (const orc_edge*)y;
  if (a->src != b->src) return a->src < b->src ? -1 : 1;
  if (a->dst != b->dst) return a->dst < b->dst ? -1 : 1;
  if (a->kind != b->kind) return a->kind < b->kind ? -1 : 1;
  return 0;
}

/* Returns the number of distinct edges (or -1 on bad input / no memory).  If src/dst are
 * non-null, up to cap edges are written sorted by (src, dst).  kinds[3] receives the
 * number of distinct edges that are RAW, WAR, WAW on at least one datum. */
int64_t orc_dag_edges(uint32_t ntasks, const orc_access* acc, uint64_t nacc, uint32_t* src,
                      uint32_t* dst, uint64_t cap, uint64_t* kinds) {
  orc_use* use = (orc_use*)malloc((nacc ? nacc : 1) * sizeof(orc_use));
  if (!use) return -1;
  for (uint64_t i = 0; i < nacc; ++i) {
    if (acc[i].task >= ntasks || (acc[i].mode != ORC_R && acc[i].mode != ORC_RW && acc[i].mode != ORC_CW)) {
      free(use);
      return -1;
    }
    use[i].datum = acc[i].datum;
    use[i].task = acc[i].task;
    use[i].mode = acc[i].mode;
  }
  qsort(use, nacc, sizeof(orc_use), cmp_use);
  /* one entry per (datum, task): a task that names a datum twice with two different
   * modes writes it (reading and commutatively writing the same datum is a plain write) */
  uint64_t m = 0;
  for (uint64_t i = 0; i < nacc; ++i) {
    if (m > 0 && use[m - 1].datum == use[i].datum && use[m - 1].task == use[i].task) {
      if (use[i].mode != use[m - 1].mode) use[m - 1].mode = ORC_RW;
    } else {
      use[m++] = use[i];
    }
  }
  /* groups: runs of consecutive commutative writes of a datum, at most ORC_GROUP_MAX each */
  {
    int64_t next = 0, size = 0;
    for (uint64_t i = 0; i < m; ++i) {
      use[i].group = -1;
      if (use[i].mode != ORC_CW) continue;
      int cont = i > 0 && use[i - 1].datum == use[i].datum && use[i - 1].mode == ORC_CW &&
                 size < ORC_GROUP_MAX;
      if (!cont) {
        ++next;
        size = 0;
      }
      use[i].group = next;
      ++size;
    }
  }
  uint64_t ecap = 1024, ne = 0;
  orc_edge* e = (orc_edge*)malloc(ecap * sizeof(orc_edge));
  if (!e) {
    free(use);
    return -1;
  }
  uint64_t g0 = 0;
  while (g0 < m) {
    uint64_t g1 = g0;
    while (g1 < m && use[g1].datum == use[g0].datum) ++g1;
    for (uint64_t p = g0; p < g1; ++p) {
      for (uint64_t q = p + 1; q < g1; ++q) {
        int wp = use[p].mode != ORC_R, wq = use[q].mode != ORC_R;
        if (!wp && !wq) continue;
        int64_t gp = use[p].group, gq = use[q].group;
        if (gp >= 0 && gp == gq) continue; /* two members of one group */
        /* what lies strictly between: writes outside a's group, writes outside b's
         * group, anything outside both groups */
        int w_not_p = 0, w_not_q = 0, any_not_pq = 0;
        for (uint64_t t = p + 1; t < q; ++t) {
          int64_t gt = use[t].group;
          int in_p = gt >= 0 && gt == gp, in_q = gt >= 0 && gt == gq;
          if (use[t].mode != ORC_R) {
            if (!in_p) w_not_p = 1;
            if (!in_q) w_not_q = 1;
          }
          if (!in_p && !in_q) any_not_pq = 1;
        }
        int kind = -1;
        if (wp && !wq && !w_not_p) kind = 0;       /* RAW */
        else if (!wp && wq && !w_not_q) kind = 1;  /* WAR */
        else if (wp && wq && !any_not_pq) kind = 2;/* WAW */
        if (kind < 0) continue;
        if (ne == ecap) {
          ecap *= 2;
          orc_edge* ne_ = (orc_edge*)realloc(e, ecap * sizeof(orc_edge));
          if (!ne_) {
            free(e);
            free(use);
            return -1;
          }
          e = ne_;
        }
        e[ne].src = use[p].task;
        e[ne].dst = use[q].task;
        e[ne].kind = (uint32_t)kind;
        ++ne;
      }
    }
    g0 = g1;
  }
  free(use);
  qsort(e, ne, sizeof(orc_edge), cmp_edge);
  if (kinds) kinds[0] = kinds[1] = kinds[2] = 0;
  int64_t nd = 0;
  for (uint64_t i = 0; i < ne; ++i) {
    int same_edge = i > 0 && e[i].src == e[i - 1].src && e[i].dst == e[i - 1].dst;
    int same_kind = same_edge && e[i].kind == e[i - 1].kind;
    if (kinds && !same_kind) kinds[e[i].kind]++;
    if (same_edge) continue;
    if (src && (uint64_t)nd < cap) {
      src[nd] = e[i].src;
      dst[nd] = e[i].dst;
    }
    ++nd;
  }
  free(e);
  return nd;
}

/* ------------------------------------------------------------------------------------
 * Cholesky and solve task programs (right-looking, lower triangle)
 * ---------------------------------------------------------------------------------- */

enum { T_POTRF = 0, T_TRSM = 1, T_SYRK = 2, T_GEMM = 3, T_FTRSM = 4, T_FGEMM = 5, T_BTRSM = 6, T_BGEMM = 7,
       T_MGEMM = 8 };

typedef struct {
  int32_t type, i, j, k;
} orc_task;

/* datum ids: tile (i,j) of A -> i*nt + j; block k of the right-hand side -> nt*nt + k */
static uint64_t dA(int nt, int i, int j) { return (uint64_t)i * (uint64_t)nt + (uint64_t)j; }
static uint64_t dB(int nt, int k) { return (uint64_t)nt * (uint64_t)nt + (uint64_t)k; }

/* Writes the task program into tasks/acc (each may be null to count).  flags bit 0
 * (with_solve) adds the forward (L y = b) and backward (L^T x = y) block substitutions
 * after the factor; bit 8 declares the updates (SYRK and GEMM on their tile, FGEMM and
 * BGEMM on their block of the right-hand side) as commutative writes.  Returns the task
 * count; *nacc_out receives the access count. */
int64_t orc_cholesky_program(int nt, int with_solve, orc_task* tasks, orc_access* acc,
                             uint64_t* nacc_out) {
  int64_t nt_ = 0;
  uint64_t na = 0;
  const uint32_t UPD = (with_solve & 0x100) ? ORC_CW : ORC_RW;
  with_solve &= 1;
#define ADD_TASK(TY, I, J, K)                                 \
  do {                                                        \
    if (tasks) {                                              \
      tasks[nt_].type = (TY); tasks[nt_].i = (I);             \
      tasks[nt_].j = (J); tasks[nt_].k = (K);                 \
    }                                                         \
    ++nt_;                                                    \
  } while (0)
#define ADD_ACC(MODE, D)                                      \
  do {                                                        \
    if (acc) {                                                \
      acc[na].task = (uint32_t)(nt_ - 1); acc[na].mode = (MODE); \
      acc[na].datum = (D);                                    \
    }                                                         \
    ++na;                                                     \
  } while (0)
  for (int k = 0; k < nt; ++k) {
    ADD_TASK(T_POTRF, k, k, k);
    ADD_ACC(ORC_RW, dA(nt, k, k));
    for (int i = k + 1; i < nt; ++i) {
      ADD_TASK(T_TRSM, i, k, k);
      ADD_ACC(ORC_R, dA(nt, k, k));
      ADD_ACC(ORC_RW, dA(nt, i, k));
    }
    for (int i = k + 1; i < nt; ++i) {
      ADD_TASK(T_SYRK, i, i, k);
      ADD_ACC(ORC_R, dA(nt, i, k));
      ADD_ACC(UPD, dA(nt, i, i));
      for (int j = k + 1; j < i; ++j) {
        ADD_TASK(T_GEMM, i, j, k);
        ADD_ACC(ORC_R, dA(nt, i, k));
        ADD_ACC(ORC_R, dA(nt, j, k));
        ADD_ACC(UPD, dA(nt, i, j));
      }
    }
  }
  if (with_solve) {
    for (int k = 0; k < nt; ++k) {
      ADD_TASK(T_FTRSM, k, k, k);
      ADD_ACC(ORC_R, dA(nt, k, k));
      ADD_ACC(ORC_RW, dB(nt, k));
      for (int i = k + 1; i < nt; ++i) {
        ADD_TASK(T_FGEMM, i, k, k);
        ADD_ACC(ORC_R, dA(nt, i, k));
        ADD_ACC(ORC_R, dB(nt, k));
        ADD_ACC(UPD, dB(nt, i));
      }
    }
    for (int k = nt - 1; k >= 0; --k) {
      ADD_TASK(T_BTRSM, k, k, k);
      ADD_ACC(ORC_R, dA(nt, k, k));
      ADD_ACC(ORC_RW, dB(nt, k));
      for (int i = 0; i < k; ++i) {
        ADD_TASK(T_BGEMM, i, k, k);
        ADD_ACC(ORC_R, dA(nt, k, i));
        ADD_ACC(ORC_R, dB(nt, k));
        ADD_ACC(UPD, dB(nt, i));
      }
    }
  }
  if (nacc_out) *nacc_out = na;
  return nt_;
}

/* The tiled matrix product of Sec. 5.2 (the GEMM application): C <- C + A B for three
 * nt x nt tile matrices, one task per (i, j, k) updating C_ij with A_ik B_kj.  Inserted
 * with k outermost.  Datum ids: A_ik -> i*nt + k, B_kj -> nt^2 + k*nt + j, C_ij ->
 * 2 nt^2 + i*nt + j.  commute: the updates of C_ij are commutative writes.  Returns the
 * task count; *nacc_out receives the access count. */
int64_t orc_gemm_program(int nt, int commute, orc_task* tasks, orc_access* acc, uint64_t* nacc_out) {
  int64_t nt_ = 0;
  uint64_t na = 0;
  const uint64_t n2 = (uint64_t)nt * (uint64_t)nt;
  for (int k = 0; k < nt; ++k)
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nt; ++j) {
        ADD_TASK(T_MGEMM, i, j, k);
        ADD_ACC(ORC_R, (uint64_t)i * nt + k);
        ADD_ACC(ORC_R, n2 + (uint64_t)k * nt + j);
        ADD_ACC(commute ? ORC_CW : ORC_RW, 2 * n2 + (uint64_t)i * nt + j);
      }
  if (nacc_out) *nacc_out = na;
  return nt_;
}
#undef ADD_TASK
#undef ADD_ACC

/* ------------------------------------------------------------------------------------
 * Tile kernels.  Column-major storage with leading dimension ld; every kernel works in
 * place, walks the contraction index in the order stated, and keeps no temporaries.
 * ---------------------------------------------------------------------------------- */

#define AT(p, ld, r, c) (p)[(size_t)(c) * (size_t)(ld) + (size_t)(r)]

/* A_kk <- chol(A_kk), lower.  Returns 0, or the 1-based local column whose pivot is not
 * positive (or is NaN). */
static int potrf_tile(double* a, int64_t ld, int nb) {
  for (int c = 0; c < nb; ++c) {
    double p = AT(a, ld, c, c);
    if (!(p > 0.0)) return c + 1;
    double d = sqrt(p);
    AT(a, ld, c, c) = d;
    for (int r = c + 1; r < nb; ++r) AT(a, ld, r, c) = AT(a, ld, r, c) / d;
    for (int j = c + 1; j < nb; ++j)
      for (int r = j; r < nb; ++r) AT(a, ld, r, j) = AT(a, ld, r, j) - AT(a, ld, r, c) * AT(a, ld, j, c);
  }
  return 0;
}

/* B <- B * L^{-T} (B is an off-diagonal tile of the same block column as L). */
static void trsm_tile(double* b, const double* l, int64_t ld, int nb) {
  for (int c = 0; c < nb; ++c) {
    for (int r = 0; r < nb; ++r) AT(b, ld, r, c) = AT(b, ld, r, c) / AT(l, ld, c, c);
    for (int j = c + 1; j < nb; ++j)
      for (int r = 0; r < nb; ++r) AT(b, ld, r, j) = AT(b, ld, r, j) - AT(b, ld, r, c) * AT(l, ld, j, c);
  }
}

/* C <- C - A * A^T, lower triangle of C only, m ascending. */
static void syrk_tile(double* cm, const double* a, int64_t ld, int nb) {
  for (int m = 0; m < nb; ++m)
    for (int j = 0; j < nb; ++j)
      for (int r = j; r < nb; ++r) AT(cm, ld, r, j) = AT(cm, ld, r, j) - AT(a, ld, r, m) * AT(a, ld, j, m);
}

/* C <- C - A * B^T, m ascending. */
static void gemm_tile(double* cm, const double* a, const double* b, int64_t ld, int nb) {
  for (int m = 0; m < nb; ++m)
    for (int j = 0; j < nb; ++j)
      for (int r = 0; r < nb; ++r) AT(cm, ld, r, j) = AT(cm, ld, r, j) - AT(a, ld, r, m) * AT(b, ld, j, m);
}

/* C <- C + A * B (the GEMM application's task), m ascending. */
static void mgemm_tile(double* cm, const double* a, const double* b, int64_t ld, int nb) {
  for (int m = 0; m < nb; ++m)
    for (int j = 0; j < nb; ++j)
      for (int r = 0; r < nb; ++r) AT(cm, ld, r, j) = AT(cm, ld, r, j) + AT(a, ld, r, m) * AT(b, ld, m, j);
}

/* Forward block substitution.  y is a block of rows of the right-hand side (ldb). */
static void ftrsm_tile(double* y, int64_t ldb, int nrhs, const double* l, int64_t ld, int nb) {
  for (int q = 0; q < nrhs; ++q) {
    double* v = y + (size_t)q * (size_t)ldb;
    for (int c = 0; c < nb; ++c) {
      v[c] = v[c] / AT(l, ld, c, c);
      for (int r = c + 1; r < nb; ++r) v[r] = v[r] - AT(l, ld, r, c) * v[c];
    }
  }
}
/* y_i <- y_i - L_ik * y_k, m ascending. */
static void fgemm_tile(double* yi, const double* yk, int64_t ldb, int nrhs, const double* l, int64_t ld, int nb) {
  for (int q = 0; q < nrhs; ++q)
    for (int m = 0; m < nb; ++m)
      for (int r = 0; r < nb; ++r)
        yi[(size_t)q * ldb + r] = yi[(size_t)q * ldb + r] - AT(l, ld, r, m) * yk[(size_t)q * ldb + m];
}
/* Backward block substitution with L_kk^T, column index descending. */
static void btrsm_tile(double* y, int64_t ldb, int nrhs, const double* l, int64_t ld, int nb) {
  for (int q = 0; q < nrhs; ++q) {
    double* v = y + (size_t)q * (size_t)ldb;
    for (int c = nb - 1; c >= 0; --c) {
      v[c] = v[c] / AT(l, ld, c, c);
      for (int r = 0; r < c; ++r) v[r] = v[r] - AT(l, ld, c, r) * v[c];
    }
  }
}
/* y_i <- y_i - L_ki^T * y_k (i < k), m descending.  l points at tile (k,i). */
static void bgemm_tile(double* yi, const double* yk, int64_t ldb, int nrhs, const double* l, int64_t ld, int nb) {
  for (int q = 0; q < nrhs; ++q)
    for (int m = nb - 1; m >= 0; --m)
      for (int r = 0; r < nb; ++r)
        yi[(size_t)q * ldb + r] = yi[(size_t)q * ldb + r] - AT(l, ld, m, r) * yk[(size_t)q * ldb + m];
}

/* Runs one task on the dense column-major matrix a (n x n, ld = n) and right-hand side
 * y (n x nrhs, ld = n).  For the GEMM program a holds A, B and C side by side (n x 3n,
 * ld = n): tile (i, k) of A, (k, j) of B at tile column nt + j, (i, j) of C at 2 nt + j.
 * Returns 0 or the 1-based global column of a failed pivot. */
static int run_task(const orc_task* t, double* a, int64_t n, int nb, double* y, int nrhs) {
  const int64_t ld = n;
#define TILE(I, J) (a + (size_t)(J) * (size_t)nb * (size_t)ld + (size_t)(I) * (size_t)nb)
#define YB(I) (y + (size_t)(I) * (size_t)nb)
  switch (t->type) {
    case T_POTRF: {
      int c = potrf_tile(TILE(t->k, t->k), ld, nb);
      return c ? t->k * nb + c : 0;
    }
    case T_TRSM: trsm_tile(TILE(t->i, t->k), TILE(t->k, t->k), ld, nb); return 0;
    case T_SYRK: syrk_tile(TILE(t->i, t->i), TILE(t->i, t->k), ld, nb); return 0;
    case T_GEMM: gemm_tile(TILE(t->i, t->j), TILE(t->i, t->k), TILE(t->j, t->k), ld, nb); return 0;
    case T_FTRSM: ftrsm_tile(YB(t->k), n, nrhs, TILE(t->k, t->k), ld, nb); return 0;
    case T_FGEMM: fgemm_tile(YB(t->i), YB(t->k), n, nrhs, TILE(t->i, t->k), ld, nb); return 0;
    case T_BTRSM: btrsm_tile(YB(t->k), n, nrhs, TILE(t->k, t->k), ld, nb); return 0;
    case T_BGEMM: bgemm_tile(YB(t->i), YB(t->j), n, nrhs, TILE(t->j, t->i), ld, nb); return 0;
    case T_MGEMM: {
      const int nt = (int)(n / nb);
      mgemm_tile(TILE(t->i, 2 * nt + t->j), TILE(t->i, t->k), TILE(t->k, nt + t->j), ld, nb);
      return 0;
    }
  }
#undef TILE
#undef YB
  return 0;
}

/* ------------------------------------------------------------------------------------
 * Sequential STF executor (Kahn's algorithm over the pairwise DAG)
 * ---------------------------------------------------------------------------------- */

static uint64_t splitmix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct {
  int64_t ntasks, nedges;
  orc_task* tasks;
  int64_t* off; /* CSR successors */
  uint32_t* succ;
  uint32_t* indeg;
} orc_prog;

static void prog_free(orc_prog* p) {
  free(p->tasks);
  free(p->off);
  free(p->succ);
  free(p->indeg);
}

/* flags < 0: the GEMM program instead of the Cholesky one (-2: with commutative
 * updates); otherwise the flags of orc_cholesky_program. */
static int prog_make(int nt, int with_solve, const uint32_t* drop_edge /* nullable: {src,dst} */,
                     orc_prog* p) {
  memset(p, 0, sizeof(*p));
  uint64_t na = 0;
  const int gcomm = with_solve == -2;
  int64_t T = with_solve < 0 ? orc_gemm_program(nt, gcomm, NULL, NULL, &na)
                             : orc_cholesky_program(nt, with_solve, NULL, NULL, &na);
  p->tasks = (orc_task*)malloc((T ? T : 1) * sizeof(orc_task));
  orc_access* acc = (orc_access*)malloc((na ? na : 1) * sizeof(orc_access));
  if (!p->tasks || !acc) {
    free(acc);
    prog_free(p);
    return -1;
  }
  if (with_solve < 0)
    orc_gemm_program(nt, gcomm, p->tasks, acc, &na);
  else
    orc_cholesky_program(nt, with_solve, p->tasks, acc, &na);
  int64_t E = orc_dag_edges((uint32_t)T, acc, na, NULL, NULL, 0, NULL);
  uint32_t* src = (uint32_t*)malloc((E ? E : 1) * sizeof(uint32_t));
  uint32_t* dst = (uint32_t*)malloc((E ? E : 1) * sizeof(uint32_t));
  p->off = (int64_t*)calloc(T + 1, sizeof(int64_t));
  p->succ = (uint32_t*)malloc((E ? E : 1) * sizeof(uint32_t));
  p->indeg = (uint32_t*)calloc(T ? T : 1, sizeof(uint32_t));
  if (E < 0 || !src || !dst || !p->off || !p->succ || !p->indeg) {
    free(acc); free(src); free(dst);
    prog_free(p);
    return -1;
  }
  orc_dag_edges((uint32_t)T, acc, na, src, dst, (uint64_t)E, NULL);
  free(acc);
  int64_t w = 0;
  for (int64_t e = 0; e < E; ++e) {
    if (drop_edge && src[e] == drop_edge[0] && dst[e] == drop_edge[1]) continue;
    src[w] = src[e];
    dst[w] = dst[e];
    ++w;
  }
  E = w;
  for (int64_t e = 0; e < E; ++e) p->off[src[e] + 1]++;
  for (int64_t t = 0; t < T; ++t) p->off[t + 1] += p->off[t];
  for (int64_t e = 0; e < E; ++e) {
    p->succ[e] = dst[e]; /* edges are sorted by src, so CSR order = sorted order */
    p->indeg[dst[e]]++;
  }
  free(src);
  free(dst);
  p->ntasks = T;
  p->nedges = E;
  return 0;
}

/* Priority key of the sequential "priority" order: lower sorts first. */
static int64_t prio_key(const orc_task* t, int64_t idx) {
  int rank;
  switch (t->type) {
    case T_POTRF: rank = 0; break;
    case T_TRSM: rank = 1; break;
    case T_SYRK: rank = 2; break;
    case T_GEMM: rank = 3; break;
    default: rank = 4; break;
  }
  return ((int64_t)rank << 40) | ((int64_t)t->k << 24) | idx;
}

/* order: 0 = smallest ready index first (the insertion order), 1 = seeded random choice
 * among the ready tasks, 2 = priority (POTRF > TRSM > SYRK > GEMM, then smaller k),
 * 3 = the order given in order_out (every task must be ready at its turn, else -2).
 * order_out (nullable) receives the executed task indices.
 * Returns 0, a positive 1-based failing column, or a negative error. */
static int64_t exec_seq(orc_prog* p, int order, uint64_t seed, double* a, int64_t n, int nb,
                        double* y, int nrhs, int64_t* order_out, int64_t* nrun_out) {
  int64_t T = p->ntasks;
  uint32_t* cnt = (uint32_t*)malloc((T ? T : 1) * sizeof(uint32_t));
  int64_t* ready = (int64_t*)malloc((T ? T : 1) * sizeof(int64_t));
  if (!cnt || !ready) {
    free(cnt);
    free(ready);
    return -1;
  }
  memcpy(cnt, p->indeg, T * sizeof(uint32_t));
  int64_t nready = 0, nrun = 0, info = 0;
  for (int64_t t = 0; t < T; ++t)
    if (cnt[t] == 0) ready[nready++] = t;
  uint64_t s = seed;
  if (order == 3 && !order_out) nready = 0;
  while (nready > 0) {
    int64_t pick = 0;
    if (order == 3) {
      if (nrun >= T) break;
      const int64_t want = order_out[nrun];
      pick = -1;
      for (int64_t q = 0; q < nready; ++q)
        if (ready[q] == want) pick = q;
      if (pick < 0) {
        info = -2;
        break;
      }
    } else if (order == 0) {
      for (int64_t q = 1; q < nready; ++q)
        if (ready[q] < ready[pick]) pick = q;
    } else if (order == 1) {
      pick = (int64_t)(splitmix64(&s) % (uint64_t)nready);
    } else {
      for (int64_t q = 1; q < nready; ++q)
        if (prio_key(&p->tasks[ready[q]], ready[q]) < prio_key(&p->tasks[ready[pick]], ready[pick])) pick = q;
    }
    int64_t t = ready[pick];
    ready[pick] = ready[--nready];
    int r = run_task(&p->tasks[t], a, n, nb, y, nrhs);
    if (order_out) order_out[nrun] = t;
    ++nrun;
    if (r) { /* a failed pivot: the successors never run */
      info = r;
      break;
    }
    for (int64_t e = p->off[t]; e < p->off[t + 1]; ++e)
      if (--cnt[p->succ[e]] == 0) ready[nready++] = p->succ[e];
  }
  free(cnt);
  free(ready);
  if (nrun_out) *nrun_out = nrun;
  return info;
}

/* ------------------------------------------------------------------------------------
 * Parallel executor: the same DAG and kernels run by a pool of host threads.  Ready
 * tasks are taken smallest index first; the result is the sequential one because every
 * write to a tile is chained in insertion order (all updates of a tile are WAW-ordered).
 * With limit > 0 only tasks [0, limit) run: all edges point forward, so that prefix of
 * the insertion order is closed under predecessors (used for a bounded timing sample).
 * ---------------------------------------------------------------------------------- */

typedef struct {
  orc_prog* p;
  double* a;
  double* y;
  int64_t n;
  int nb, nrhs;
  pthread_mutex_t mu;
  pthread_cond_t cv;
  uint32_t* cnt;
  int64_t* ready;
  int64_t nready, ndone, info, limit;
} par_state;

static void* par_worker(void* arg) {
  par_state* st = (par_state*)arg;
  pthread_mutex_lock(&st->mu);
  for (;;) {
    while (st->nready == 0 && st->ndone < st->limit) pthread_cond_wait(&st->cv, &st->mu);
    if (st->nready == 0) break;
    int64_t pick = 0;
    for (int64_t q = 1; q < st->nready; ++q)
      if (st->ready[q] < st->ready[pick]) pick = q;
    int64_t t = st->ready[pick];
    st->ready[pick] = st->ready[--st->nready];
    int skip = st->info != 0; /* after a failed pivot the rest drain without computing */
    pthread_mutex_unlock(&st->mu);
    int r = skip ? 0 : run_task(&st->p->tasks[t], st->a, st->n, st->nb, st->y, st->nrhs);
    pthread_mutex_lock(&st->mu);
    if (r && (st->info == 0 || r < st->info)) st->info = r;
    st->ndone++;
    for (int64_t e = st->p->off[t]; e < st->p->off[t + 1]; ++e) {
      uint32_t s = st->p->succ[e];
      if (--st->cnt[s] == 0 && (int64_t)s < st->limit) st->ready[st->nready++] = s;
    }
    pthread_cond_broadcast(&st->cv);
  }
  pthread_mutex_unlock(&st->mu);
  return NULL;
}

static int64_t exec_par(orc_prog* p, int nthreads, double* a, int64_t n, int nb, double* y, int nrhs,
                        int64_t limit) {
  par_state st;
  memset(&st, 0, sizeof(st));
  st.p = p;
  st.a = a;
  st.y = y;
  st.n = n;
  st.nb = nb;
  st.nrhs = nrhs;
  st.limit = (limit > 0 && limit < p->ntasks) ? limit : p->ntasks;
  st.cnt = (uint32_t*)malloc((p->ntasks ? p->ntasks : 1) * sizeof(uint32_t));
  st.ready = (int64_t*)malloc((p->ntasks ? p->ntasks : 1) * sizeof(int64_t));
  pthread_t* th = (pthread_t*)malloc((nthreads > 0 ? nthreads : 1) * sizeof(pthread_t));
  if (!st.cnt || !st.ready || !th) {
    free(st.cnt);
    free(st.ready);
    free(th);
    return -1;
  }
  memcpy(st.cnt, p->indeg, p->ntasks * sizeof(uint32_t));
  for (int64_t t = 0; t < st.limit; ++t)
    if (st.cnt[t] == 0) st.ready[st.nready++] = t;
  pthread_mutex_init(&st.mu, NULL);
  pthread_cond_init(&st.cv, NULL);
  if (nthreads < 1) nthreads = 1;
  for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, par_worker, &st);
  for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
  free(th);
  pthread_mutex_destroy(&st.mu);
  pthread_cond_destroy(&st.cv);
  free(st.cnt);
  free(st.ready);
  return st.info;
}

/* ------------------------------------------------------------------------------------
 * Public entry points
 * ---------------------------------------------------------------------------------- */

/* Tile Cholesky of the n x n SPD matrix a (column-major, ld = n, lower triangle read and
 * overwritten by L; the strict upper triangle is not touched) with tile size nb (n % nb
 * == 0), then, if y != NULL and nrhs > 0, the solve A x = y in place (y is n x nrhs,
 * column-major, ld = n).
 *   nthreads <= 1: sequential executor with the given order (0 insertion, 1 seeded
 *   random, 2 priority); order_out (nullable, ntasks entries) receives the run order.
 *   nthreads > 1: parallel executor.
 *   limit > 0: run only tasks [0, limit) of the insertion order (on the thread pool,
 *   with one thread if nthreads <= 1).
 *   drop_edge (nullable {src,dst}): remove one DAG edge (a planted mistake for tests).
 *   commute: the updates are commutative writes (sequential executor only).
 * Returns 0, the 1-based global column of the first non-positive pivot, or -1 (-2: a
 * given order that is not valid). */
int64_t orc_cholesky(int64_t n, int nb, double* a, double* y, int nrhs, int order, uint64_t seed,
                     int nthreads, int64_t* order_out, int64_t limit, const uint32_t* drop_edge,
                     int64_t* nrun_out, int commute) {
  if (n <= 0 || nb <= 0 || n % nb != 0 || !a) return -1;
  if (commute && (nthreads > 1 || limit > 0)) return -1;
  int nt = (int)(n / nb);
  int with_solve = (y != NULL && nrhs > 0) | (commute ? 0x100 : 0);
  orc_prog p;
  if (prog_make(nt, with_solve, drop_edge, &p) != 0) return -1;
  int64_t info;
  if (nthreads <= 1 && limit <= 0)
    info = exec_seq(&p, order, seed, a, n, nb, y, nrhs, order_out, nrun_out);
  else
    info = exec_par(&p, nthreads, a, n, nb, y, nrhs, limit);
  prog_free(&p);
  return info;
}

/* The GEMM program: abc holds A, B and C (each n x n) side by side, column-major n x 3n
 * (ld = n); C is overwritten by C + A B computed tile by tile (tile size nb, n % nb == 0)
 * in the chosen order (as for orc_cholesky; nthreads > 1: thread pool).  drop_edge and
 * commute as for orc_cholesky.  Returns 0 or -1 (-2: a given order that is not valid). */
int64_t orc_gemm(int64_t n, int nb, double* abc, int order, uint64_t seed, int nthreads, int64_t* order_out,
                 const uint32_t* drop_edge, int64_t* nrun_out, int commute) {
  if (n <= 0 || nb <= 0 || n % nb != 0 || !abc) return -1;
  if (commute && nthreads > 1) return -1;
  orc_prog p;
  if (prog_make((int)(n / nb), commute ? -2 : -1, drop_edge, &p) != 0) return -1;
  int64_t info;
  if (nthreads <= 1)
    info = exec_seq(&p, order, seed, abc, n, nb, NULL, 0, order_out, nrun_out);
  else
    info = exec_par(&p, nthreads, abc, n, nb, NULL, 0, 0);
  prog_free(&p);
  return info;
}

/* Edges of the GEMM program (as orc_cholesky_dag). */
int64_t orc_gemm_dag(int nt, int commute, uint32_t* src, uint32_t* dst, uint64_t cap, uint64_t* kinds,
                     int64_t* ntasks_out) {
  uint64_t na = 0;
  int64_t T = orc_gemm_program(nt, commute, NULL, NULL, &na);
  orc_access* acc = (orc_access*)malloc((na ? na : 1) * sizeof(orc_access));
  if (!acc) return -1;
  orc_gemm_program(nt, commute, NULL, acc, &na);
  int64_t E = orc_dag_edges((uint32_t)T, acc, na, src, dst, cap, kinds);
  free(acc);
  if (ntasks_out) *ntasks_out = T;
  return E;
}

/* Sampled entries of C0 + A B, one by one (for sizes the executor cannot run in a test):
 * out[s] = C0(i, j) + sum over m ascending of A(i, m) B(m, j), plain FP64, for (i, j) =
 * (ii[s], jj[s]).  A, B, C0 column-major n x n (ld = n). */
void orc_gemm_entries(const double* a, const double* b, const double* c0, int64_t n, const int64_t* ii,
                      const int64_t* jj, int64_t count, double* out) {
  for (int64_t s = 0; s < count; ++s) {
    const int64_t i = ii[s], j = jj[s];
    double c = c0[(size_t)j * n + i];
    for (int64_t m = 0; m < n; ++m) c = c + a[(size_t)m * n + i] * b[(size_t)j * n + m];
    out[s] = c;
  }
}

/* Runs one task of the program (type codes as in orc_cholesky_program) on the dense
 * column-major matrix a (n x n, ld = n, tile size nb) and right-hand side y (n x nrhs,
 * ld = n).  Returns 0 or the 1-based global column of a failed pivot. */
int64_t orc_run_task(int type, int i, int j, int k, double* a, int64_t n, int nb, double* y, int nrhs) {
  if (!a || nb <= 0 || n % nb || type < 0 || type > T_BGEMM) return -1;
  orc_task t = {type, i, j, k};
  return run_task(&t, a, n, nb, y, nrhs);
}

/* The DAG of the Cholesky (+ solve) program as CSR-free edge arrays; returns the edge
 * count, or -1.  Same definition as orc_dag_edges, applied to orc_cholesky_program. */
int64_t orc_cholesky_dag(int nt, int with_solve, uint32_t* src, uint32_t* dst, uint64_t cap,
                         uint64_t* kinds, int64_t* ntasks_out) {
  uint64_t na = 0;
  int64_t T = orc_cholesky_program(nt, with_solve, NULL, NULL, &na);
  orc_access* acc = (orc_access*)malloc((na ? na : 1) * sizeof(orc_access));
  if (!acc) return -1;
  orc_cholesky_program(nt, with_solve, NULL, acc, &na);
  int64_t E = orc_dag_edges((uint32_t)T, acc, na, src, dst, cap, kinds);
  free(acc);
  if (ntasks_out) *ntasks_out = T;
  return E;
}

/* ------------------------------------------------------------------------------------
 * Residuals with compensated dot products (Ogita, Rump, Oishi 2005, algorithm Dot2):
 * each product is split exactly into a rounded part and its error (Dekker / Veltkamp
 * splitting, no FMA), each sum by Knuth's TwoSum, and the errors are summed apart.
 * The matrix argument is always the lower triangle of a symmetric matrix (column-major,
 * ld = n); entry (i,j) with i < j is read as (j,i).
 * ---------------------------------------------------------------------------------- */

typedef struct {
  double s, c;
} dot2;

static void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}
static void split27(double a, double* hi, double* lo) {
  double c = 134217729.0 * a; /* 2^27 + 1 */
  double t = c - a;
  *hi = c - t;
  *lo = a - *hi;
}
static void two_prod(double a, double b, double* p, double* e) {
  double x = a * b, ah, al, bh, bl;
  split27(a, &ah, &al);
  split27(b, &bh, &bl);
  *e = al * bl - (((x - ah * bh) - al * bh) - ah * bl);
  *p = x;
}
static void d2_sub_prod(dot2* d, double a, double b) {
  double p, q, s, e;
  two_prod(a, b, &p, &q);
  two_sum(d->s, -p, &s, &e);
  d->s = s;
  d->c += e - q;
}
static double d2_val(const dot2* d) { return d->s + d->c; }

static double sym(const double* a, int64_t n, int64_t i, int64_t j) {
  return i >= j ? a[(size_t)j * n + i] : a[(size_t)i * n + j];
}

double orc_dot2(const double* x, const double* y, int64_t n) {
  dot2 d = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) d2_sub_prod(&d, -x[i], y[i]);
  return d2_val(&d);
}

/* ||A||_inf of the symmetric matrix. */
double orc_norm_inf_sym(const double* a, int64_t n) {
  double best = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += fabs(sym(a, n, i, j));
    if (s > best || s != s) best = s;
  }
  return best;
}

/* ||A - L L^T||_F / ||A||_F, exact up to the compensated rounding (O(n^3)). */
double orc_factor_residual(const double* a, const double* l, int64_t n) {
  double num = 0.0, den = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t i = j; i < n; ++i) {
      dot2 d = {a[(size_t)j * n + i], 0.0};
      for (int64_t m = 0; m <= j; ++m) d2_sub_prod(&d, l[(size_t)m * n + i], l[(size_t)m * n + j]);
      double r = d2_val(&d), v = a[(size_t)j * n + i];
      double w = (i == j) ? 1.0 : 2.0;
      num += w * r * r;
      den += w * v * v;
    }
  }
  return sqrt(num) / sqrt(den);
}

static double gauss(uint64_t* s) {
  double u1 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  double u2 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* ||(A - L L^T) v||_2 / ||A v||_2 for one vector v (n entries), with w = L^T v rounded
 * once and both products accumulated with Dot2.  O(n^2). */
static double residual_ratio(const double* a, const double* l, int64_t n, const double* v, double* w) {
  /* w = L^T v */
  for (int64_t m = 0; m < n; ++m) {
    dot2 d = {0.0, 0.0};
    for (int64_t i = m; i < n; ++i) d2_sub_prod(&d, -l[(size_t)m * n + i], v[i]);
    w[m] = d2_val(&d);
  }
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    dot2 r = {0.0, 0.0}, av = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
      double aij = sym(a, n, i, j);
      d2_sub_prod(&r, -aij, v[j]);
      d2_sub_prod(&av, -aij, v[j]);
    }
    for (int64_t m = 0; m <= i; ++m) d2_sub_prod(&r, l[(size_t)m * n + i], w[m]);
    double rv = d2_val(&r), avv = d2_val(&av);
    num += rv * rv;
    den += avv * avv;
  }
  return sqrt(num) / sqrt(den);
}

/* The largest ||(A - L L^T) v||_2 / ||A v||_2 over the nvec caller-given vectors
 * (column-major n x nvec, ld = n).  Returns -1 if out of memory. */
double orc_factor_residual_vectors(const double* a, const double* l, int64_t n, const double* vecs, int nvec) {
  double* w = (double*)malloc(n * sizeof(double));
  if (!w) return -1.0;
  double worst = 0.0;
  for (int q = 0; q < nvec; ++q) {
    double e = residual_ratio(a, l, n, vecs + (size_t)q * n, w);
    if (e > worst || e != e) worst = e;
  }
  free(w);
  return worst;
}

/* Randomised estimate of the factor residual for large n (Freivalds-style probing):
 * max over nvec Gaussian vectors v of ||(A - L L^T) v||_2 / ||A v||_2.  O(n^2) each. */
double orc_factor_residual_probe(const double* a, const double* l, int64_t n, int nvec, uint64_t seed) {
  double* v = (double*)malloc(n * sizeof(double));
  double* w = (double*)malloc(n * sizeof(double));
  if (!v || !w) {
    free(v);
    free(w);
    return -1.0;
  }
  uint64_t s = seed;
  double worst = 0.0;
  for (int q = 0; q < nvec; ++q) {
    for (int64_t i = 0; i < n; ++i) v[i] = gauss(&s);
    double e = residual_ratio(a, l, n, v, w);
    if (e > worst || e != e) worst = e;
  }
  free(v);
  free(w);
  return worst;
}

/* Normwise backward error per right-hand side (Rigal and Gaches):
 *   eta_q = ||b_q - A x_q||_inf / (||A||_inf ||x_q||_inf + ||b_q||_inf).
 * x, b: n x nrhs column-major with leading dimension ld.  anorm < 0: computed here. */
void orc_backward_error(const double* a, int64_t n, const double* x, const double* b, int64_t ld,
                        int nrhs, double anorm, double* eta) {
  if (anorm < 0) anorm = orc_norm_inf_sym(a, n);
  for (int q = 0; q < nrhs; ++q) {
    const double* xq = x + (size_t)q * ld;
    const double* bq = b + (size_t)q * ld;
    double rmax = 0.0, xmax = 0.0, bmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      dot2 d = {bq[i], 0.0};
      for (int64_t j = 0; j < n; ++j) d2_sub_prod(&d, sym(a, n, i, j), xq[j]);
      double r = fabs(d2_val(&d));
      if (r > rmax || r != r) rmax = r;
      if (fabs(xq[i]) > xmax) xmax = fabs(xq[i]);
      if (fabs(bq[i]) > bmax) bmax = fabs(bq[i]);
    }
    eta[q] = rmax / (anorm * xmax + bmax);
  }
}

/* Check of sampled entries of a factor against its defining equations, for sizes the
 * oracle cannot factor itself: for each sampled (i,j), i >= j,
 *     A_ij - sum_{m<=j} L_im L_jm
 * relative to sqrt(A_ii A_jj).  Returns the largest such value. */
double orc_factor_entry_check(const double* a, const double* l, int64_t n, const int64_t* ii,
                              const int64_t* jj, int64_t count) {
  double worst = 0.0;
  for (int64_t s = 0; s < count; ++s) {
    int64_t i = ii[s], j = jj[s];
    if (i < j) {
      int64_t t = i;
      i = j;
      j = t;
    }
    dot2 d = {sym(a, n, i, j), 0.0};
    for (int64_t m = 0; m <= j; ++m) d2_sub_prod(&d, l[(size_t)m * n + i], l[(size_t)m * n + j]);
    double e = fabs(d2_val(&d)) / sqrt(fabs(sym(a, n, i, i)) * fabs(sym(a, n, j, j)));
    if (e > worst || e != e) worst = e;
  }
  return worst;
}
