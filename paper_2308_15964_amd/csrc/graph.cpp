// Host-side STF graph builder (Specx Sec. 2.1, Sec. 4.1, Sec. 4.7).
//
// Tasks arrive in insertion order with their declared accesses.  Per datum the builder
// keeps the last writer and the set of tasks that read it since that write, which is the
// information Specx keeps in its per-datum dependency lists.  From it each new task gets:
//   read:  an edge from the last writer (read after write);
//   write: an edge from every reader since the last write (write after read), or from
//          the last writer when nobody read in between (write after write).
// Instead of walking per-datum lists at run time, the edges are materialised once (CSR
// successors + in-degree) so the device scheduler can release successors with one atomic
// decrement each.
#include "spx_internal.h"

#include <algorithm>
#include <cstdio>
#include <unordered_map>

namespace spx {

namespace {
// Per datum: the current writer set (the last writer, or every member of the last closed
// commutative group), the reads since, and the open commutative group (its members and
// the dependencies every member takes: the state before the group).
struct DatumState {
  std::vector<uint32_t> writers;
  std::vector<uint32_t> readers;  // since the writer set
  int64_t group = -1;             // open group id
  std::vector<uint32_t> members, pre;
};
void close_group(DatumState& s) {
  if (s.group < 0) return;
  s.writers.swap(s.members);
  s.members.clear();
  s.readers.clear();
  s.pre.clear();
  s.group = -1;
}
// a task that names a datum more than once: reads and commutative writes together are an
// ordinary write
uint32_t merge_mode(uint32_t a, uint32_t b) {
  if (a == b) return a;
  return SPX_ACC_RW;
}
}  // namespace

int build_graph(uint32_t ntasks, const spx_access* acc, uint64_t nacc, const int32_t* priority, Graph& g) {
  g = Graph();
  g.ntasks = ntasks;
  std::unordered_map<uint64_t, DatumState> state;
  state.reserve(nacc / 2 + 16);
  std::vector<std::pair<uint32_t, uint32_t>> edges;  // (src, dst) while building
  edges.reserve(nacc * 2);
  std::vector<std::pair<uint64_t, uint32_t>> mine;  // this task's (datum, mode)
  std::vector<uint32_t> preds;
  std::vector<std::pair<uint32_t, uint32_t>> comm;  // (task, group << 6 | slot)
  std::vector<std::vector<uint32_t>> gmembers;      // per group: member tasks by slot
  uint64_t p = 0;
  for (uint32_t t = 0; t < ntasks; ++t) {
    mine.clear();
    while (p < nacc && acc[p].task == t) {
      if (acc[p].mode != SPX_ACC_R && acc[p].mode != SPX_ACC_RW && acc[p].mode != SPX_ACC_CW)
        return fail(SPX_EINVAL, "graph: bad access mode");
      mine.emplace_back(acc[p].datum, acc[p].mode);
      ++p;
    }
    if (p < nacc && acc[p].task < t) return fail(SPX_EINVAL, "graph: accesses not grouped by task in order");
    std::sort(mine.begin(), mine.end());
    preds.clear();
    for (size_t q = 0; q < mine.size(); ++q) {
      uint64_t d = mine[q].first;
      uint32_t mode = mine[q].second;
      while (q + 1 < mine.size() && mine[q + 1].first == d) {  // same datum named twice
        mode = merge_mode(mode, mine[q + 1].second);
        ++q;
      }
      DatumState& s = state[d];
      if (mode == SPX_ACC_CW) {
        if (s.group >= 0 && s.members.size() < (size_t)kGroupMax) {
          preds.insert(preds.end(), s.pre.begin(), s.pre.end());
        } else {
          close_group(s);  // a full group: the next one follows all its members
          s.pre = s.readers.empty() ? s.writers : s.readers;
          preds.insert(preds.end(), s.pre.begin(), s.pre.end());
          s.group = (int64_t)gmembers.size();
          gmembers.emplace_back();
        }
        comm.emplace_back(t, (uint32_t)(s.group << 6) | (uint32_t)s.members.size());
        gmembers[(size_t)s.group].push_back(t);
        s.members.push_back(t);
        continue;
      }
      close_group(s);
      if (mode == SPX_ACC_R) {
        preds.insert(preds.end(), s.writers.begin(), s.writers.end());
        s.readers.push_back(t);
      } else {
        const std::vector<uint32_t>& dep = s.readers.empty() ? s.writers : s.readers;
        preds.insert(preds.end(), dep.begin(), dep.end());
        s.readers.clear();
        s.writers.assign(1, t);
      }
    }
    std::sort(preds.begin(), preds.end());
    preds.erase(std::unique(preds.begin(), preds.end()), preds.end());
    for (uint32_t s : preds) edges.emplace_back(s, t);
  }
  if (p != nacc) return fail(SPX_EINVAL, "graph: access names a task index >= ntasks");
  if (gmembers.size() >= (1u << 26)) return fail(SPX_EINVAL, "graph: too many commutative groups");
  std::sort(edges.begin(), edges.end());  // by (src, dst)
  g.off.assign(ntasks + 1, 0);
  g.succ.resize(edges.size());
  g.indeg.assign(ntasks, 0);
  for (auto& e : edges) g.off[e.first + 1]++;
  for (uint32_t t = 0; t < ntasks; ++t) g.off[t + 1] += g.off[t];
  for (size_t e = 0; e < edges.size(); ++e) {
    g.succ[e] = edges[e].second;
    g.indeg[edges[e].second]++;
  }
  g.prio.assign(ntasks, 0);
  if (priority) std::copy(priority, priority + ntasks, g.prio.begin());
  if (!gmembers.empty()) {
    // comm is in task order; within a task, by datum, so sort each task's list by group
    g.ngroups = (uint32_t)gmembers.size();
    g.coff.assign(ntasks + 1, 0);
    for (auto& c : comm) g.coff[c.first + 1]++;
    for (uint32_t t = 0; t < ntasks; ++t) g.coff[t + 1] += g.coff[t];
    g.cent.resize(comm.size());
    for (size_t i = 0; i < comm.size(); ++i) g.cent[i] = comm[i].second;
    for (uint32_t t = 0; t < ntasks; ++t) std::sort(g.cent.begin() + g.coff[t], g.cent.begin() + g.coff[t + 1]);
    g.goff.assign(g.ngroups + 1, 0);
    for (uint32_t k = 0; k < g.ngroups; ++k) g.goff[k + 1] = g.goff[k] + (uint32_t)gmembers[k].size();
    g.gtask.resize(g.goff[g.ngroups]);
    g.gidx.resize(g.goff[g.ngroups]);
    for (uint32_t t = 0; t < ntasks; ++t)
      for (uint32_t i = g.coff[t]; i < g.coff[t + 1]; ++i) {
        const uint32_t grp = g.cent[i] >> 6, slot = g.cent[i] & 63u;
        g.gtask[g.goff[grp] + slot] = t;
        g.gidx[g.goff[grp] + slot] = i - g.coff[t];
      }
  }
  return SPX_OK;
}

// Right-looking tile Cholesky program (lower), optionally followed by one inversion task
// per diagonal tile and the block forward and backward substitution.  Datum ids: tile
// (i,j) -> i*nt + j; right-hand-side block k -> nt*nt + k; M_k = L_kk^{-T} -> nt*nt + nt + k.
// commute: the updates (SYRK and GEMM on their tile, FGEMM and BGEMM on their block of the
// right-hand sides) are commutative writes.
void cholesky_program(int nt, bool with_solve, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc,
                      bool with_inverse, int potrf_steps, bool commute) {
  tasks.clear();
  acc.clear();
  const uint32_t UPD = commute ? SPX_ACC_CW : SPX_ACC_RW;
  auto A = [nt](int i, int j) { return (uint64_t)i * (uint64_t)nt + (uint64_t)j; };
  auto B = [nt](int k) { return (uint64_t)nt * (uint64_t)nt + (uint64_t)k; };
  auto Minv = [nt](int k) { return (uint64_t)nt * (uint64_t)nt + (uint64_t)nt + (uint64_t)k; };
  // with the inversions, the diagonal solves write a second copy of the right-hand sides
  // (block k of Y2), so their rows can be split over workgroups; forward: FTRSM(k) reads
  // B(k), writes Y2(k); FGEMM(i,k) reads Y2(k), updates B(i).  Backward: BTRSM(k) reads
  // Y2(k), writes B(k); BGEMM(i,k) reads B(k), updates Y2(i).  The solution ends in B.
  auto Y2 = [nt](int k) { return (uint64_t)nt * (uint64_t)nt + 2 * (uint64_t)nt + (uint64_t)k; };
  auto task = [&](int type, int i, int j, int k) {
    TaskDesc d;
    d.type = (uint8_t)type;
    d.i = (uint16_t)i;
    d.j = (uint16_t)j;
    d.k = (uint16_t)k;
    tasks.push_back(d);
  };
  auto use = [&](uint32_t mode, uint64_t datum) {
    acc.push_back(spx_access{(uint32_t)(tasks.size() - 1), mode, datum});
  };
  for (int k = 0; k < nt; ++k) {
    // a diagonal factorization split into steps is a chain of tasks on the same tile
    for (int st = 0; st < potrf_steps; ++st) {
      task(SPX_T_POTRF, k, k, k);
      if (potrf_steps > 1) tasks.back().pad = (uint16_t)(st | (potrf_steps << 8));
      use(SPX_ACC_RW, A(k, k));
    }
    for (int i = k + 1; i < nt; ++i) {
      task(SPX_T_TRSM, i, k, k);
      use(SPX_ACC_R, A(k, k));
      use(SPX_ACC_RW, A(i, k));
    }
    for (int i = k + 1; i < nt; ++i) {
      task(SPX_T_SYRK, i, i, k);
      if (i == k + 1) tasks.back().pad = 1;  // on the critical path: cut into finer parts
      use(SPX_ACC_R, A(i, k));
      use(UPD, A(i, i));
      for (int j = k + 1; j < i; ++j) {
        task(SPX_T_GEMM, i, j, k);
        use(SPX_ACC_R, A(i, k));
        use(SPX_ACC_R, A(j, k));
        use(UPD, A(i, j));
      }
    }
  }
  if (with_inverse) {
    for (int k = 0; k < nt; ++k) {
      task(SPX_T_INV, k, k, k);
      use(SPX_ACC_R, A(k, k));
      use(SPX_ACC_RW, Minv(k));
    }
  }
  if (!with_solve) return;
  if (!with_inverse) {  // the paper's in-place substitution
    for (int k = 0; k < nt; ++k) {
      task(SPX_T_FTRSM, k, k, k);
      use(SPX_ACC_R, A(k, k));
      use(SPX_ACC_RW, B(k));
      for (int i = k + 1; i < nt; ++i) {
        task(SPX_T_FGEMM, i, k, k);
        use(SPX_ACC_R, A(i, k));
        use(SPX_ACC_R, B(k));
        use(UPD, B(i));
      }
    }
    for (int k = nt - 1; k >= 0; --k) {
      task(SPX_T_BTRSM, k, k, k);
      use(SPX_ACC_R, A(k, k));
      use(SPX_ACC_RW, B(k));
      for (int i = 0; i < k; ++i) {
        task(SPX_T_BGEMM, i, k, k);
        use(SPX_ACC_R, A(k, i));
        use(SPX_ACC_R, B(k));
        use(UPD, B(i));
      }
    }
    return;
  }
  for (int k = 0; k < nt; ++k) {
    task(SPX_T_FTRSM, k, k, k);
    tasks.back().pad = 1;  // the inverse-based, row-split variant
    use(SPX_ACC_R, Minv(k));
    use(SPX_ACC_R, B(k));
    use(SPX_ACC_RW, Y2(k));
    for (int i = k + 1; i < nt; ++i) {
      task(SPX_T_FGEMM, i, k, k);
      tasks.back().pad = 1;
      use(SPX_ACC_R, A(i, k));
      use(SPX_ACC_R, Y2(k));
      use(UPD, B(i));
    }
  }
  for (int k = nt - 1; k >= 0; --k) {
    task(SPX_T_BTRSM, k, k, k);
    tasks.back().pad = 1;
    use(SPX_ACC_R, Minv(k));
    use(SPX_ACC_R, Y2(k));
    use(SPX_ACC_RW, B(k));
    for (int i = 0; i < k; ++i) {
      task(SPX_T_BGEMM, i, k, k);
      tasks.back().pad = 1;
      use(SPX_ACC_R, A(k, i));
      use(SPX_ACC_R, B(k));
      use(UPD, Y2(i));
    }
  }
}

// The block substitution alone (L tiles and the M_k are only read): the tasks
// cholesky_program appends after the factor and the inversions, so its edges are the fused
// program's edges among those tasks.
void solve_program(int nt, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc, bool commute) {
  std::vector<TaskDesc> all;
  std::vector<spx_access> all_acc;
  cholesky_program(nt, true, all, all_acc, true, 1, commute);
  uint32_t first = 0;
  while (all[first].type != SPX_T_FTRSM) ++first;
  tasks.assign(all.begin() + first, all.end());
  acc.clear();
  for (const spx_access& a : all_acc)
    if (a.task >= first) acc.push_back(spx_access{a.task - first, a.mode, a.datum});
}

void gemm_program(int nt, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc, bool commute) {
  tasks.clear();
  acc.clear();
  const uint64_t n2 = (uint64_t)nt * (uint64_t)nt;
  for (int k = 0; k < nt; ++k)
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nt; ++j) {
        const uint32_t t = (uint32_t)tasks.size();
        TaskDesc d;
        d.type = SPX_T_MGEMM;
        d.i = (uint16_t)i;
        d.j = (uint16_t)j;
        d.k = (uint16_t)k;
        tasks.push_back(d);
        acc.push_back(spx_access{t, SPX_ACC_R, (uint64_t)i * nt + k});
        acc.push_back(spx_access{t, SPX_ACC_R, n2 + (uint64_t)k * nt + j});
        acc.push_back(spx_access{t, commute ? (uint32_t)SPX_ACC_CW : (uint32_t)SPX_ACC_RW, 2 * n2 + (uint64_t)i * nt + j});
      }
}

// Program of one matrix in a batched or served graph: LOAD writes every tile (and the
// right-hand-side blocks), so each tile's first update depends on it; STORE reads the
// solution blocks after the backward substitution.
void io_program(int nt, bool with_solve, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc,
                bool with_inverse, int potrf_steps, bool commute) {
  std::vector<TaskDesc> body;
  std::vector<spx_access> body_acc;
  cholesky_program(nt, with_solve, body, body_acc, with_inverse, potrf_steps, commute);
  auto A = [nt](int i, int j) { return (uint64_t)i * (uint64_t)nt + (uint64_t)j; };
  auto B = [nt](int k) { return (uint64_t)nt * (uint64_t)nt + (uint64_t)k; };
  tasks.clear();
  acc.clear();
  TaskDesc load;
  load.type = SPX_T_LOAD;
  load.i = (uint16_t)nt;  // parts: one per lower tile (plus one for the right-hand sides)
  tasks.push_back(load);
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j <= i; ++j) acc.push_back(spx_access{0, SPX_ACC_RW, A(i, j)});
  if (with_solve)
    for (int k = 0; k < nt; ++k) acc.push_back(spx_access{0, SPX_ACC_RW, B(k)});
  tasks.insert(tasks.end(), body.begin(), body.end());
  for (const spx_access& a : body_acc) acc.push_back(spx_access{a.task + 1, a.mode, a.datum});
  if (with_solve) {
    TaskDesc store;
    store.type = SPX_T_STORE;
    const uint32_t t = (uint32_t)tasks.size();
    tasks.push_back(store);
    for (int k = 0; k < nt; ++k) acc.push_back(spx_access{t, SPX_ACC_R, B(k)});
  }
}

void solve_io_program(int nt, std::vector<TaskDesc>& tasks, std::vector<spx_access>& acc, bool commute) {
  std::vector<TaskDesc> body;
  std::vector<spx_access> body_acc;
  solve_program(nt, body, body_acc, commute);
  auto B = [nt](int k) { return (uint64_t)nt * (uint64_t)nt + (uint64_t)k; };
  tasks.clear();
  acc.clear();
  TaskDesc load;
  load.type = SPX_T_LOAD;
  load.j = 1;  // right-hand sides only: one part
  tasks.push_back(load);
  for (int k = 0; k < nt; ++k) acc.push_back(spx_access{0, SPX_ACC_RW, B(k)});
  tasks.insert(tasks.end(), body.begin(), body.end());
  for (const spx_access& a : body_acc) acc.push_back(spx_access{a.task + 1, a.mode, a.datum});
  TaskDesc store;
  store.type = SPX_T_STORE;
  const uint32_t t = (uint32_t)tasks.size();
  tasks.push_back(store);
  for (int k = 0; k < nt; ++k) acc.push_back(spx_access{t, SPX_ACC_R, B(k)});
}

// Estimated latency of a task (parts in parallel), in units of one 512-tile update; only
// the ratios matter.  A step of a split POTRF is one of its b/32 column steps.
static double task_cost(const TaskDesc& d) {
  switch (d.type) {
    case SPX_T_POTRF: return (d.pad >> 8) ? 0.3 : 3.0;
    case SPX_T_TRSM: return 1.2;
    case SPX_T_SYRK:
    case SPX_T_GEMM:
    case SPX_T_INV:
    case SPX_T_MGEMM: return 1.0;
    case SPX_T_FGEMM:
    case SPX_T_BGEMM: return 0.3;
    case SPX_T_FTRSM:
    case SPX_T_BTRSM: return 0.15;
    default: return 0.2;
  }
}

// Default priorities of the library's programs (larger = sooner): the upward rank, i.e.
// the task's own latency plus the longest chain of latencies (tasks and hops) from it to
// the end of the graph, so that among the ready tasks the one with the most work still chained behind it
// runs first.  In the tile Cholesky this puts the panel chain first, then the updates by
// how soon their tile is consumed, and an early update of a tile that still has a long
// chain of updates ahead of it (the last diagonal tiles) before a late one of a short
// chain.  The class (priority >> 16, 0..63) grows linearly with the rank; the low bits
// keep the finer rank.  Two exceptions take class 0: LOAD (a new matrix of a batch starts
// when nothing urgent is ready) and the tiled product's updates (one bulk class: its
// chains are all alike, and bulk levels hand out several parts per claim).  Edges run
// from earlier to later tasks, so one pass in reverse insertion order computes every rank.
void rank_priorities(const std::vector<TaskDesc>& tasks, Graph& g) {
  const uint32_t T = g.ntasks;
  std::vector<double> r(T, 0.0);
  double mx = 0.0;
  // every edge also costs a hop (completion, push and pop: about a third of an update),
  // so of two chains with the same work the one with more hand-overs ranks higher
  constexpr double kHop = 0.3;
  for (uint32_t t = T; t-- > 0;) {
    double m = 0.0;
    for (uint64_t q = g.off[t]; q < g.off[t + 1]; ++q) m = std::max(m, kHop + r[g.succ[q]]);
    r[t] = task_cost(tasks[t]) + m;
    mx = std::max(mx, r[t]);
  }
  g.prio.assign(T, 0);
  if (mx <= 0.0) return;
  for (uint32_t t = 0; t < T; ++t) {
    const double f = r[t] / mx;  // (0, 1]
    const bool bulk = tasks[t].type == SPX_T_LOAD || tasks[t].type == SPX_T_MGEMM;
    const int cls = bulk ? 0 : std::min(kMaxLevels - 1, (int)(f * kMaxLevels));
    g.prio[t] = cls * 65536 + std::min(65535, (int)(f * 65535.0));
  }
}

}  // namespace spx

using namespace spx;

extern "C" {

int spx_graph_build(uint32_t ntasks, const spx_access* acc, uint64_t nacc, const int32_t* priority,
                    spx_graph** out) {
  if (!out || (nacc && !acc)) return fail(SPX_EINVAL, "spx_graph_build: null argument");
  *out = nullptr;
  try {
    std::unique_ptr<spx_graph> g(new spx_graph());
    int rc = build_graph(ntasks, acc, nacc, priority, g->g);
    if (rc) return rc;
    *out = g.release();
    return SPX_OK;
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_graph_build: out of host memory");
  }
}

int spx_graph_info(const spx_graph* g, uint32_t* ntasks, uint64_t* nedges) {
  if (!g) return fail(SPX_EINVAL, "spx_graph_info: null graph");
  if (ntasks) *ntasks = g->g.ntasks;
  if (nedges) *nedges = g->g.succ.size();
  return SPX_OK;
}

int spx_graph_edges(const spx_graph* g, uint32_t* src, uint32_t* dst, uint64_t cap) {
  if (!g || !src || !dst) return fail(SPX_EINVAL, "spx_graph_edges: null argument");
  if (cap < g->g.succ.size()) return fail(SPX_EINVAL, "spx_graph_edges: capacity too small");
  uint64_t e = 0;
  for (uint32_t t = 0; t < g->g.ntasks; ++t)
    for (uint64_t q = g->g.off[t]; q < g->g.off[t + 1]; ++q, ++e) {
      src[e] = t;
      dst[e] = g->g.succ[q];
    }
  return SPX_OK;
}

int spx_graph_indegree(const spx_graph* g, uint32_t* indeg, uint32_t cap) {
  if (!g || !indeg) return fail(SPX_EINVAL, "spx_graph_indegree: null argument");
  if (cap < g->g.ntasks) return fail(SPX_EINVAL, "spx_graph_indegree: capacity too small");
  std::copy(g->g.indeg.begin(), g->g.indeg.end(), indeg);
  return SPX_OK;
}

int spx_graph_to_dot(const spx_graph* g, const char* path) {
  if (!g || !path) return fail(SPX_EINVAL, "spx_graph_to_dot: null argument");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(SPX_EINVAL, "spx_graph_to_dot: cannot open file");
  static const char* names[] = {"POTRF", "TRSM", "SYRK", "GEMM", "FTRSM", "FGEMM", "BTRSM", "BGEMM", "LOAD", "STORE", "INV",
                                "MGEMM", "SPIN"};
  std::fprintf(f, "digraph spx {\n");
  for (uint32_t t = 0; t < g->g.ntasks; ++t) {
    if (t < g->tasks.size()) {
      const TaskDesc& d = g->tasks[t];
      std::fprintf(f, "  t%u [label=\"%s(%d,%d,%d) p%d\"];\n", t, d.type < 13 ? names[d.type] : "?", d.i, d.j, d.k,
                   g->g.prio[t]);
    } else {
      std::fprintf(f, "  t%u [label=\"t%u p%d\"];\n", t, t, g->g.prio[t]);
    }
  }
  for (uint32_t t = 0; t < g->g.ntasks; ++t)
    for (uint64_t q = g->g.off[t]; q < g->g.off[t + 1]; ++q) std::fprintf(f, "  t%u -> t%u;\n", t, g->g.succ[q]);
  std::fprintf(f, "}\n");
  std::fclose(f);
  return SPX_OK;
}

void spx_graph_destroy(spx_graph* g) { delete g; }

int spx_cholesky_graph(int32_t nt, int32_t with_solve, spx_graph** out, int32_t* task_types, uint32_t cap) {
  if (!out || nt < 1 || nt > 4096 || with_solve < 0 || with_solve > 0xffff || (with_solve & 0xf0))
    return fail(SPX_EINVAL, "spx_cholesky_graph: bad argument");
  const bool commute = (with_solve & 8) != 0;
  const int steps = (with_solve >> 8) ? (with_solve >> 8) : 1;  // POTRF steps, bits 8-15
  if (steps > 64) return fail(SPX_EINVAL, "spx_cholesky_graph: at most 64 POTRF steps");
  *out = nullptr;
  try {
    std::unique_ptr<spx_graph> g(new spx_graph());
    std::vector<spx_access> acc;
    if (with_solve & 2)
      io_program(nt, (with_solve & 1) != 0, g->tasks, acc, (with_solve & 4) != 0, steps, commute);
    else
      cholesky_program(nt, (with_solve & 1) != 0, g->tasks, acc, (with_solve & 4) != 0, steps, commute);
    int rc = build_graph((uint32_t)g->tasks.size(), acc.data(), acc.size(), nullptr, g->g);
    if (rc) return rc;
    rank_priorities(g->tasks, g->g);
    if (task_types) {
      if (cap < g->tasks.size()) return fail(SPX_EINVAL, "spx_cholesky_graph: capacity too small");
      for (size_t t = 0; t < g->tasks.size(); ++t) task_types[t] = g->tasks[t].type;
    }
    *out = g.release();
    return SPX_OK;
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_cholesky_graph: out of host memory");
  }
}

int spx_gemm_graph(int32_t nt, spx_graph** out, int32_t* task_types, uint32_t cap) {
  // nt | SPX_GEMM_COMMUTE: the updates of C_ij are commutative writes
  const bool commute = (nt & SPX_GEMM_COMMUTE) != 0;
  nt &= ~SPX_GEMM_COMMUTE;
  if (!out || nt < 1 || nt > 512) return fail(SPX_EINVAL, "spx_gemm_graph: bad argument");
  *out = nullptr;
  try {
    std::unique_ptr<spx_graph> g(new spx_graph());
    std::vector<spx_access> acc;
    gemm_program(nt, g->tasks, acc, commute);
    int rc = build_graph((uint32_t)g->tasks.size(), acc.data(), acc.size(), nullptr, g->g);
    if (rc) return rc;
    rank_priorities(g->tasks, g->g);
    if (task_types) {
      if (cap < g->tasks.size()) return fail(SPX_EINVAL, "spx_gemm_graph: capacity too small");
      for (size_t t = 0; t < g->tasks.size(); ++t) task_types[t] = g->tasks[t].type;
    }
    *out = g.release();
    return SPX_OK;
  } catch (const std::bad_alloc&) {
    return fail(SPX_ENOMEM, "spx_gemm_graph: out of host memory");
  }
}

}  // extern "C"
