"""Pins of the oracle's dependency inference (STF, Specx Sec. 2.1 / Sec. 4.1 / Sec. 4.7).

The oracle's C enumeration is checked against things fixed independently of it:
  * a literal pure-Python brute force of the pairwise definition (tiny programs);
  * closed forms derived by hand for the right-looking tile Cholesky program:
      tasks   T(nt) = nt + 2 C(nt,2) + C(nt,3)
      RAW     POTRF(k)->TRSM(i,k): C(nt,2); TRSM(i,k)->SYRK(i,k): C(nt,2);
              TRSM->GEMM (two per GEMM): 2 C(nt,3)
      WAW     chain SYRK(i,0..i-1)->POTRF(i): C(nt,2); chain GEMM(i,j,0..j-1)->TRSM(i,j): C(nt,3)
      WAR     none (every tile is only read after its last write)
      => E(nt) = 3 C(nt,2) + 3 C(nt,3); critical path 3 nt - 2 tasks;
      with the block solve appended, WAR = C(nt,2): each forward reader FGEMM(i,k) of
      block k precedes the first backward writer of block k, BGEMM(k, nt-1);
  * a hand-derived golden edge list (tests/golden/dag_nt2_solve.txt);
  * equality of transitive closures with the full conflict relation.
"""
import os
from math import comb

import numpy as np
import pytest

import oracle
from oracle import dag_brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_program(rs, ntasks, ndata, maxacc):
    acc = []
    for t in range(ntasks):
        for _ in range(rs.integers(1, maxacc + 1)):
            acc.append((t, int(rs.choice([1, 2])), int(rs.integers(0, ndata))))
    return acc


@pytest.mark.parametrize("seed", range(60))
def test_random_programs_match_brute_force(seed):
    rs = np.random.default_rng(1000 + seed)
    ntasks = int(rs.integers(1, 15))
    acc = random_program(rs, ntasks, int(rs.integers(1, 6)), 3)
    e, kinds = oracle.dag_edges(ntasks, acc)
    be, bkinds = dag_brute.edges(ntasks, acc)
    assert [tuple(x) for x in e.tolist()] == be
    assert kinds == bkinds
    # every edge points forward (acyclic), and the closure is the full conflict closure
    assert all(a < b for a, b in be)
    assert dag_brute.closure(ntasks, be) == dag_brute.conflict_closure(ntasks, acc)


@pytest.mark.parametrize("nt", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("with_solve", [False, True])
def test_cholesky_program_matches_brute_force(nt, with_solve):
    tasks, acc = oracle.cholesky_program(nt, with_solve)
    e, kinds = oracle.dag_edges(len(tasks), acc)
    be, bkinds = dag_brute.edges(len(tasks), acc)
    assert [tuple(x) for x in e.tolist()] == be
    assert kinds == bkinds
    assert dag_brute.closure(len(tasks), be) == dag_brute.conflict_closure(len(tasks), acc)


@pytest.mark.parametrize("nt", list(range(1, 13)) + [32])
def test_cholesky_closed_forms(nt):
    T, e, kinds = oracle.cholesky_dag(nt)
    assert T == nt + 2 * comb(nt, 2) + comb(nt, 3)
    assert len(e) == 3 * comb(nt, 2) + 3 * comb(nt, 3)
    assert kinds == {"RAW": 2 * comb(nt, 2) + 2 * comb(nt, 3), "WAR": 0, "WAW": comb(nt, 2) + comb(nt, 3)}


@pytest.mark.parametrize("nt", [2, 3, 8, 32])
def test_fused_solve_closed_forms(nt):
    T, e, kinds = oracle.cholesky_dag(nt, with_solve=True)
    assert T == nt + 2 * comb(nt, 2) + comb(nt, 3) + 2 * (nt + comb(nt, 2))
    assert kinds["WAR"] == comb(nt, 2)
    assert all(a < b for a, b in e.tolist())


def test_indegree_histogram_nt8():
    tasks, _ = oracle.cholesky_program(8)
    T, e, _ = oracle.cholesky_dag(8)
    indeg = np.bincount(e[:, 1], minlength=T)
    hist = {}
    for (name, *_), d in zip(tasks, indeg):
        hist.setdefault(name, {}).setdefault(int(d), 0)
        hist[name][int(d)] += 1
    assert hist == {"POTRF": {0: 1, 1: 7}, "TRSM": {1: 7, 2: 21}, "SYRK": {1: 7, 2: 21}, "GEMM": {2: 21, 3: 35}}
    assert int((indeg == 0).sum()) == 1 and tasks[int(np.argmin(indeg))][0] == "POTRF"


@pytest.mark.parametrize("nt", [1, 2, 8, 32])
def test_critical_path(nt):
    T, e, _ = oracle.cholesky_dag(nt)
    depth = np.ones(T, np.int64)
    for a, b in e.tolist():  # sorted by src; edges point forward
        depth[b] = max(depth[b], depth[a] + 1)
    assert depth.max() == 3 * nt - 2


def test_golden_nt2_with_solve():
    rows = []
    with open(os.path.join(GOLDEN, "dag_nt2_solve.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a, b, k = line.split()
                rows.append((int(a), int(b), k))
    tasks, acc = oracle.cholesky_program(2, True)
    assert [t[0] for t in tasks] == ["POTRF", "TRSM", "SYRK", "POTRF", "FTRSM", "FGEMM", "FTRSM", "BTRSM",
                                     "BGEMM", "BTRSM"]
    e, kinds = oracle.dag_edges(len(tasks), acc)
    assert [tuple(x) for x in e.tolist()] == [(a, b) for a, b, _ in rows]
    want = {"RAW": 0, "WAR": 0, "WAW": 0}
    for _, _, k in rows:
        want[k] += 1
    assert kinds == want


def test_duplicate_access_in_one_task_uses_stronger_mode():
    # task 0 names datum 7 twice (read, then write); task 1 reads it: one RAW edge
    e, kinds = oracle.dag_edges(2, [(0, 1, 7), (0, 2, 7), (1, 1, 7)])
    assert e.tolist() == [[0, 1]] and kinds == {"RAW": 1, "WAR": 0, "WAW": 0}


def test_invalid_access_rejected():
    with pytest.raises(ValueError):
        oracle.dag_edges(1, [(3, 1, 0)])
    with pytest.raises(ValueError):
        oracle.dag_edges(1, [(0, 5, 0)])
