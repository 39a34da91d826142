"""Pins of the oracle's tiled matrix product (the GEMM application, Specx Sec. 5.2).

The program is one task per tile triple (i, j, k), C_ij <- C_ij + A_ik B_kj, reading A_ik
and B_kj and writing C_ij.  Checked against things fixed independently of the oracle:
  * the literal brute force of the pairwise dependency definition (tiny programs);
  * closed forms derived by hand: nt^3 tasks; every C_ij is written by a chain of nt tasks
    and nothing reads it, so the edges are nt^2 (nt - 1) write-after-write edges and no
    others, nt^2 roots, every other task has in-degree 1, the longest path has nt tasks;
  * exact integer arithmetic (small integers keep every sum exact: C + A B equals
    numpy's integer product bit for bit);
  * tile-size invariance: each entry takes its m terms in increasing m whatever the tile
    size, so every b | n gives the unblocked result bit for bit, which is also the
    one-entry-at-a-time loop;
  * order invariance: every topological order gives the same bits; a DAG with one edge of
    a chain removed does not;
  * numpy's matmul (LAPACK-class library routine) within the rounding bound.
"""
import numpy as np
import pytest

import oracle
from oracle import dag_brute


@pytest.mark.parametrize("nt", [1, 2, 3, 4])
def test_dag_matches_brute_force(nt):
    tasks, acc = oracle.gemm_program(nt)
    T, e, kinds = oracle.gemm_dag(nt)
    want, wk = dag_brute.edges(T, acc)
    assert [tuple(x) for x in e.tolist()] == want
    assert kinds == wk


@pytest.mark.parametrize("nt", [1, 2, 5, 8])
def test_dag_closed_forms(nt):
    tasks, _ = oracle.gemm_program(nt)
    T, e, kinds = oracle.gemm_dag(nt)
    assert T == nt ** 3 == len(tasks)
    assert len(e) == nt * nt * (nt - 1)
    assert kinds["WAW"] == nt * nt * (nt - 1) and kinds["RAW"] == 0 and kinds["WAR"] == 0
    indeg = np.zeros(T, int)
    np.add.at(indeg, e[:, 1], 1)
    assert (indeg == 0).sum() == nt * nt and (indeg <= 1).all()
    # every edge joins consecutive k of the same (i, j)
    for s, d in e.tolist():
        (_, i1, j1, k1), (_, i2, j2, k2) = tasks[s], tasks[d]
        assert (i1, j1, k2) == (i2, j2, k1 + 1)
    # longest path: nt tasks
    depth = np.ones(T, int)
    for s, d in e.tolist():
        depth[d] = max(depth[d], depth[s] + 1)
    assert depth.max() == nt


def test_integer_exact():
    rs = np.random.default_rng(3)
    n = 48
    A = rs.integers(-9, 10, (n, n))
    B = rs.integers(-9, 10, (n, n))
    C = rs.integers(-99, 100, (n, n))
    want = (C + A @ B).astype(np.float64)
    for nb in (1, 6, 16, 48):
        assert np.array_equal(oracle.gemm(A, B, C, nb), want), nb


def test_tile_size_invariance_and_entries():
    rs = np.random.default_rng(4)
    n = 48
    A, B, C = rs.standard_normal((3, n, n))
    ref = oracle.gemm(A, B, C, n)
    for nb in (1, 2, 3, 4, 8, 12, 16, 24):
        assert np.array_equal(oracle.gemm(A, B, C, nb), ref), nb
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert np.array_equal(oracle.gemm_entries(A, B, C, ii.ravel(), jj.ravel()).reshape(n, n), ref)


def test_order_invariance_and_dropped_edge():
    rs = np.random.default_rng(5)
    n, nb = 48, 8
    A, B, C = rs.standard_normal((3, n, n))
    ref = oracle.gemm(A, B, C, nb)
    orders = set()
    for seed in range(12):
        out, od = oracle.gemm(A, B, C, nb, order=oracle.ORDER_RANDOM, seed=seed, return_order=True)
        assert np.array_equal(out, ref)
        orders.add(tuple(od))
    assert len(orders) >= 10
    out = oracle.gemm(A, B, C, nb, nthreads=4)
    assert np.array_equal(out, ref)
    # planted mistake: remove the edge between the k = 0 and k = 1 updates of C_00
    tasks, _ = oracle.gemm_program(n // nb)
    src, dst = tasks.index(("MGEMM", 0, 0, 0)), tasks.index(("MGEMM", 0, 0, 1))
    differs = 0
    for seed in range(30):
        out = oracle.gemm(A, B, C, nb, order=oracle.ORDER_RANDOM, seed=seed, drop_edge=(src, dst))
        differs += not np.array_equal(out, ref)
    assert differs > 0


def test_matches_numpy_within_rounding_bound():
    rs = np.random.default_rng(6)
    n, nb = 96, 32
    A, B, C = rs.standard_normal((3, n, n))
    out = oracle.gemm(A, B, C, nb)
    bound = (n + 1) * np.finfo(float).eps * (np.abs(C) + np.abs(A) @ np.abs(B))
    assert (np.abs(out - (C + A @ B)) <= bound).all()
