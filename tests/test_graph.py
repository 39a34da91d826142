"""The product's STF graph builder (per-datum last writer / readers, host C++) against the
oracle's pairwise definition of the dependency edges (Specx Sec. 2.1, Sec. 4.1, Sec. 4.7).
Integer work: the edge sets must be identical."""
import os
from math import comb

import numpy as np
import pytest

import oracle
from paper_2308_15964_amd import spx


def random_program(rs, ntasks, ndata, maxacc):
    acc = []
    for t in range(ntasks):
        for _ in range(rs.integers(1, maxacc + 1)):
            acc.append((t, int(rs.choice([1, 2])), int(rs.integers(0, ndata))))
    return acc


@pytest.mark.parametrize("seed", range(200))
def test_random_programs_bit_exact(seed):
    rs = np.random.default_rng(5000 + seed)
    ntasks = int(rs.integers(1, 40))
    acc = random_program(rs, ntasks, int(rs.integers(1, 12)), 4)
    want, _ = oracle.dag_edges(ntasks, acc)
    g = spx.Graph.build(ntasks, acc)
    got = g.edges()
    assert np.array_equal(got, want)
    assert np.array_equal(g.indegree(), np.bincount(want[:, 1], minlength=ntasks).astype(np.uint32))


@pytest.mark.parametrize("nt", [1, 2, 3, 5, 8, 13, 32])
@pytest.mark.parametrize("with_solve", [False, True])
def test_cholesky_graph_bit_exact(nt, with_solve):
    T, want, _ = oracle.cholesky_dag(nt, with_solve)
    g = spx.Graph.cholesky(nt, with_solve)
    assert g.info() == (T, len(want))
    assert np.array_equal(g.edges(), want)
    tasks, _ = oracle.cholesky_program(nt, with_solve)
    assert [spx.TASK_NAMES[t] for t in g.task_types] == [t[0] for t in tasks]


def test_cholesky_graph_nt64_counts():
    nt = 64
    g = spx.Graph.cholesky(nt)
    T, E = g.info()
    assert T == nt + 2 * comb(nt, 2) + comb(nt, 3) == 45760
    assert E == 3 * comb(nt, 2) + 3 * comb(nt, 3) == 131040
    e = g.edges()
    assert (e[:, 0] < e[:, 1]).all()


def test_priorities_and_dot(tmp_path):
    g = spx.Graph.build(3, [(0, 2, 5), (1, 1, 5), (2, 2, 5)], priority=[3, 1, 2])
    assert g.edges().tolist() == [[0, 1], [1, 2]]
    p = tmp_path / "g.dot"
    g.to_dot(str(p))
    text = p.read_text()
    assert text.startswith("digraph") and "t0 -> t1;" in text and "t1 -> t2;" in text
    gc = spx.Graph.cholesky(2)
    gc.to_dot(str(p))
    text = p.read_text()
    assert 'POTRF(0,0,0)' in text and "t2 -> t3;" in text


def test_invalid_inputs_rejected():
    with pytest.raises(spx.SpxError) as e:
        spx.Graph.build(2, [(0, 3, 1)])
    assert e.value.code == spx.SPX_EINVAL
    with pytest.raises(spx.SpxError):
        spx.Graph.build(2, [(5, 1, 1)])
    with pytest.raises(spx.SpxError):
        spx.Graph.build(3, [(1, 1, 1), (0, 1, 1)])  # not grouped in task order
    with pytest.raises(spx.SpxError):
        spx.Graph.cholesky(0)


def test_empty_graph():
    g = spx.Graph.build(0, [])
    assert g.info() == (0, 0)
    g = spx.Graph.build(4, [])
    assert g.info() == (4, 0) and g.indegree().tolist() == [0, 0, 0, 0]
