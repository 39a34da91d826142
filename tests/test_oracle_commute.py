"""Pins of the oracle's commutative writes (Specx Sec. 4.1 SpCommutativeWrite, Sec. 4.7).

A commutative write is a read-modify-write whose order among the commutative writes of
the same datum inserted one after another does not matter; the runtime may run them in
any order, one at a time.  The oracle's pairwise edge rules are checked against things
fixed independently of them:
  * hand-derived edge lists of small programs (tests/golden/commute_edges.txt);
  * the semantics: the transitive closure of the oracle's edges equals the closure of
    the order a parallel run must keep (every two uses of a datum, at least one a write,
    stay ordered, except two commutative writes of one group), on random programs;
  * on one datum, the members of a group are mutually unordered (no path), so the
    reordering the mode allows is really there;
  * numerics: a sum of integers is exact in any order, so a commutative tiled product or
    Cholesky of integer data gives the plain program's bits in every order; on random
    data the commutative result differs from the plain one by no more than rounding;
  * a run order given back to the oracle reproduces its bits; an order that breaks an
    edge is refused.
Groups are cut every 63 members (a reading: the later cut adds order, never removes it).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import dag_brute

R, W, C = 1, 2, 3
HERE = os.path.dirname(__file__)


def load_golden():
    cases = []
    with open(os.path.join(HERE, "golden", "commute_edges.txt")) as f:
        cur = None
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, _, rest = line.partition(":")
            if key == "program":
                cur = {"acc": [], "edges": []}
                cases.append(cur)
                cur["n"] = int(rest)
            elif key == "use":
                t, m, d = rest.split()
                cur["acc"].append((int(t), {"R": R, "W": W, "C": C}[m], int(d)))
            elif key == "edges":
                cur["edges"] = [tuple(int(x) for x in p.split("-")) for p in rest.split()]
    return cases


@pytest.mark.parametrize("case", load_golden(), ids=lambda c: f"n{c['n']}_{len(c['acc'])}")
def test_hand_derived_edges(case):
    e, _ = oracle.dag_edges(case["n"], case["acc"])
    assert [tuple(x) for x in e.tolist()] == sorted(case["edges"])


def test_group_cut_at_63():
    # 65 commutative writes of one datum: members 0..62 form the first group, 63..64 the
    # second, which follows every member of the first
    acc = [(t, C, 1) for t in range(65)]
    e, _ = oracle.dag_edges(65, acc)
    want = sorted((a, b) for a in range(63) for b in (63, 64))
    assert [tuple(x) for x in e.tolist()] == want


def random_program(rs, ntasks, ndata, maxacc, modes=(R, W, C)):
    acc = []
    for t in range(ntasks):
        for _ in range(int(rs.integers(1, maxacc + 1))):
            acc.append((t, int(rs.choice(modes)), int(rs.integers(0, ndata))))
    return acc


@pytest.mark.parametrize("seed", range(120))
def test_closure_is_the_required_order(seed):
    rs = np.random.default_rng(9000 + seed)
    n = int(rs.integers(1, 36))
    acc = random_program(rs, n, int(rs.integers(1, 7)), 3)
    e, _ = oracle.dag_edges(n, acc)
    got = dag_brute.closure(n, [tuple(x) for x in e.tolist()])
    assert got == dag_brute.commutative_conflict_closure(n, acc)


@pytest.mark.parametrize("seed", range(40))
def test_one_datum_groups_are_unordered(seed):
    rs = np.random.default_rng(9500 + seed)
    n = int(rs.integers(2, 80))
    acc = [(t, int(rs.choice([R, W, C, C, C])), 5) for t in range(n)]
    e, _ = oracle.dag_edges(n, acc)
    reach = dag_brute.closure(n, [tuple(x) for x in e.tolist()])
    per, groups = dag_brute.commutative_groups(n, acc)
    for a in range(n):
        for b in range(a + 1, n):
            same = 5 in groups[a] and groups[a].get(5) == groups[b].get(5)
            if same:
                assert (a, b) not in reach, (a, b)
            elif per[a][5] != R or per[b][5] != R:
                assert (a, b) in reach, (a, b)


def test_gemm_commutative_program():
    T, e, _ = oracle.gemm_dag(4, commute=True)
    assert T == 64 and len(e) == 0  # every update of C_ij in one group: no order at all


def test_gemm_any_order_integer_exact():
    rs = np.random.default_rng(11)
    n, nb = 40, 8
    A = rs.integers(-9, 10, (n, n))
    B = rs.integers(-9, 10, (n, n))
    Cm = rs.integers(-99, 100, (n, n))
    want = (Cm + A @ B).astype(np.float64)
    for seed in range(4):
        got, order = oracle.gemm(A, B, Cm, nb, order=oracle.ORDER_RANDOM, seed=seed, commute=True,
                                 return_order=True)
        assert np.array_equal(got, want)
    # the orders really differ from the insertion order in the k of a tile
    ks = [t for t in order.tolist()]
    assert ks != sorted(ks)


def test_gemm_random_data_within_rounding_and_replay():
    rs = np.random.default_rng(12)
    n, nb = 48, 8
    A, B, Cm = rs.standard_normal((3, n, n))
    plain = oracle.gemm(A, B, Cm, nb)
    got, order = oracle.gemm(A, B, Cm, nb, order=oracle.ORDER_RANDOM, seed=3, commute=True, return_order=True)
    # each entry is C + the same n products summed in another order: |diff| <= 2 n u sum|terms|
    bound = 2 * n * 2.0 ** -53 * (np.abs(Cm) + np.abs(A) @ np.abs(B))
    assert (np.abs(got - plain) <= bound).all()
    assert not np.array_equal(got, plain)  # the order did change the rounding
    again = oracle.gemm(A, B, Cm, nb, order=oracle.ORDER_GIVEN, given=order, commute=True)
    assert np.array_equal(again, got)
    bad = order.copy()
    bad[[0, -1]] = bad[[-1, 0]]
    with pytest.raises(ValueError):
        oracle.gemm(A, B, Cm, nb, order=oracle.ORDER_GIVEN, given=bad)  # plain program: k order fixed


def test_cholesky_commutative_any_order():
    from paper_2308_15964_amd import inputs

    A, _, _, Bv = inputs.integer_factor(48, seed=4, nrhs=2)
    L0, X0, info0 = oracle.cholesky(A, 8, Bv)
    assert info0 == 0
    for seed in range(3):
        L, X, info = oracle.cholesky(A, 8, Bv, order=oracle.ORDER_RANDOM, seed=seed, commute=True)
        assert info == 0
        assert np.array_equal(L, L0) and np.array_equal(X, X0)
    rs = np.random.default_rng(13)
    G = rs.standard_normal((48, 48))
    S = G @ G.T / 48 + np.eye(48)
    L0, _, _ = oracle.cholesky(S, 8)
    L, _, _, order = oracle.cholesky(S, 8, order=oracle.ORDER_RANDOM, seed=5, commute=True, return_order=True)
    assert np.abs(L - L0).max() <= 1e-13 * np.abs(L0).max()
    L2, _, _ = oracle.cholesky(S, 8, order=oracle.ORDER_GIVEN, given=order, commute=True)
    assert np.array_equal(L2, L)


def test_commute_parallel_executor_refused():
    rs = np.random.default_rng(14)
    A, B, Cm = rs.standard_normal((3, 16, 16))
    with pytest.raises(RuntimeError):
        oracle.gemm(A, B, Cm, 4, nthreads=2, commute=True)
