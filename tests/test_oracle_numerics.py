"""Pins of the oracle's arithmetic (tiled Cholesky and solve in FP64, Specx Sec. 5.2).

Nothing here re-types the oracle's formulas.  The oracle is checked against:
  * exact integer arithmetic: A = L0 L0^T with small-integer L0 and diagonal in {1,2,4}
    keeps every intermediate an exact integer, so L == L0 and X == X0 bit for bit (any
    dropped term, wrong index or transposed operand breaks exactness);
  * the textbook closed forms of the 2x2 and 3x3 Cholesky factors;
  * LAPACK through numpy (an independent library routine) on well-conditioned inputs;
  * a known factor (A = L0 L0^T with dominant positive diagonal);
  * invariants: every tile size gives the unblocked result bit for bit (I2); every
    topological order gives the same bits (I1), and a DAG with one edge removed does not;
  * leading principal minors in exact rational arithmetic for the failing pivot index;
  * closed-form residuals and backward errors for planted perturbations.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2308_15964_amd import inputs


def test_integer_factor_and_solve_are_exact():
    A, L0, X0, B = inputs.integer_factor(48, seed=11, nrhs=3)
    for nb in (1, 6, 16, 48):
        L, X, info = oracle.cholesky(A, nb, B)
        assert info == 0
        assert np.array_equal(L, L0)
        assert np.array_equal(X, X0)


def test_closed_form_2x2_and_3x3():
    a = np.array([[4.3, 0.0], [1.7, 3.1]])
    A = np.tril(a) + np.tril(a, -1).T
    L, _, _ = oracle.cholesky(A, 1)
    l11 = np.sqrt(4.3)
    l21 = 1.7 / l11
    l22 = np.sqrt(3.1 - l21 * l21)
    assert L[0, 0] == l11 and L[1, 0] == l21 and L[1, 1] == l22 and L[0, 1] == 0.0

    A = np.array([[5.0, 1.2, -0.7], [1.2, 4.0, 0.9], [-0.7, 0.9, 3.5]])
    L, _, _ = oracle.cholesky(A, 3)
    l11 = np.sqrt(5.0)
    l21, l31 = 1.2 / l11, -0.7 / l11
    l22 = np.sqrt(4.0 - l21 * l21)
    l32 = (0.9 - l31 * l21) / l22
    l33 = np.sqrt((3.5 - l31 * l31) - l32 * l32)
    assert np.array_equal(L, np.array([[l11, 0, 0], [l21, l22, 0], [l31, l32, l33]]))


@pytest.mark.parametrize("n,nb,maker", [(256, 32, "gram"), (512, 64, "shift"), (384, 128, "haar")])
def test_matches_lapack(n, nb, maker):
    if maker == "gram":
        A, B = inputs.gram_spd(n, seed=21, nrhs=2)
    elif maker == "shift":
        A, b = inputs.lower_plus_shift(n, seed=22)
        B = b[:, None]
    else:
        A, B = inputs.haar_spd(n, 10.0, seed=23, nrhs=2)
    L, X, info = oracle.cholesky(A, nb, B)
    assert info == 0
    Lr = np.linalg.cholesky(A)
    Xr = np.linalg.solve(A, B)
    assert np.linalg.norm(L - Lr) / np.linalg.norm(Lr) <= 1e-13
    assert np.linalg.norm(X - Xr) / np.linalg.norm(Xr) <= 1e-13


def test_known_factor():
    A, L0 = inputs.known_factor(256, seed=31)
    L, _, info = oracle.cholesky(A, 32)
    assert info == 0
    assert np.linalg.norm(L - L0) / np.linalg.norm(L0) <= 1e-12


def test_tile_size_invariance_bitwise():
    """I2: in-place, m-ascending tile kernels give the unblocked result for every b | n."""
    n = 48
    A, B = inputs.gram_spd(n, seed=41, nrhs=2)
    L1, X1, _ = oracle.cholesky(A, n, B)  # one tile: the unblocked algorithm
    for nb in (1, 2, 3, 4, 6, 8, 12, 16, 24):
        L, X, info = oracle.cholesky(A, nb, B)
        assert info == 0
        assert np.array_equal(L, L1), nb
        assert np.array_equal(X, X1), nb


def test_order_invariance_bitwise():
    """I1: every topological order gives the sequential result bit for bit."""
    A, B = inputs.gram_spd(96, seed=51, nrhs=2)
    L0, X0, _, ord0 = oracle.cholesky(A, 16, B, return_order=True)
    orders = {tuple(ord0)}
    for seed in range(20):
        L, X, info, od = oracle.cholesky(A, 16, B, order=oracle.ORDER_RANDOM, seed=seed, return_order=True)
        assert info == 0
        assert np.array_equal(L, L0) and np.array_equal(X, X0)
        orders.add(tuple(od))
    L, X, _ = oracle.cholesky(A, 16, B, order=oracle.ORDER_PRIORITY)
    assert np.array_equal(L, L0) and np.array_equal(X, X0)
    assert len(orders) >= 15  # the random orders really differ


def test_dropped_edge_breaks_invariance():
    """Planted mistake: without the TRSM(1,0) -> SYRK(1,0) edge some order reads the tile
    before it is solved, so at least one random order must change the result."""
    tasks, _ = oracle.cholesky_program(6, True)
    src = tasks.index(("TRSM", 1, 0, 0))
    dst = tasks.index(("SYRK", 1, 1, 0))
    A, B = inputs.gram_spd(96, seed=52, nrhs=1)
    L0, X0, _ = oracle.cholesky(A, 16, B)
    differs = 0
    for seed in range(20):
        L, X, _ = oracle.cholesky(A, 16, B, order=oracle.ORDER_RANDOM, seed=seed, drop_edge=(src, dst))
        differs += not (np.array_equal(L, L0) and np.array_equal(X, X0))
    assert differs > 0


def test_parallel_executor_bitwise_equal():
    A, B = inputs.gram_spd(256, seed=61, nrhs=3)
    L0, X0, _ = oracle.cholesky(A, 32, B)
    for th in (2, 4, 8):
        L, X, info = oracle.cholesky(A, 32, B, nthreads=th)
        assert info == 0 and np.array_equal(L, L0) and np.array_equal(X, X0)


def first_bad_minor(M):
    """1-based index of the first leading principal minor that is not positive, computed
    with exact rationals (Gaussian elimination without pivoting); 0 if all are positive."""
    n = len(M)
    a = [[Fraction(int(M[i][j])) for j in range(n)] for i in range(n)]
    det = Fraction(1)
    for k in range(n):
        piv = a[k][k]
        det_k = det * piv
        if det_k <= 0:
            return k + 1
        det = det_k
        for i in range(k + 1, n):
            f = a[i][k] / piv
            for j in range(k, n):
                a[i][j] -= f * a[k][j]
    return 0


@pytest.mark.parametrize("seed", range(6))
def test_failing_pivot_index(seed):
    rs = np.random.default_rng(70 + seed)
    n = 24
    M = rs.integers(-2, 3, (n, n)).astype(np.float64)
    M = np.tril(M) + np.tril(M, -1).T
    M[np.diag_indices(n)] = rs.integers(3, 9, n)
    bad = int(rs.integers(1, n))
    M[bad, bad] = -5.0  # leading minor bad+1 turns non-positive at the latest
    want = first_bad_minor(M)
    assert want != 0
    for nb in (1, 4, 8, 24):
        _, _, info = oracle.cholesky(M, nb)
        assert info == want, (nb, info, want)


def test_dot2_recovers_cancelled_terms():
    x = np.array([1e16, 1.0, -1e16, 3.0])
    y = np.ones(4)
    assert sum(x * y) != 4.0  # plain summation loses the 1
    assert oracle.dot2(x, y) == 4.0
    # an exact product error: (1 + 2^-30)^2 = 1 + 2^-29 + 2^-60, and 1 is then subtracted
    e = 1.0 + 2.0 ** -30
    assert oracle.dot2(np.array([e, -1.0]), np.array([e, 1.0])) == 2.0 ** -29 + 2.0 ** -60


def test_backward_error_closed_form():
    n = 16
    A = np.eye(n)
    b = np.linspace(-1.0, 2.0, n)
    assert oracle.backward_error(A, b, b)[0] == 0.0
    x = b.copy()
    x[5] += 0.25  # r = -0.25 e_5 exactly
    eta = oracle.backward_error(A, x, b)[0]
    assert eta == 0.25 / (1.0 * np.abs(x).max() + np.abs(b).max())
    # ||A||_inf of a symmetric matrix from its lower triangle
    M = np.array([[2.0, -1.0, 0.5], [-1.0, 3.0, 4.0], [0.5, 4.0, -1.0]])
    assert oracle.norm_inf(M) == 8.0


def test_factor_residual_closed_form():
    A, L0, _, _ = inputs.integer_factor(20, seed=81, nrhs=1)
    assert oracle.factor_residual(A, L0) == 0.0
    # the probe rounds w = L^T v once, so an exact factor shows only that rounding
    assert oracle.factor_residual_probe(A, L0, nvec=4) <= 1e-15
    L = L0.copy()
    L[7, 3] += 0.5
    # entries (7,j) for j >= 3 and (i,7) change: compare with the plainly formed residual
    R = A - L @ L.T  # exact: half-integers of modest size
    want = np.linalg.norm(R) / np.linalg.norm(A)
    assert abs(oracle.factor_residual(A, L) - want) <= 1e-15 * want


def test_entry_check_closed_form():
    """A = [[4, 2], [2, 10]] has the factor [[2, 0], [1, 3]].  With L(1,0) = 1.5 instead,
    entry (1,0) of A - L L^T is 2 - 3 = -1 and entry (1,1) is 10 - (2.25 + 9) = -1.25;
    relative to sqrt(A_ii A_jj) they are 1/sqrt(40) and 1.25/10 exactly."""
    A = np.array([[4.0, 2.0], [2.0, 10.0]])
    L = np.array([[2.0, 0.0], [1.5, 3.0]])
    one = lambda i, j: oracle.entry_check(A, L, np.array([i]), np.array([j]))
    assert one(0, 0) == 0.0
    assert one(1, 0) == 1.0 / np.sqrt(40.0)
    assert one(0, 1) == 1.0 / np.sqrt(40.0)  # an upper index pair is read as its mirror
    assert one(1, 1) == 0.125
    assert oracle.entry_check(A, L, np.array([0, 1, 1]), np.array([0, 1, 0])) == 1.0 / np.sqrt(40.0)
    assert oracle.entry_check(A, np.array([[2.0, 0.0], [1.0, 3.0]]), np.array([1, 1]), np.array([0, 1])) == 0.0


def _exact_residual_entry(A, L, i, j):
    """A_ij - sum_{m <= min(i, j)} L_im L_jm in exact rational arithmetic."""
    from fractions import Fraction as Fr

    i, j = max(i, j), min(i, j)
    return Fr(float(A[i, j])) - sum(Fr(float(L[i, m])) * Fr(float(L[j, m])) for m in range(j + 1))


@pytest.mark.parametrize("seed", range(3))
def test_entry_check_matches_exact_arithmetic(seed):
    """Sampled entries of A - L L^T for a factor with planted half-integer errors, against
    the same quantity formed in exact rationals (only the final sqrt and division round)."""
    A, L0, _, _ = inputs.integer_factor(24, seed=90 + seed, nrhs=1)
    rs = np.random.default_rng(seed)
    L = L0.copy()
    for _ in range(4):
        i = int(rs.integers(1, 24))
        L[i, int(rs.integers(0, i + 1))] += 0.5 * int(rs.choice([-3, -1, 1, 3]))
    ii = rs.integers(0, 24, 40)
    jj = rs.integers(0, 24, 40)
    want = 0.0
    for i, j in zip(ii, jj):
        one = oracle.entry_check(A, L, np.array([i]), np.array([j]))
        exact = abs(float(_exact_residual_entry(A, L, int(i), int(j)))) / np.sqrt(A[i, i] * A[j, j])
        assert abs(one - exact) <= 4 * np.finfo(float).eps * exact, (i, j, one, exact)
        want = max(want, exact)
    assert abs(oracle.entry_check(A, L, ii, jj) - want) <= 4 * np.finfo(float).eps * want
    assert want > 0.0


def test_residual_probe_closed_forms():
    """For A = a I and L = l I every vector gives |a - l^2| / a: 1/3 for (3, 2), and
    0.5625 for (4, 2.5), whatever vectors the probe draws."""
    n = 50
    assert abs(oracle.factor_residual_probe(3.0 * np.eye(n), 2.0 * np.eye(n), nvec=3) - 1.0 / 3.0) <= 1e-15
    assert abs(oracle.factor_residual_probe(4.0 * np.eye(n), 2.5 * np.eye(n), nvec=3) - 0.5625) <= 1e-15
    assert oracle.factor_residual_probe(4.0 * np.eye(n), 2.0 * np.eye(n), nvec=3) == 0.0


def test_residual_vectors_match_exact_arithmetic():
    """||(A - L L^T) v|| / ||A v|| on dyadic vectors and a factor with planted half-integer
    errors: every intermediate is exact, so the value equals the exact rational ratio's
    square root up to the final sqrt and division."""
    from fractions import Fraction as Fr

    n = 16
    A, L0, _, _ = inputs.integer_factor(n, seed=97, nrhs=1)
    L = L0.copy()
    L[9, 4] += 0.5
    L[13, 13] -= 1.5
    rs = np.random.default_rng(5)
    V = rs.integers(-16, 17, (n, 3)) / 8.0
    ratios = []
    for q in range(3):
        v = [Fr(float(x)) for x in V[:, q]]
        Af = [[Fr(float(A[i, j])) for j in range(n)] for i in range(n)]
        Lf = [[Fr(float(L[i, j])) for j in range(n)] for i in range(n)]
        Av = [sum(Af[i][j] * v[j] for j in range(n)) for i in range(n)]
        w = [sum(Lf[i][m] * v[i] for i in range(n)) for m in range(n)]  # L^T v
        LLv = [sum(Lf[i][m] * w[m] for m in range(n)) for i in range(n)]
        num = sum((Av[i] - LLv[i]) ** 2 for i in range(n))
        den = sum(x * x for x in Av)
        ratios.append(np.sqrt(float(num)) / np.sqrt(float(den)))
        got = oracle.factor_residual_vectors(A, L, V[:, q])
        assert abs(got - ratios[-1]) <= 4 * np.finfo(float).eps * ratios[-1], (q, got, ratios[-1])
    assert abs(oracle.factor_residual_vectors(A, L, V) - max(ratios)) <= 4 * np.finfo(float).eps * max(ratios)
    assert oracle.factor_residual_vectors(A, L0, V) == 0.0


def test_backward_error_matches_exact_arithmetic():
    """eta per column for an integer SPD matrix and dyadic x, b: the residual, the norms and
    the maxima are exact, so eta equals the exact ratio up to its final division."""
    from fractions import Fraction as Fr

    n = 12
    A, _, _, _ = inputs.integer_factor(n, seed=99, nrhs=1)
    rs = np.random.default_rng(6)
    X = rs.integers(-40, 41, (n, 3)) / 16.0
    B = rs.integers(-40, 41, (n, 3)) / 4.0
    anorm = max(sum(abs(Fr(float(A[i, j]))) for j in range(n)) for i in range(n))
    eta = oracle.backward_error(A, X, B)
    for q in range(3):
        r = [Fr(float(B[i, q])) - sum(Fr(float(A[i, j])) * Fr(float(X[j, q])) for j in range(n)) for i in range(n)]
        want = float(max(abs(x) for x in r)) / float(anorm * max(abs(Fr(float(x))) for x in X[:, q]) +
                                                     max(abs(Fr(float(x))) for x in B[:, q]))
        assert abs(eta[q] - want) <= 2 * np.finfo(float).eps * want, (q, eta[q], want)
