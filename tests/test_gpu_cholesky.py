"""GPU parity of the tile-DAG Cholesky factorisation and solve (Specx Sec. 5.2) against the
oracle, through the C ABI.

Tolerances (FP64; the device uses fused multiply-add and matrix-core accumulation, the
oracle separately rounded products, so results agree to rounding, not bit for bit):
  factor:  |L_ij - Lo_ij| <= 1e-12 sqrt(A_ii)  (row i of L has 2-norm sqrt(A_ii))
           and ||L - Lo||_F <= 1e-12 ||Lo||_F
  solve:   |x_iq - xo_iq| <= 1e-12 ||xo_q||_inf (well-conditioned inputs, kappa <= 5)
           and the normwise backward error eta <= 1e-14.
Integer-valued inputs (unit-diagonal factor with entries in {-1,0,1}) are exact on both
sides: every product and sum, and every entry of the inverted 32x32 diagonal blocks the
device multiplies by, is an integer below 2^53, so the device factor must equal the known
factor bit for bit, and with 32-wide tiles the solution too.
"""
import numpy as np
import pytest

import oracle
from paper_2308_15964_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_15964_amd import spx

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = spx.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def host(t):
    return t.cpu().numpy()


def oracle_tile(n):
    """A tile size dividing n for the oracle (every valid tile gives the same bits)."""
    for nb in (64, 50, 48, 40, 32, 25, 24, 20, 16, 10, 8, 5, 4, 2, 1):
        if n % nb == 0:
            return nb
    return 1


def check_factor(A, L, Lo, tol=1e-12):
    d = np.sqrt(np.diag(A))
    err = np.abs(L - Lo)
    assert (err <= tol * d[:, None]).all(), float((err / d[:, None]).max())
    assert np.linalg.norm(L - Lo) <= tol * np.linalg.norm(Lo)
    assert np.all(np.triu(L, 1) == 0)


def check_solve(X, Xo, eta_o, tol=1e-12):
    X = X.reshape(Xo.shape)
    scale = np.abs(Xo).max(axis=0)
    assert (np.abs(X - Xo) <= tol * scale).all(), float((np.abs(X - Xo) / scale).max())
    assert (eta_o <= 1e-14).all(), eta_o


CASES = [(32, 32, 1), (64, 32, 2), (100, 32, 3), (128, 64, 9), (200, 64, 1), (256, 128, 4), (384, 128, 1),
         (500, 128, 2), (512, 256, 1), (512, 512, 3), (700, 256, 1), (1536, 512, 2), (1100, 256, 2),
         (2100, 512, 1)]


@pytest.mark.parametrize("n,b,nrhs", CASES)
def test_factor_and_solve_parity(ctx, n, b, nrhs):
    print(f"case n={n} b={b} nrhs={nrhs}", flush=True)
    A, B = inputs.gram_spd(n, seed=100 + n + b, nrhs=nrhs)
    Lo, Xo, info = oracle.cholesky(A, oracle_tile(n), B)
    assert info == 0
    Ad, Bd = dev(A), dev(B)
    F = ctx.potrf(Ad, tile=b)
    L = host(F.L())
    check_factor(A, L, Lo)
    X = host(ctx.potrs(F, Bd))
    eta = oracle.backward_error(A, X, B)
    check_solve(X, Xo, eta)
    # the device residual is plain FP64: it agrees with the compensated one to within its
    # own rounding error, about n u relative to ||A|| ||x||
    eta_dev = ctx.backward_error(Ad, dev(X), Bd)
    assert (np.abs(eta_dev - eta) <= 2.0 * n * 2.0 ** -53).all(), (eta_dev, eta)
    F.close()


def test_config1_parity(ctx):
    """N=1024, tile 128 (8x8 tiles, 120 factor tasks), A = L0 L0^T + N I, one right-hand side."""
    n, b = 1024, 128
    A, bvec = inputs.lower_plus_shift(n, seed=1)
    Lo, xo, info = oracle.cholesky(A, b, bvec)
    assert info == 0
    F = ctx.potrf(dev(A), tile=b)
    st = ctx.stats()
    assert st["ntasks"] == 120 + 8 and st["tile"] == 128  # the program + one inversion per diagonal tile
    check_factor(A, host(F.L()), Lo)
    x = host(ctx.potrs(F, dev(bvec)))
    check_solve(x[:, None], xo[:, None], oracle.backward_error(A, x, bvec))
    assert ctx.stats()["ntasks"] == 72  # solve tasks 2(nt + C(nt,2))
    F.close()


@pytest.mark.parametrize("n,b", [(96, 32), (100, 32), (200, 64), (640, 128)])
def test_integer_inputs_exact(ctx, n, b):
    # The factor is exact for every tile size.  The solve multiplies by the inverse of each
    # diagonal tile: for 32-wide tiles that inverse is the 32x32 block inverse, an integer
    # matrix below 2^31, so the solution is exact too; inverses of wider unit-triangular
    # integer tiles can outgrow 2^53, so there only the factor is pinned bit for bit.
    A, L0, X0, B = inputs.integer_factor(n, seed=n, nrhs=3, unit=True)
    F = ctx.potrf(dev(A), tile=b)
    assert np.array_equal(host(F.L()), L0)
    if b == 32:
        assert np.array_equal(host(ctx.potrs(F, dev(B))), X0)
    F.close()


def test_schedules_bitwise_identical(ctx):
    """Every tile's updates are chained in insertion order, so any schedule gives the
    same bits: FIFO vs priority queues, and different numbers of workgroups."""
    from paper_2308_15964_amd import spx

    A, B = inputs.gram_spd(1024, seed=9, nrhs=2)
    Ad, Bd = dev(A), dev(B)
    ref_L = ref_X = None
    for policy, nwg in [(spx.Q_PRIORITY, 0), (spx.Q_FIFO, 0), (spx.Q_PRIORITY, 7), (spx.Q_FIFO, 1), (spx.Q_PRIORITY, 61),
                        (spx.Q_SHARDED, 0), (spx.Q_SHARDED, 13)]:
        F = ctx.potrf(Ad, tile=128, queue_policy=policy, num_wg=nwg)
        L = host(F.L())
        X = host(ctx.potrs(F, Bd))
        if ref_L is None:
            ref_L, ref_X = L, X
        assert np.array_equal(L, ref_L) and np.array_equal(X, ref_X), (policy, nwg)
        F.close()


def test_trace_respects_every_edge(ctx):
    """Device timestamps: every part of a task ends before any part of a successor starts,
    and every part runs exactly once."""
    from paper_2308_15964_amd import spx

    n, b = 1024, 128
    A, _ = inputs.gram_spd(n, seed=11)
    F = ctx.potrf(dev(A), tile=b, flags=spx.F_TRACE)
    tr = ctx.trace()
    st = ctx.stats()
    assert len(tr) == st["nparts"]
    task = tr[:, 0].astype(np.int64)
    part = (tr[:, 1] & 0xFFFF).astype(np.int64)
    assert len(set(zip(task.tolist(), part.tolist()))) == len(tr)
    T = st["ntasks"]
    start = np.full(T, np.iinfo(np.int64).max)
    end = np.zeros(T, np.int64)
    np.minimum.at(start, task, tr[:, 2].astype(np.int64))
    np.maximum.at(end, task, tr[:, 3].astype(np.int64))
    g = spx.Graph.cholesky(n // b)
    e = g.edges()
    assert (end[e[:, 0]] <= start[e[:, 1]]).all()
    F.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_not_positive_definite(ctx, seed):
    from paper_2308_15964_amd import spx

    rs = np.random.default_rng(300 + seed)
    n = 300
    A, _ = inputs.gram_spd(n, seed=400 + seed)
    bad = int(rs.integers(40, n - 1))
    A[bad, bad] = -1.0
    _, _, info = oracle.cholesky(A, oracle_tile(n))
    assert info > 0
    with pytest.raises(spx.NotPositiveDefinite) as e:
        ctx.potrf(dev(A), tile=64)
    assert e.value.info == info
    # the context stays usable
    F = ctx.potrf(dev(inputs.gram_spd(n, seed=5)[0]), tile=64)
    F.close()


def test_potrf_steps_integer_exact(ctx):
    """Tiles of 256 and 512 in matrices of at least four tile columns factor their diagonal
    tiles in 32-column step tasks spread over workgroups; on an integer factor every
    rounding order gives the exact L0."""
    for n, b in [(1000, 256), (1900, 512)]:
        print(f"steps n={n} b={b}", flush=True)
        A, L0, X0, B = inputs.integer_factor(n, seed=n, nrhs=2, unit=True)
        F = ctx.potrf(dev(A), tile=b)
        assert np.array_equal(host(F.L()), L0)
        F.close()


@pytest.mark.parametrize("bad", [5, 300, 543, 990])
def test_potrf_steps_not_positive_definite(ctx, bad):
    """A pivot that fails inside a step task reports the same 1-based column as the oracle."""
    from paper_2308_15964_amd import spx

    n = 1000
    A, _ = inputs.gram_spd(n, seed=410)
    A[bad, bad] = -1.0
    _, _, info = oracle.cholesky(A, oracle_tile(n))
    assert info > 0
    with pytest.raises(spx.NotPositiveDefinite) as e:
        ctx.potrf(dev(A), tile=256)
    assert e.value.info == info
    F = ctx.potrf(dev(inputs.gram_spd(n, seed=5)[0]), tile=256)
    F.close()


def test_potrf_steps_schedules_bitwise_identical(ctx):
    """With the step tasks every schedule still gives the same bits."""
    from paper_2308_15964_amd import spx

    A, B = inputs.gram_spd(1024, seed=19, nrhs=1)
    Ad, Bd = dev(A), dev(B)
    ref = None
    for policy, nwg in [(spx.Q_PRIORITY, 0), (spx.Q_FIFO, 0), (spx.Q_PRIORITY, 3), (spx.Q_FIFO, 1), (spx.Q_SHARDED, 0)]:
        F = ctx.potrf(Ad, tile=256, queue_policy=policy, num_wg=nwg)
        L = host(F.L())
        if ref is None:
            ref = L
            Lo, _, _ = oracle.cholesky(A, oracle_tile(1024))
            check_factor(A, L, Lo)
        assert np.array_equal(L, ref), (policy, nwg)
        F.close()


def test_invalid_arguments(ctx):
    from paper_2308_15964_amd import spx

    A = dev(np.eye(64))
    with pytest.raises(spx.SpxError) as e:
        ctx.potrf(A, tile=48)
    assert e.value.code == spx.SPX_EINVAL
    with pytest.raises(spx.SpxError):
        ctx.potrf(A, queue_policy=7)


def test_config2_full_size_parity(ctx):
    """N=16384, tile 512 (32x32 tiles, 5984 tasks), A = G G^T/N + I, one right-hand side,
    in the launch configuration the benchmark times, element by element against the
    oracle (its thread-pool executor: the same bits as its sequential one, by order
    invariance), plus the definitions: sampled entries of A = L L^T (each O(N),
    compensated), a randomised factor residual, and the backward error of the solution."""
    import os
    import sys
    import time

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench

    n, b = 16384, 512
    A, Bd = bench.gen_input(n, 2, 1, "cuda:0")
    F = ctx.potrf(A, tile=b)
    st = ctx.stats()
    # the program, one inversion per diagonal tile, and each diagonal factorization cut
    # into b/32 chained steps (15 more tasks per diagonal tile)
    assert st["ntasks"] == 5984 + 32 + 32 * 15
    X = ctx.potrs(F, Bd).cpu().numpy()
    L = F.L().cpu().numpy()
    F.close()
    Ah = A.cpu().numpy()
    Bh = Bd.cpu().numpy()
    del A
    torch.cuda.empty_cache()
    rs = np.random.default_rng(99)
    ii = rs.integers(0, n, 400)
    jj = rs.integers(0, n, 400)
    ii[:8] = n - 1
    jj[:8] = np.arange(n - 8, n)  # the last columns see the most updates
    assert oracle.entry_check(Ah, L, ii, jj) <= 1e-13
    assert oracle.factor_residual_probe(Ah, L, nvec=2, seed=5) <= 1e-13
    eta = oracle.backward_error(Ah, X, Bh)
    assert eta.max() <= 1e-14, eta
    threads = max(1, min(16, os.cpu_count() or 1))
    print(f"oracle N={n} tile {b} on {threads} threads", flush=True)
    t0 = time.perf_counter()
    Lo, Xo, info = oracle.cholesky(Ah, b, Bh, nthreads=threads)
    print(f"oracle done in {time.perf_counter() - t0:.1f} s", flush=True)
    assert info == 0
    check_factor(Ah, L, Lo)
    check_solve(X, Xo, eta)
