"""GPU parity of the tiled matrix product (the GEMM application, Specx Sec. 5.2) against the
oracle, through the C ABI.

The device takes each C_ij's k terms in increasing k (the write-after-write chain), but
sums inside a tile on the matrix cores with fused multiply-adds, so it agrees with the
oracle to rounding: |C - Co| <= (n + 2) u (|C0| + |A| |B|) entry by entry (the classical
bound for two computations of the same sums).  Integer inputs small enough that every
partial sum is exact must match bit for bit.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U = np.finfo(float).eps / 2


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_15964_amd import spx

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = spx.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def oracle_tile(n):
    for nb in (64, 50, 48, 40, 32, 25, 24, 20, 16, 10, 8, 5, 4, 2, 1):
        if n % nb == 0:
            return nb
    return 1


def check(got, A, B, C, want):
    bound = (A.shape[0] + 2) * U * (np.abs(C) + np.abs(A) @ np.abs(B))
    err = np.abs(got - want)
    assert (err <= bound).all(), float((err / np.maximum(bound, 1e-300)).max())


@pytest.mark.parametrize("n,b", [(32, 32), (64, 32), (100, 32), (256, 64), (300, 128), (700, 256), (1024, 128),
                                 (1100, 512)])
def test_gemm_parity(ctx, n, b):
    print(f"gemm n={n} b={b}", flush=True)
    rs = np.random.default_rng(1000 + n + b)
    A, B, C = rs.standard_normal((3, n, n))
    want = oracle.gemm(A, B, C, oracle_tile(n), nthreads=8)
    Cd = dev(C)
    ctx.gemm(dev(A), dev(B), Cd, tile=b)
    st = ctx.stats()
    nt = -(-n // b)
    assert st["ntasks"] == nt ** 3 and st["tile"] == b
    check(Cd.cpu().numpy(), A, B, C, want)


@pytest.mark.parametrize("n,b", [(96, 32), (200, 64), (512, 128), (1024, 256)])
def test_gemm_integer_exact(ctx, n, b):
    rs = np.random.default_rng(n)
    A = rs.integers(-8, 9, (n, n)).astype(np.float64)
    B = rs.integers(-8, 9, (n, n)).astype(np.float64)
    C = rs.integers(-100, 101, (n, n)).astype(np.float64)
    Cd = dev(C)
    ctx.gemm(dev(A), dev(B), Cd, tile=b)
    assert np.array_equal(Cd.cpu().numpy(), oracle.gemm(A, B, C, oracle_tile(n)))


def test_gemm_schedules_bitwise_identical(ctx):
    from paper_2308_15964_amd import spx

    rs = np.random.default_rng(7)
    n = 640
    A, B, C = rs.standard_normal((3, n, n))
    Ad, Bd = dev(A), dev(B)
    ref = None
    for policy, nwg in [(spx.Q_PRIORITY, 0), (spx.Q_FIFO, 0), (spx.Q_PRIORITY, 5), (spx.Q_FIFO, 1), (spx.Q_SHARDED, 0)]:
        Cd = dev(C)
        ctx.gemm(Ad, Bd, Cd, tile=128, queue_policy=policy, num_wg=nwg)
        got = Cd.cpu().numpy()
        if ref is None:
            ref = got
        assert np.array_equal(got, ref), (policy, nwg)


def test_gemm_trace_respects_every_edge(ctx):
    from paper_2308_15964_amd import spx

    rs = np.random.default_rng(8)
    n, b = 512, 128
    A, B, C = rs.standard_normal((3, n, n))
    ctx.gemm(dev(A), dev(B), dev(C), tile=b, flags=spx.F_TRACE)
    tr = ctx.trace()
    st = ctx.stats()
    assert len(tr) == st["nparts"] == (n // b) ** 3 * (b // 128) ** 2
    task = tr[:, 0].astype(np.int64)
    start = np.full(st["ntasks"], np.iinfo(np.int64).max)
    end = np.zeros(st["ntasks"], np.int64)
    np.minimum.at(start, task, tr[:, 2].astype(np.int64))
    np.maximum.at(end, task, tr[:, 3].astype(np.int64))
    e = spx.Graph.gemm(n // b).edges()
    assert len(e) == (n // b) ** 2 * (n // b - 1)
    assert (end[e[:, 0]] <= start[e[:, 1]]).all()


def test_gemm_full_size_sampled(ctx):
    """N = 16384, tile 512 (32^3 = 32768 tasks) in the benchmark's launch configuration;
    sampled entries against the oracle's one-entry-at-a-time sums."""
    n, b = 16384, 512
    g = torch.Generator(device="cuda:0").manual_seed(11)
    A = torch.randn((n, n), dtype=torch.float64, device="cuda:0", generator=g)
    B = torch.randn((n, n), dtype=torch.float64, device="cuda:0", generator=g)
    C = torch.randn((n, n), dtype=torch.float64, device="cuda:0", generator=g)
    rs = np.random.default_rng(12)
    ii = rs.integers(0, n, 300)
    jj = rs.integers(0, n, 300)
    ii[:4] = n - 1
    jj[:4] = [0, 1, n - 2, n - 1]
    Ah, Bh, C0 = A.cpu().numpy(), B.cpu().numpy(), C.cpu().numpy()
    ctx.gemm(A, B, C, tile=b)
    got = C.cpu().numpy()[ii, jj]
    want = oracle.gemm_entries(Ah, Bh, C0, ii, jj)
    bound = (n + 2) * U * (np.abs(C0[ii, jj]) + np.einsum("sm,ms->s", np.abs(Ah[ii]), np.abs(Bh[:, jj])))
    assert (np.abs(got - want) <= bound).all()
