"""Batched factorisation and solve: many matrices in one persistent launch (Specx Sec. 4.1:
one engine runs several task graphs), through the C ABI.

Pinned against the oracle per matrix (same tolerances as the single-matrix parity tests)
and against the single-matrix entry points: a batched member runs exactly the same tile
kernels in the same dependency order as spx_potrf_tiled + spx_potrs with the same tile
size, so the results must be bitwise equal.
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


def batch(count, lo, hi, seed, rhs_hi=5):
    rs = np.random.default_rng(seed)
    out = []
    for m in range(count):
        n = int(rs.integers(lo, hi + 1))
        q = int(rs.integers(1, rhs_hi + 1))
        A, B = inputs.batch_matrix(n, seed=seed * 1000 + m, nrhs=q)
        out.append((A, B))
    return out


def test_posv_batched_vs_oracle_and_single(ctx):
    items = batch(24, 1, 300, seed=11)
    for tile in (32, 64, 128):
        print(f"posv_batched tile={tile}", flush=True)
        As = [dev(A) for A, _ in items]
        Bs = [dev(B) for _, B in items]
        Xs, info = ctx.posv_batched(As, Bs, tile=tile)
        assert (info == 0).all()
        for (A, B), Ad, Bd, X in zip(items, As, Bs, Xs):
            X = X.cpu().numpy()
            _, Xo, oi = oracle.cholesky(A, A.shape[0], B)
            assert oi == 0
            scale = np.abs(Xo).max(axis=0)
            assert (np.abs(X - Xo) <= 1e-12 * scale).all()
            F = ctx.potrf(Ad, tile=tile)
            Xs1 = ctx.potrs(F, Bd).cpu().numpy()
            assert np.array_equal(X, Xs1)  # same kernels, same order: same bits
            F.close()


def test_potrf_batched_factors_bitwise_single(ctx):
    items = batch(10, 20, 400, seed=12, rhs_hi=2)
    As = [dev(A) for A, _ in items]
    fs, info = ctx.potrf_batched(As, tile=64)
    assert (info == 0).all()
    for (A, B), Ad, F in zip(items, As, fs):
        L = F.L().cpu().numpy()
        Lo, _, _ = oracle.cholesky(A, A.shape[0])
        d = np.sqrt(np.diag(A))
        assert (np.abs(L - Lo) <= 1e-12 * d[:, None]).all()
        F1 = ctx.potrf(Ad, tile=64)
        assert np.array_equal(L, F1.L().cpu().numpy())
        # the batched factor serves the ordinary solve
        X = ctx.potrs(F, dev(B)).cpu().numpy()
        assert np.array_equal(X, ctx.potrs(F1, dev(B)).cpu().numpy())
        F1.close()
        F.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batched_integer_inputs_exact(ctx, prec):
    items = [inputs.integer_factor(n, seed=300 + n, nrhs=3, unit=True) for n in (5, 33, 64, 130, 257)]
    As = [dev(A) for A, _, _, _ in items]
    Bs = [dev(B) for _, _, _, B in items]
    Xs, info = ctx.posv_batched(As, Bs, tile=32, update_prec=prec)
    assert (info == 0).all()
    for (A, L0, X0, B), X in zip(items, Xs):
        assert np.array_equal(X.cpu().numpy(), X0)


def test_batched_not_pd_member(ctx):
    items = batch(6, 40, 200, seed=13, rhs_hi=2)
    A_bad = items[3][0].copy()
    n = A_bad.shape[0]
    j = n // 2
    A_bad[j, j] = -1.0  # leading minor of order j+1 fails first (earlier ones unchanged)
    items[3] = (A_bad, items[3][1])
    As = [dev(A) for A, _ in items]
    Bs = [dev(B) for _, B in items]
    Xs, info = ctx.posv_batched(As, Bs, tile=32)
    _, _, oi = oracle.cholesky(A_bad, A_bad.shape[0], items[3][1])
    assert info[3] == oi == j + 1
    assert (np.delete(info, 3) == 0).all()
    for m in (0, 1, 2, 4, 5):
        A, B = items[m]
        _, Xo, _ = oracle.cholesky(A, A.shape[0], B)
        assert np.abs(Xs[m].cpu().numpy() - Xo).max() <= 1e-12 * np.abs(Xo).max()


def test_tile_table_and_mixed_tiles(ctx):
    from paper_2308_15964_amd import spx

    ctx.set_tile_table(spx.PREC_FP64, [(64, 32), (200, 64), (10**6, 128)])
    assert [ctx.tile_for(0, n) for n in (1, 64, 65, 200, 201, 5000)] == [32, 32, 64, 64, 128, 128]
    items = batch(12, 10, 350, seed=14)
    As = [dev(A) for A, _ in items]
    Bs = [dev(B) for _, B in items]
    Xs, info = ctx.posv_batched(As, Bs)  # tiles from the table, several sizes in one launch
    assert (info == 0).all()
    for Ad, Bd, X in zip(As, Bs, Xs):
        F = ctx.potrf(Ad, tile=ctx.tile_for(0, Ad.shape[0]))
        assert np.array_equal(X.cpu().numpy(), ctx.potrs(F, Bd).cpu().numpy())
        F.close()
    ctx.set_tile_table(spx.PREC_FP64, [])
    assert ctx.tile_for(0, 5000) == 256


def test_autotuner_sets_table(ctx, tmp_path):
    from paper_2308_15964_amd import autotune

    path = str(tmp_path / "tiles.json")
    e = autotune.ensure(ctx, 0, path, sizes=[48, 160], nrhs=2, copies=32, reps=1)
    assert [s for s, _ in e["table"]] == [48, 160]
    for (s, b) in e["table"]:
        assert b in (32, 64, 128, 256)
        assert ctx.tile_for(0, s) == b
        ms = e["ms"][str(s)]
        assert ms[str(b)] == min(v for v in ms.values() if v > 0)
    ctx.set_tile_table(0, [])
    e2 = autotune.ensure(ctx, 0, path, sizes=[48, 160], nrhs=2)  # restored, not re-tuned
    assert e2["table"] == e["table"] and ctx.tile_for(0, 160) == e["table"][1][1]
    ctx.set_tile_table(0, [])


def test_batched_argument_errors(ctx):
    from paper_2308_15964_amd import spx

    A, B = inputs.batch_matrix(50, seed=1, nrhs=2)
    Ad, Bd = dev(A), dev(B)
    with pytest.raises(spx.SpxError):
        ctx.posv_batched([Ad], [Bd], Xs=[Bd])  # X aliases B
    with pytest.raises(spx.SpxError):
        ctx.posv_batched([Ad], [Bd], tile=48)
    with pytest.raises(ValueError):
        ctx.posv_batched([], [])


@pytest.mark.parametrize("prec", [0, 1])
def test_potrs_batched_matches_single_and_refines(ctx, prec):
    items = [inputs.reflector_spd(n, 1e4, seed=400 + n, nrhs=q) for n, q in ((40, 1), (130, 3), (257, 2), (390, 9))]
    As = [dev(A) for A, _ in items]
    Bs = [dev(B) for _, B in items]
    fs, info = ctx.potrf_batched(As, tile=64, update_prec=prec)
    assert (info == 0).all()
    # plain batched solve == single solves, bit for bit
    Xs, st = ctx.potrs_batched(fs, Bs)
    for F, Bd, X, s in zip(fs, Bs, Xs, st):
        assert np.array_equal(X.cpu().numpy(), ctx.potrs(F, Bd).cpu().numpy())
        assert s["eta_max"] == -1.0
    # refined batched solve == single refined solves (same steps, same launches per system)
    Xr, st = ctx.potrs_batched(fs, Bs, As=As, tol=1e-12, method=1)
    for (A, B), F, Ad, Bd, X, s in zip(items, fs, As, Bs, Xr, st):
        X1, s1 = ctx.potrs(F, Bd, A=Ad, tol=1e-12, method=1, return_stats=True)
        assert np.array_equal(X.cpu().numpy(), X1.cpu().numpy())
        assert s["iters"] == s1["iters"] and s["eta_max"] == s1["eta_max"]
        assert oracle.backward_error(A, X.cpu().numpy(), B).max() <= 1e-12
    eta = ctx.backward_error_batched(As, Xr, Bs)
    assert np.array_equal(eta, np.array([s["eta_max"] for s in st]))
    for F in fs:
        F.close()
