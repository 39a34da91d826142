"""Batched factorisation and solve: many matrices in one persistent launch (Specx Sec. 4.1:
one engine runs several task graphs), through the C ABI.

Pinned against the oracle per matrix (same tolerances as the single-matrix parity tests)
and against the single-matrix entry points.  A factor made in a batch runs exactly the
same tile kernels in the same dependency order as spx_potrf_tiled with the same tile size,
so it is bitwise equal, and so is a solve with kept factors to spx_potrs.  A one-shot
batched solve (factors not kept) uses the in-place block substitution instead of the
tile inverses, so it is pinned bitwise to a task-by-task replay of the same program
through spx_run_task, and to the oracle within tolerance.
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
        Xk, info_k, fs = ctx.posv_batched(As, Bs, tile=tile, keep=True)
        assert (info_k == 0).all()
        for m, ((A, B), Ad, Bd, X) in enumerate(zip(items, As, Bs, Xs)):
            X = X.cpu().numpy()
            _, Xo, oi = oracle.cholesky(A, A.shape[0], B)
            assert oi == 0
            scale = np.abs(Xo).max(axis=0)
            assert (np.abs(X - Xo) <= 1e-12 * scale).all()
            assert (np.abs(Xk[m].cpu().numpy() - Xo) <= 1e-12 * scale).all()
            if m % 6 == 0:  # a member alone in its launch: the other members change nothing
                X1, _ = ctx.posv_batched([Ad], [Bd], tile=tile)
                assert np.array_equal(X, X1[0].cpu().numpy())
            F = ctx.potrf(Ad, tile=tile)
            assert np.array_equal(fs[m].L().cpu().numpy(), F.L().cpu().numpy())
            Xs1 = ctx.potrs(F, Bd).cpu().numpy()
            assert np.array_equal(Xk[m].cpu().numpy(), Xs1)  # same kernels, same order: same bits
            F.close()
            fs[m].close()


def pack_padded(A, b):
    """Lower tiles of A padded with the identity to a multiple of b (column-major tiles)."""
    n = A.shape[0]
    nt = max(1, -(-n // b))
    M = np.eye(nt * b)
    M[:n, :n] = A
    t = np.zeros((nt * (nt + 1) // 2, b * b))
    for i in range(nt):
        for j in range(i + 1):
            t[i * (i + 1) // 2 + j] = M[i * b:(i + 1) * b, j * b:(j + 1) * b].T.ravel()
    return t, nt


def program_order(nt):
    """The in-place factor + substitution program in insertion order (Sec. 5.2 task types)."""
    out = []
    for k in range(nt):
        out.append(("POTRF", k, k, k))
        out += [("TRSM", i, k, k) for i in range(k + 1, nt)]
        for i in range(k + 1, nt):
            out.append(("SYRK", i, i, k))
            out += [("GEMM", i, j, k) for j in range(k + 1, i)]
    for k in range(nt):
        out.append(("FTRSM", k, k, k))
        out += [("FGEMM", i, k, k) for i in range(k + 1, nt)]
    for k in range(nt - 1, -1, -1):
        out.append(("BTRSM", k, k, k))
        out += [("BGEMM", i, k, k) for i in range(k)]
    return out


@pytest.mark.parametrize("tile", [32, 64])
def test_one_shot_batched_solve_equals_task_replay(ctx, tile):
    from paper_2308_15964_amd import spx

    items = [inputs.batch_matrix(n, seed=900 + n, nrhs=q) for n, q in ((1, 1), (37, 3), (64, 9), (130, 2), (200, 17))]
    As = [dev(A) for A, _ in items]
    Bs = [dev(B) for _, B in items]
    Xs, info = ctx.posv_batched(As, Bs, tile=tile)
    assert (info == 0).all()
    for (A, B), X in zip(items, Xs):
        n, q = B.shape
        print(f"replay n={n} nrhs={q} tile={tile}", flush=True)
        t, nt = pack_padded(A, tile)
        tiles = dev(t)
        y = np.zeros((q, nt * tile))
        y[:, :n] = B.T
        rhs = dev(y)  # column-major n_pad x nrhs
        for name, i, j, k in program_order(nt):
            assert ctx.run_task(spx.TASK_NAMES.index(name), i, j, k, nt, tile, tiles, rhs, q) == 0
        assert np.array_equal(X.cpu().numpy(), rhs.cpu().numpy()[:, :n].T)


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
    Xs, info, fs = ctx.posv_batched(As, Bs, keep=True)  # tiles from the table, several sizes in one launch
    assert (info == 0).all()
    X1s, info1 = ctx.posv_batched(As, Bs)
    assert (info1 == 0).all()
    for (A, B), Ad, Bd, X, X1, Fk in zip(items, As, Bs, Xs, X1s, fs):
        assert Fk.tile == ctx.tile_for(0, Ad.shape[0])
        F = ctx.potrf(Ad, tile=Fk.tile)
        assert np.array_equal(X.cpu().numpy(), ctx.potrs(F, Bd).cpu().numpy())
        _, Xo, _ = oracle.cholesky(A, A.shape[0], B)
        assert (np.abs(X1.cpu().numpy() - Xo) <= 1e-12 * np.abs(Xo).max(axis=0)).all()
        F.close()
        Fk.close()
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


def test_posv_batched_keeps_factors_and_refines_from_its_solution(ctx):
    from paper_2308_15964_amd import spx

    items = [inputs.reflector_spd(n, 1e5, seed=500 + n, nrhs=q) for n, q in ((70, 2), (300, 1), (513, 4))]
    As = [dev(A) for A, _ in items]
    Bs = [dev(B) for _, B in items]
    Xs, info, fs = ctx.posv_batched(As, Bs, tile=64, update_prec=spx.PREC_FP32, keep=True)
    assert (info == 0).all() and all(F is not None for F in fs)
    for F, Bd, X in zip(fs, Bs, Xs):  # the fused solve equals a separate solve with the kept factor
        assert np.array_equal(X.cpu().numpy(), ctx.potrs(F, Bd).cpu().numpy())
    X0 = [x.clone() for x in Xs]
    Xr, st = ctx.potrs_batched(fs, Bs, As=As, tol=1e-12, method=1, Xs=Xs, x_init=True)
    for (A, B), F, Ad, Bd, x0, X, s in zip(items, fs, As, Bs, X0, Xr, st):
        assert oracle.backward_error(A, X.cpu().numpy(), B).max() <= 1e-12
        # the same as single refinement started from that solution
        X1 = x0.clone()
        X1, s1 = ctx.potrs(F, Bd, X=X1, A=Ad, tol=1e-12, method=1, return_stats=True, x_init=True)
        assert np.array_equal(X.cpu().numpy(), X1.cpu().numpy()) and s["iters"] == s1["iters"]
    for F in fs:
        F.close()
