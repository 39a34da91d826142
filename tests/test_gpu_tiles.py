"""Each HIP tile kernel against the oracle's tile kernel (Specx Sec. 5.2 task types), one
task at a time on a 3 x 3 tile matrix, through spx_run_task.

Inputs: off-diagonal tiles iid U[-1,1]; the diagonal tile a triangular task reads is a
well-conditioned lower factor (diagonal U[1,2], below-diagonal U[-1,1]/b); the tile POTRF
factors is SPD (G G^T/b + I).  Tolerance: max |gpu - oracle| <= 1e-12 max |oracle| over
the written tile or block (FP64 with a different summation order on the device).
"""
import zlib

import numpy as np
import pytest

import oracle

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


def pack(M, nt, b):
    t = np.zeros((nt * (nt + 1) // 2, b * b))
    for i in range(nt):
        for j in range(i + 1):
            t[i * (i + 1) // 2 + j] = M[i * b:(i + 1) * b, j * b:(j + 1) * b].T.ravel()
    return t


def tile_of(t, i, j, b):
    return t[i * (i + 1) // 2 + j].reshape(b, b).T


def make(nt, b, rs, nrhs):
    n = nt * b
    M = rs.uniform(-1.0, 1.0, (n, n))
    for d in range(nt):
        T = np.tril(rs.uniform(-1.0, 1.0, (b, b)) / b, -1) + np.diag(rs.uniform(1.0, 2.0, b))
        M[d * b:(d + 1) * b, d * b:(d + 1) * b] = T
    G = rs.standard_normal((b, b))
    M[b:2 * b, b:2 * b] = np.tril(G @ G.T / b + np.eye(b))  # SPD tile (1,1) for POTRF
    Y = rs.uniform(-1.0, 1.0, (n, nrhs))
    return M, Y


TASKS = [("POTRF", 1, 1, 1), ("TRSM", 2, 0, 0), ("SYRK", 2, 2, 0), ("GEMM", 2, 1, 0), ("FTRSM", 1, 1, 1),
         ("FGEMM", 2, 0, 0), ("BTRSM", 1, 1, 1), ("BGEMM", 0, 2, 2)]


@pytest.mark.parametrize("b", [32, 64, 128, 256, 512])
@pytest.mark.parametrize("name,i,j,k", TASKS)
def test_tile_kernel(ctx, b, name, i, j, k):
    from paper_2308_15964_amd import spx

    print(f"tile {name}({i},{j},{k}) b={b}", flush=True)
    nt, nrhs = 3, 11
    rs = np.random.default_rng(zlib.crc32(f"{name}:{b}".encode()))
    M, Y = make(nt, b, rs, nrhs)
    Mo, Yo, info_o = oracle.run_task(name, i, j, k, M, b, Y)
    tiles = torch.from_numpy(pack(M, nt, b)).to("cuda:0")
    rhs = torch.from_numpy(np.asfortranarray(Y).T.copy()).to("cuda:0")  # column-major n x nrhs
    info = ctx.run_task(spx.TASK_NAMES.index(name), i, j, k, nt, b, tiles, rhs, nrhs)
    assert info == info_o == 0
    tg = tiles.cpu().numpy()
    yg = rhs.cpu().numpy().T
    if name in ("POTRF", "TRSM", "SYRK", "GEMM"):
        got = tile_of(tg, i, j, b)
        want = Mo[i * b:(i + 1) * b, j * b:(j + 1) * b]
        if name in ("POTRF", "SYRK"):
            got, want = np.tril(got), np.tril(want)
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= 1e-12, err
        # no other tile changed
        for ii in range(nt):
            for jj in range(ii + 1):
                if (ii, jj) != (i, j):
                    assert np.array_equal(tile_of(tg, ii, jj, b), M[ii * b:(ii + 1) * b, jj * b:(jj + 1) * b])
    else:
        blk = i if name in ("FGEMM", "BGEMM") else k
        got, want = yg[blk * b:(blk + 1) * b], Yo[blk * b:(blk + 1) * b]
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= 1e-12, err
        mask = np.ones(nt * b, bool)
        mask[blk * b:(blk + 1) * b] = False
        assert np.array_equal(yg[mask], Y[mask])


def test_potrf_reports_failing_column(ctx):
    from paper_2308_15964_amd import spx

    b, nt = 64, 2
    rs = np.random.default_rng(7)
    M, _ = make(nt, b, rs, 1)
    M[b + 37, b + 37] = -3.0
    _, _, info_o = oracle.run_task("POTRF", 1, 1, 1, M, b)
    tiles = torch.from_numpy(pack(M, nt, b)).to("cuda:0")
    info = ctx.run_task(spx.T_POTRF, 1, 1, 1, nt, b, tiles)
    assert info == info_o and info > b
