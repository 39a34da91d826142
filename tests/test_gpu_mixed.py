"""Mixed-precision updates (SYRK/GEMM on FP32 or BF16 copies with FP32 accumulation,
POTRF/TRSM in FP64) and FP64 iterative refinement, through the C ABI.

The low-precision factor itself is not compared with the oracle entry by entry (it is a
different, rounded computation: parity unpinned).  Pinned instead:
  * integer inputs (unit-diagonal factor with entries in {-1,0,1}): every product and sum
    is an exact small integer in FP32 and BF16 too, so the mixed factor equals L0 bit for bit
    (and, with 32-wide tiles, the solution equals X0);
  * the refined solution reaches eta <= 1e-12 (oracle's compensated backward error) and
    its forward error against the oracle's FP64 solution is <= kappa * 1e-12;
  * the factor residual is of the order of the low precision's unit roundoff.
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


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("n,b", [(200, 64), (640, 128), (1024, 256)])
def test_integer_inputs_exact_mixed(ctx, prec, n, b):
    A, L0, X0, B = inputs.integer_factor(n, seed=n + prec, nrhs=2, unit=True)
    F = ctx.potrf(dev(A), tile=b, update_prec=prec)
    assert np.array_equal(F.L().cpu().numpy(), L0)
    F.close()
    F = ctx.potrf(dev(A), tile=32, update_prec=prec)  # solution exact with 32-wide tiles
    assert np.array_equal(ctx.potrs(F, dev(B)).cpu().numpy(), X0)
    F.close()


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_fp32_updates_refined_to_1e12(ctx, kappa):
    from paper_2308_15964_amd import spx

    n, b, nrhs = 1024, 128, 4
    print(f"fp32 kappa={kappa}", flush=True)
    A, B = inputs.haar_spd(n, kappa, seed=int(np.log10(kappa)), nrhs=nrhs)
    _, Xo, info = oracle.cholesky(A, b, B)
    assert info == 0
    Ad, Bd = dev(A), dev(B)
    F = ctx.potrf(Ad, tile=b, update_prec=spx.PREC_FP32)
    L = F.L().cpu().numpy()
    assert oracle.factor_residual(A, L) <= 1e-5
    X, st = ctx.potrs(F, Bd, A=Ad, tol=1e-12, max_iter=30, method=1, return_stats=True)
    X = X.cpu().numpy()
    eta = oracle.backward_error(A, X, B)
    assert eta.max() <= 1e-12 and st["eta_max"] <= 1e-12, (eta, st)
    assert st["iters"] <= 6
    fwd = np.abs(X - Xo).max(axis=0) / np.abs(Xo).max(axis=0)
    assert fwd.max() <= kappa * 1e-12
    F.close()


def test_bf16_updates_refined_to_1e12(ctx):
    from paper_2308_15964_amd import spx

    n, b, nrhs = 1024, 128, 3
    A, B = inputs.gram_spd(n, seed=77, nrhs=nrhs)  # kappa about 5
    _, Xo, _ = oracle.cholesky(A, b, B)
    Ad, Bd = dev(A), dev(B)
    F = ctx.potrf(Ad, tile=b, update_prec=spx.PREC_BF16)
    L = F.L().cpu().numpy()
    assert oracle.factor_residual(A, L) <= 5e-2
    X, st = ctx.potrs(F, Bd, A=Ad, tol=1e-12, max_iter=50, method=1, return_stats=True)
    X = X.cpu().numpy()
    eta = oracle.backward_error(A, X, B)
    assert eta.max() <= 1e-12, (eta, st)
    assert np.abs(X - Xo).max() / np.abs(Xo).max() <= 1e-11
    F.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_ragged_last_tile_mixed_refined(ctx, prec):
    """N = 1100 with 256-wide tiles: the last tile row holds 76 rows (96 live after rounding
    to 32), so the step-split POTRF of the last diagonal tile has identity steps, the TRSM
    strips and update sub-blocks of the padding are skipped, and the skipped strips' low-
    precision copies are cleared.  A larger factor made first leaves stale values in the
    reused device memory.  The refined solution must reach eta <= 1e-12 (oracle)."""
    from paper_2308_15964_amd import spx

    big, _ = inputs.gram_spd(1280, seed=90 + prec)
    F = ctx.potrf(dev(big), tile=256, update_prec=prec)
    F.close()
    n, b, nrhs = 1100, 256, 2
    print(f"ragged mixed prec={prec} n={n} tile={b}", flush=True)
    A, B = inputs.gram_spd(n, seed=91 + prec, nrhs=nrhs)
    _, Xo, info = oracle.cholesky(A, 100, B)  # the oracle's tile divides n
    assert info == 0
    Ad, Bd = dev(A), dev(B)
    F = ctx.potrf(Ad, tile=b, update_prec=prec)
    L = F.L().cpu().numpy()
    assert np.isfinite(L).all()
    assert oracle.factor_residual(A, L) <= (1e-5 if prec == spx.PREC_FP32 else 5e-2)
    X, st = ctx.potrs(F, Bd, A=Ad, tol=1e-12, max_iter=50, method=1, return_stats=True)
    X = X.cpu().numpy()
    eta = oracle.backward_error(A, X, B)
    assert eta.max() <= 1e-12, (eta, st)
    assert np.abs(X - Xo).max() / np.abs(Xo).max() <= 1e-11
    F.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_mixed_schedules_bitwise_identical(ctx, prec):
    from paper_2308_15964_amd import spx

    A, _ = inputs.gram_spd(768, seed=3)
    Ad = dev(A)
    ref = None
    for policy, nwg in [(spx.Q_PRIORITY, 0), (spx.Q_FIFO, 5), (spx.Q_PRIORITY, 33)]:
        F = ctx.potrf(Ad, tile=128, update_prec=prec, queue_policy=policy, num_wg=nwg)
        L = F.L().cpu().numpy()
        ref = L if ref is None else ref
        assert np.array_equal(L, ref)
        F.close()


def test_refinement_argument_checks(ctx):
    from paper_2308_15964_amd import spx

    A, B = inputs.gram_spd(128, seed=4)
    Ad, Bd = dev(A), dev(B)
    F = ctx.potrf(Ad, tile=64)
    with pytest.raises(spx.SpxError):
        ctx.potrs(F, Bd, method=1)  # no original matrix
    with pytest.raises(spx.SpxError):
        ctx.potrs(F, Bd, A=Ad, method=5)
    X, st = ctx.potrs(F, Bd, A=Ad, tol=1e-12, method=1, return_stats=True)
    assert st["eta_max"] <= 1e-14 and st["iters"] == 0  # FP64 factor: already converged
    F.close()


def test_scaled_shifted_factor_parity(ctx):
    """SPX_F_SCALED factors D^-1/2 A D^-1/2 + shift I: against the oracle's factor of that
    matrix formed on the host with the same operation order (1/sqrt of the diagonal, then
    A_ij d_i d_j, then the shift)."""
    n, shift = 300, 0.25
    A, _ = inputs.haar_spd(n, 1e3, seed=21)
    d = 1.0 / np.sqrt(np.diag(A))
    As = A * d[:, None] * d[None, :]
    As[np.diag_indices(n)] += shift
    Lo, _, info = oracle.cholesky(As, n)
    assert info == 0
    F = ctx.potrf(dev(A), tile=64, shift=shift)
    L = F.L().cpu().numpy()
    dd = np.sqrt(np.diag(As))
    assert (np.abs(L - Lo) <= 1e-12 * dd[:, None]).all()
    F.close()


@pytest.mark.parametrize("kappa,shift", [(1e4, 1e-3), (1e6, 1e-2)])
def test_bf16_scaled_pcg_to_1e12(ctx, kappa, shift):
    """BF16 updates break down on ill-conditioned inputs; the scaled, shifted BF16 factor
    as a preconditioner for FP64 conjugate gradients still reaches eta <= 1e-12."""
    from paper_2308_15964_amd import spx

    n, b, nrhs = 1024, 128, 3
    print(f"bf16 pcg kappa={kappa}", flush=True)
    A, B = inputs.haar_spd(n, kappa, seed=31, nrhs=nrhs)
    _, Xo, _ = oracle.cholesky(A, b, B)
    Ad, Bd = dev(A), dev(B)
    F = ctx.potrf(Ad, tile=b, update_prec=spx.PREC_BF16, shift=shift)
    X, st = ctx.potrs(F, Bd, A=Ad, tol=1e-12, max_iter=400, method=2, return_stats=True)
    X = X.cpu().numpy()
    eta = oracle.backward_error(A, X, B)
    assert eta.max() <= 1e-12 and st["eta_max"] <= 1e-12, (eta, st)
    assert 1 <= st["iters"] <= 400
    fwd = np.abs(X - Xo).max(axis=0) / np.abs(Xo).max(axis=0)
    assert fwd.max() <= kappa * 1e-12
    F.close()


def test_pcg_with_exact_factor_converges_at_once(ctx):
    A, B = inputs.gram_spd(500, seed=41, nrhs=2)
    Ad, Bd = dev(A), dev(B)
    F = ctx.potrf(Ad, tile=128)
    X, st = ctx.potrs(F, Bd, A=Ad, tol=1e-12, method=2, return_stats=True)
    assert st["iters"] == 0 and st["eta_max"] <= 1e-14
    # wide leading dimension of X: the dense work copy is written back
    Xw = torch.zeros((500, 5), dtype=torch.float64, device="cuda:0")
    X2 = ctx.potrs(F, Bd, X=Xw[:, :2], A=Ad, tol=1e-12, method=2)
    assert np.array_equal(X2.cpu().numpy(), X.cpu().numpy())
    F.close()
