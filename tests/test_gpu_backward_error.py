"""GPU backward errors against the oracle on planted residuals.

The device computes eta_q = ||b_q - A x_q||_inf / (||A||_inf ||x_q||_inf + ||b_q||_inf) in
plain FP64 (Rigal-Gaches normwise backward error); the refinement loops stop on it and the
batched and served calls report it.  An accurate solution has eta near the unit roundoff,
where the device's own rounding (up to about n u) swamps the value, so these tests plant
a known error instead: x = x_o + delta e_j in chosen rows and columns, which makes eta of
order 1e-6 .. 1e-2.  The device value must then match the oracle's compensated one to
|eta_dev - eta_o| <= 2 n u (the rounding bound of a plain FP64 residual) and to 1e-8
relative; a wrong norm, a dropped term or a swapped maximum fails by far more.
"""
import numpy as np
import pytest

import oracle
from paper_2308_15964_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U = 2.0 ** -53


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


def planted(n, nrhs, seed):
    """A, B, the oracle's solution with planted errors, and the oracle's eta of it."""
    A, B = inputs.gram_spd(n, seed=seed, nrhs=nrhs)
    # one tile: the oracle gives the same bits for every tile size
    _, Xo, info = oracle.cholesky(A, n, B)
    assert info == 0
    rs = np.random.default_rng(seed)
    X = Xo.reshape(n, nrhs).copy()
    for q in range(nrhs):
        scale = np.abs(X[:, q]).max()
        for _ in range(1 + q % 3):
            j = int(rs.integers(0, n))
            X[j, q] += scale * 10.0 ** float(rs.uniform(-5.5, -1.5)) * rs.choice([-1.0, 1.0])
    eta = oracle.backward_error(A, X, B)
    assert (eta > 1e-8).all() and (eta < 1e-1).all(), eta
    return A, B, X, eta


def check(eta_dev, eta_o, n):
    eta_dev = np.asarray(eta_dev, np.float64)
    err = np.abs(eta_dev - eta_o)
    assert (err <= 2.0 * n * U).all(), (eta_dev, eta_o)
    assert (err <= 1e-8 * eta_o).all(), (eta_dev, eta_o)


@pytest.mark.parametrize("n,nrhs", [(64, 1), (300, 3), (1000, 9), (2100, 2)])
def test_single_planted(ctx, n, nrhs):
    print(f"planted eta n={n} nrhs={nrhs}", flush=True)
    A, B, X, eta = planted(n, nrhs, seed=500 + n)
    check(ctx.backward_error(dev(A), dev(X), dev(B)), eta, n)


def test_batched_planted(ctx):
    shapes = [(64, 1), (300, 3), (777, 8), (129, 2), (1000, 5)]
    As, Bs, Xs, want = [], [], [], []
    for m, (n, q) in enumerate(shapes):
        A, B, X, eta = planted(n, q, seed=600 + m)
        As.append(dev(A))
        Bs.append(dev(B))
        Xs.append(dev(X))
        want.append(eta.max())
    got = ctx.backward_error_batched(As, Xs, Bs)
    for m, (n, _) in enumerate(shapes):
        check([got[m]], np.array([want[m]]), n)


def test_served_eta_is_the_batched_kernel(ctx):
    """The serving loop reports the batched residual kernel's value for the X it returns
    (pinned above on planted errors): the two agree bit for bit."""
    from paper_2308_15964_amd import spx

    srv = spx.Server(ctx, 8 << 30, lanes=1)
    try:
        for n, q in [(200, 3), (900, 1)]:
            A, B = inputs.gram_spd(n, seed=700 + n, nrhs=q)
            Ad, Bd = dev(A), dev(B)
            X = torch.empty((n, q), dtype=torch.float64, device="cuda:0")
            r = srv.wait(srv.submit(Ad, Bd, X, mode=spx.MODE_FP64))
            assert r["status"] == 0 and r["info"] == 0
            again = ctx.backward_error_batched([Ad], [X], [Bd])[0]
            assert r["eta_max"] == again, (r["eta_max"], again)
            eta_o = oracle.backward_error(A, X.cpu().numpy(), B).max()
            assert eta_o <= 1e-14 and r["eta_max"] <= eta_o + 2.0 * n * U
    finally:
        srv.close()
