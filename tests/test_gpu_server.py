"""Serving loop (spx_server_create / spx_submit / spx_poll): admission by an HBM budget,
continuous batching over lanes, and results that do not depend on the mix.

Pins:
  * FP64 mode: each result matches the oracle (1e-12 relative, eta <= 1e-14) and is
    bitwise equal whether the request ran alone or inside a batch with other requests
    (a batched member runs the same tile kernels in the same dependency order);
  * mixed mode (FP32 updates + FP64 refinement): eta <= 1e-12 by the oracle's compensated
    backward error, alone == in the mix bit for bit;
  * admission: peak bytes in use never exceed the budget; a request larger than the
    budget is refused at submission.
"""
import time

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


def mixture(count, seed, kappa=None):
    rs = np.random.default_rng(seed)
    out = []
    for m in range(count):
        n = int(rs.integers(16, 400))
        q = int(rs.integers(1, 6))
        if kappa is None:
            A, B = inputs.gram_spd(n, seed=seed * 1000 + m, nrhs=q)
        else:
            A, B = inputs.reflector_spd(n, kappa, seed=seed * 1000 + m, nrhs=q)
        out.append((A, B))
    return out


def run_all(srv, items, mode, tol=0.0, host=False):
    """Submits every (A, B) at once; returns (X list, result list) in submission order."""
    tickets, outs = [], []
    for A, B in items:
        if host:
            Ad = torch.from_numpy(np.ascontiguousarray(A)).pin_memory()
            Bd = torch.from_numpy(np.ascontiguousarray(B)).pin_memory()
            X = torch.empty(B.shape, dtype=torch.float64).pin_memory()
        else:
            Ad, Bd = dev(A), dev(B)
            X = torch.empty_like(Bd)
        tickets.append(srv.submit(Ad, Bd, X, mode=mode, tol=tol))
        outs.append(X)
    res = [srv.wait(t) for t in tickets]
    return [x.cpu().numpy() for x in outs], res


def test_fp64_alone_equals_mix_and_oracle(ctx):
    from paper_2308_15964_amd import spx

    srv = spx.Server(ctx, 8 << 30, lanes=2)
    target = inputs.gram_spd(300, seed=42, nrhs=3)
    [x_alone], [r_alone] = run_all(srv, [target], spx.MODE_FP64)
    assert r_alone["status"] == 0 and r_alone["info"] == 0 and r_alone["batch_size"] == 1
    items = mixture(30, seed=5)
    items.insert(17, target)
    xs, rs = run_all(srv, items, spx.MODE_FP64)
    assert all(r["status"] == 0 and r["info"] == 0 for r in rs)
    assert np.array_equal(xs[17], x_alone)
    assert max(r["batch_size"] for r in rs) > 1  # requests shared launches
    for (A, B), X, r in zip(items, xs, rs):
        _, Xo, _ = oracle.cholesky(A, A.shape[0], B)
        assert np.abs(X - Xo).max() <= 1e-12 * np.abs(Xo).max()
        assert r["eta_max"] <= 1e-14
        assert r["t_submit"] <= r["t_admit"] <= r["t_start"] <= r["t_done"]
    st = srv.stats()
    assert st["completed"] == st["submitted"] == 32 and st["bytes_in_use"] == 0
    srv.close()


def test_mixed_refined_alone_equals_mix(ctx):
    from paper_2308_15964_amd import spx

    srv = spx.Server(ctx, 8 << 30, lanes=3, mixed_min_n=1)  # every request through FP32 + refinement
    target = inputs.reflector_spd(257, 1e5, seed=9, nrhs=2)
    [x_alone], [r_alone] = run_all(srv, [target], spx.MODE_MIXED, tol=1e-12)
    items = mixture(20, seed=6, kappa=1e4)
    items.insert(3, target)
    xs, rs = run_all(srv, items, spx.MODE_MIXED, tol=1e-12)
    assert np.array_equal(xs[3], x_alone)
    for (A, B), X, r in zip(items, xs, rs):
        assert r["status"] == 0 and r["info"] == 0
        eta = oracle.backward_error(A, X, B)
        assert eta.max() <= 1e-12 and r["eta_max"] <= 1e-12, (eta.max(), r)
        assert r["method_used"] == 1 and r["iters"] >= 1
    srv.close()


def test_host_memory_requests_match_device(ctx):
    from paper_2308_15964_amd import spx

    srv = spx.Server(ctx, 4 << 30, lanes=2)
    items = mixture(6, seed=7)
    xd, _ = run_all(srv, items, spx.MODE_FP64)
    xh, rh = run_all(srv, items, spx.MODE_FP64, host=True)
    assert all(r["status"] == 0 for r in rh)
    for a, b in zip(xd, xh):
        assert np.array_equal(a, b)
    srv.close()


def test_budget_admission(ctx):
    from paper_2308_15964_amd import spx

    items = [inputs.gram_spd(384, seed=70 + i, nrhs=2) for i in range(8)]
    budget = 6 << 20  # about two requests of this size at once
    srv = spx.Server(ctx, budget, lanes=2)
    xs, rs = run_all(srv, items, spx.MODE_FP64)
    assert all(r["status"] == 0 for r in rs)
    st = srv.stats()
    assert 0 < st["bytes_peak"] <= budget
    assert any(r["t_admit"] > r["t_submit"] for r in rs)  # some waited for memory
    big = dev(inputs.gram_spd(2048, seed=1)[0])
    with pytest.raises(spx.SpxError) as e:
        srv.submit(big, dev(np.ones((2048, 1))), torch.empty((2048, 1), dtype=torch.float64, device="cuda:0"))
    assert e.value.code == spx.SPX_ENOMEM
    for (A, B), X in zip(items, xs):
        _, Xo, _ = oracle.cholesky(A, A.shape[0], B)
        assert np.abs(X - Xo).max() <= 1e-12 * np.abs(Xo).max()
    srv.close()


def test_budget_admission_mixed(ctx):
    """Mixed requests keep their factor (tiles, block inverses, the tile inverses M_k and
    the FP32 panel copies) through refinement.  With one 512 tile per request M_k is as
    large as the tiles, so admission must count it: the device pool's high-water mark
    stays within the budget (plus the lanes' small graph images)."""
    from paper_2308_15964_amd import spx

    ctx.set_tile_table(spx.PREC_FP32, [(512, 512)])
    try:
        items = [inputs.gram_spd(500, seed=90 + i, nrhs=2) for i in range(6)]
        budget = 11 << 20  # two of these requests at once
        srv = spx.Server(ctx, budget, lanes=2, mixed_min_n=1)
        xs, rs = run_all(srv, items, spx.MODE_MIXED)
        st = srv.stats()
        srv.close()
    finally:
        ctx.set_tile_table(spx.PREC_FP32, [])
    assert all(r["status"] == 0 and r["info"] == 0 for r in rs)
    assert all(r["tile"] == 512 for r in rs)
    assert 0 < st["bytes_peak"] <= budget
    print(f"pool high-water {st['pool_used_high']} bytes, budget {budget}", flush=True)
    assert st["pool_used_high"] <= budget + (1 << 20), st
    for (A, B), X in zip(items, xs):
        assert oracle.backward_error(A, X, B).max() <= 1e-12


def test_not_pd_request_and_errors(ctx):
    from paper_2308_15964_amd import spx

    srv = spx.Server(ctx, 2 << 30)
    items = mixture(4, seed=8)
    A_bad = items[1][0].copy()
    A_bad[10, 10] = -5.0
    items[1] = (A_bad, items[1][1])
    xs, rs = run_all(srv, items, spx.MODE_FP64)
    assert rs[1]["info"] == 11
    assert [r["info"] for i, r in enumerate(rs) if i != 1] == [0, 0, 0]
    with pytest.raises(spx.SpxError):
        srv.poll(123456789)
    srv.close()


def test_destroy_with_requests_in_flight(ctx):
    from paper_2308_15964_amd import spx

    srv = spx.Server(ctx, 1 << 30, lanes=1)
    items = mixture(12, seed=9)
    keep = []
    for A, B in items:
        Ad, Bd = dev(A), dev(B)
        X = torch.empty_like(Bd)
        keep.append((Ad, Bd, X))
        srv.submit(Ad, Bd, X)
    srv.close()  # running batches finish, the rest end aborted; no hang, no fault
    torch.cuda.synchronize()


@pytest.mark.parametrize("host", [False, True])
def test_per_request_completion(ctx, host):
    """One FP64 batch holding an N=4096 system and small ones: each small request's STORE
    raises its completion flag while the large factorization is still running, so its X
    is in place (t_ready) well before the large one's and before the batch ends (t_done);
    every result is still the oracle's, and the large one's backward error is tiny.  A
    larger request submitted first keeps the single lane busy while the others arrive, so
    they are taken as one batch."""
    from paper_2308_15964_amd import spx

    blocker = inputs.gram_spd(6144, seed=40, nrhs=1)
    items = [inputs.gram_spd(4096, seed=41, nrhs=1)] + mixture(6, seed=42)

    def tensors(A, B):
        if host:
            Ad = torch.from_numpy(np.ascontiguousarray(A)).pin_memory()
            Bd = torch.from_numpy(np.ascontiguousarray(B)).pin_memory()
            return Ad, Bd, torch.empty(B.shape, dtype=torch.float64).pin_memory()
        Ad, Bd = dev(A), dev(B)
        return Ad, Bd, torch.empty_like(Bd)

    srv = spx.Server(ctx, 16 << 30, lanes=1)
    try:
        run_all(srv, [blocker] + items, spx.MODE_FP64, host=host)  # warm-up: images, pool
        tb = tensors(*blocker)
        ts = [tensors(A, B) for A, B in items]
        torch.cuda.synchronize()
        launches = srv.stats()["launches"]
        t0 = srv.submit(*tb, mode=spx.MODE_FP64)
        while srv.stats()["launches"] == launches:  # the blocker's batch has started
            time.sleep(0.0001)
        tickets = [srv.submit(*t, mode=spx.MODE_FP64) for t in ts]
        srv.wait(t0)
        res = [srv.wait(t) for t in tickets]
        Xs = [t[2].cpu().numpy() for t in ts]
    finally:
        srv.close()
    assert len({r["t_start"] for r in res}) == 1  # one batch
    big, small = res[0], res[1:]
    for r in res:
        assert r["status"] == 0 and r["info"] == 0
        assert r["t_start"] <= r["t_ready"] <= r["t_done"]
    assert max(r["t_ready"] for r in small) < big["t_ready"]
    for (A, B), X in zip(items[1:], Xs[1:]):
        _, Xo, info = oracle.cholesky(A, A.shape[0], B)
        assert info == 0
        assert (np.abs(X.reshape(Xo.shape) - Xo) <= 1e-12 * np.abs(Xo).max(axis=0)).all()
    A, B = items[0]
    assert oracle.backward_error(A, Xs[0], B).max() <= 1e-14


def test_mixed_ready_at_batch_end(ctx):
    """Mixed-mode requests that go through the FP32 factor and the batched refinement are
    final only at the end of their batch; those below mixed_min_n take the FP64 path and
    complete on their own, as in FP64 mode, with the FP64 mode's bits."""
    from paper_2308_15964_amd import spx

    items = mixture(4, seed=43, kappa=1e3)
    srv = spx.Server(ctx, 4 << 30, lanes=1, mixed_min_n=1)
    try:
        _, res = run_all(srv, items, spx.MODE_MIXED, tol=1e-12)
    finally:
        srv.close()
    for r in res:
        assert r["status"] == 0 and r["t_ready"] == r["t_done"]
    srv = spx.Server(ctx, 4 << 30, lanes=1)  # default threshold: every request below it
    try:
        xs, res = run_all(srv, items, spx.MODE_MIXED, tol=1e-12)
        xs64, _ = run_all(srv, items, spx.MODE_FP64)
    finally:
        srv.close()
    for x, x64, r in zip(xs, xs64, res):
        assert r["status"] == 0 and r["method_used"] == 0 and r["t_ready"] <= r["t_done"]
        assert np.array_equal(x, x64)


def test_device_inputs_host_results(ctx):
    """where = 2 (A, B on the device, X in host memory) gives the device-only bits."""
    from paper_2308_15964_amd import spx

    items = mixture(8, seed=44)
    srv = spx.Server(ctx, 4 << 30, lanes=2)
    try:
        X1, _ = run_all(srv, items, spx.MODE_FP64)
        tickets, outs = [], []
        for A, B in items:
            X = torch.empty(B.shape, dtype=torch.float64).pin_memory()
            tickets.append(srv.submit(dev(A), dev(B), X, mode=spx.MODE_FP64))
            outs.append(X)
        res = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for x1, x2, r in zip(X1, outs, res):
        assert r["status"] == 0 and r["t_ready"] <= r["t_done"]
        assert np.array_equal(x1, x2.numpy())
