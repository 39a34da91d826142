"""The allocation-free solve (spx_potrs_noalloc) through the C ABI: the same results, bit
for bit, as spx_potrs without refinement on the same factor, with no device allocation by
the library during the call, on two calls in a row (the second smaller), and a clear
error for a solve that does not fit its scratch array."""
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


def test_noalloc_solve_matches_potrs(ctx):
    from paper_2308_15964_amd import spx

    for n, b, nrhs in [(2100, 512, 5), (700, 256, 2)]:  # the second call is smaller
        print(f"noalloc n={n} b={b} nrhs={nrhs}", flush=True)
        A, B = inputs.gram_spd(n, seed=800 + n, nrhs=nrhs)
        Ad, Bd = dev(A), dev(B)
        F = ctx.potrf(Ad, tile=b)
        want = ctx.potrs(F, Bd).cpu().numpy()
        X = torch.full_like(Bd, float("nan"))
        torch.cuda.synchronize()
        allocs = ctx.stats()["device_allocs"]
        torch_bytes = torch.cuda.memory_allocated()
        ctx.potrs_noalloc(F, Bd, X)
        torch.cuda.synchronize()
        assert ctx.stats()["device_allocs"] == allocs
        assert torch.cuda.memory_allocated() == torch_bytes
        got = X.cpu().numpy()
        assert np.array_equal(got, want)
        _, Xo, _ = oracle.cholesky(A, [nb for nb in (50, 25, 20, 10, 5, 4, 2, 1) if n % nb == 0][0], B)
        assert (np.abs(got - Xo) <= 1e-12 * np.abs(Xo).max(axis=0)).all()
        F.close()
    # too large for the scratch array: a clear error, and the context stays usable
    A, B = inputs.gram_spd(2100, seed=9, nrhs=1)
    F = ctx.potrf(dev(A), tile=512)
    Bbig = torch.ones((2100, 2048), dtype=torch.float64, device="cuda:0")
    with pytest.raises(spx.SpxError) as e:
        ctx.potrs_noalloc(F, Bbig, torch.empty_like(Bbig))
    assert e.value.code == spx.SPX_EINVAL and "scratch" in str(e.value)
    Bd = dev(B)
    X = torch.empty_like(Bd)
    ctx.potrs_noalloc(F, Bd, X)
    assert np.array_equal(X.cpu().numpy(), ctx.potrs(F, Bd).cpu().numpy())
    F.close()
