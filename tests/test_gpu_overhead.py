"""The device scheduler on graphs of empty tasks (the runtime-overhead pattern of Specx
Sec. 5.1): every task waits a fixed number of device clock ticks, so the trace shows the
scheduler alone.  Checked: every task runs once, for at least its duration, after all of
its predecessors; T independent chains of N tasks take at least N durations."""
import numpy as np
import pytest

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


def chains(T, N, d):
    """T chains of N tasks, task (s, t) inserted at s*T + t writing the d data of chain t."""
    return [(s * T + t, 2, t * d + q) for s in range(N) for t in range(T) for q in range(d)]


def spans(tr, ntasks):
    task = tr[:, 0].astype(np.int64)
    start = np.full(ntasks, np.iinfo(np.int64).max)
    end = np.zeros(ntasks, np.int64)
    np.minimum.at(start, task, tr[:, 2].astype(np.int64))
    np.maximum.at(end, task, tr[:, 3].astype(np.int64))
    return start, end


@pytest.mark.parametrize("T,N,d,ticks", [(8, 20, 1, 2000), (16, 10, 5, 1000), (64, 8, 20, 500)])
def test_chains_of_spin_tasks(ctx, T, N, d, ticks):
    from paper_2308_15964_amd import spx

    g = spx.Graph.build(T * N, chains(T, N, d))
    st = ctx.run_graph(g, ticks, flags=spx.F_TRACE)
    tr = ctx.trace()
    assert st["ntasks"] == T * N == len(tr)
    assert len(set(tr[:, 0].tolist())) == T * N
    start, end = spans(tr, T * N)
    assert ((end - start) >= ticks).all()
    e = g.edges()
    assert len(e) == T * (N - 1)
    assert (end[e[:, 0]] <= start[e[:, 1]]).all()
    assert st["kernel_ms"] * 1e5 >= N * ticks  # ms -> 100 MHz ticks
    g.close()


@pytest.mark.parametrize("seed", range(3))
def test_random_graph_respects_every_edge(ctx, seed):
    from paper_2308_15964_amd import spx

    rs = np.random.default_rng(seed)
    T = 400
    acc = []
    for t in range(T):
        for _ in range(int(rs.integers(1, 4))):
            acc.append((t, int(rs.choice([1, 2])), int(rs.integers(0, 60))))
    g = spx.Graph.build(T, acc, priority=rs.integers(0, 5, T))
    for policy in (spx.Q_PRIORITY, spx.Q_FIFO, spx.Q_SHARDED):
        st = ctx.run_graph(g, 50, queue_policy=policy, flags=spx.F_TRACE)
        tr = ctx.trace()
        assert len(tr) == T and len(set(tr[:, 0].tolist())) == T
        start, end = spans(tr, T)
        e = g.edges()
        assert (end[e[:, 0]] <= start[e[:, 1]]).all()
    g.close()


def test_bad_arguments(ctx):
    from paper_2308_15964_amd import spx

    g = spx.Graph.build(2, [(0, 2, 0), (1, 2, 0)])
    with pytest.raises(spx.SpxError) as e:
        ctx.run_graph(g, 2 * 10 ** 9)
    assert e.value.code == spx.SPX_EINVAL
    g.close()
