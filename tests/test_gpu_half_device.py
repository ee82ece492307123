"""GPU parity of half-device launches (PASGAL_FLAG_HALF_DEVICE) through the
C ABI against the oracle.

A half-device launch sizes its persistent grid for half of every compute
unit and is launched as an ordinary kernel, so that two such calls on two
streams run at the same time (the headline job overlaps its batched BFS
launch with its reach launch this way). The results must not change: every
case is compared element by element with the oracle, alone and while a
second half-device traversal runs on another stream.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    sys.stdout.write(f"[case] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pg():
    import paper_2404_17101_amd as pg_
    pg_.load()
    assert torch.cuda.is_available()
    return pg_


HALF = dict(half_device=True, wg_size=512)

GRAPHS = [("grid64x90", lambda: gg.grid(64, 90)), ("knn20k", lambda: gg.knn(20000, 5, 3)),
          ("road100", lambda: gg.road(100, 4)), ("rmat12", lambda: gg.rmat(12, 8, 2)),
          ("dchain700", lambda: gg.simple("dchain", 700))]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[x[0] for x in GRAPHS])
def test_half_device_single_calls(pg, name, make):
    g = make()
    d = pg.DeviceGraph.from_graph(g)
    srcs = gg.sources(g, 5, 11)
    for kw in [HALF, dict(HALF, tau=16), dict(HALF, frontier_capacity=64), dict(HALF, wg_size=256, blocks_per_cu=2)]:
        _say(f"half {name} {kw}")
        got = pg.bfs(d, int(srcs[0]), **kw).cpu().numpy()
        assert np.array_equal(got, oracle.bfs(g, int(srcs[0]))), kw
        m = pg.reach(d, srcs, **kw).cpu().numpy().view(np.uint64)
        assert np.array_equal(m, oracle.reach(g, srcs)), kw
    w = gg.weights(g, 5, 1, 50)
    got = pg.sssp(d, torch.from_numpy(w.view(np.int32)).cuda(), int(srcs[1]), **HALF).cpu().numpy().view(np.uint32)
    exp = oracle.sssp(g, w, int(srcs[1]))
    assert np.array_equal(np.where(got == 0xFFFFFFFF, -1, got.astype(np.int64)), exp)
    assert np.array_equal(pg.scc(d, **HALF).cpu().numpy(), oracle.scc_min_label(g))


def test_half_device_rejects_a_grid_that_cannot_share_the_cus(pg):
    """1024-thread workgroups fill a compute unit's wave slots on their own,
    so two of them per CU (one per half) cannot be resident together."""
    g = gg.grid(16, 16)
    d = pg.DeviceGraph.from_graph(g)
    with pytest.raises(pg.PasgalError) as ei:
        pg.bfs(d, 0, half_device=True, wg_size=1024)
    assert ei.value.code == -1
    # workgroups whose waves do not spread evenly over the four SIMDs of a CU
    # are refused before anything is launched
    for kw in [dict(half_device=True, wg_size=384), dict(device_share=75, wg_size=704),
               dict(device_share=25, wg_size=128, blocks_per_cu=2)]:
        with pytest.raises(pg.PasgalError) as ei:
            pg.bfs(d, 0, **kw)
        assert ei.value.code == -1, kw


def test_concurrent_batch_and_reach_on_two_streams(pg):
    """The headline schedule at small size: the reach launch is enqueued
    asynchronously on one stream, the hipGraph-captured batch runs on
    another; both results match the oracle on every repetition."""
    g = gg.knn(60000, 5, 7, layout="morton")
    d = pg.DeviceGraph.from_graph(g)
    srcs = [int(s) for s in gg.sources(g, 16, 21)]
    n = g.n
    dist = torch.empty(n * 16, dtype=torch.int32, device="cuda")
    mask = torch.empty((n, 1), dtype=torch.int64, device="cuda")
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    b = pg.Batch(d, np.array([0, n], np.int32), np.zeros(16, np.int32), np.array(srcs, np.int32),
                 np.arange(16, dtype=np.int64) * n, dist, stream=sa, **HALF)
    exp_d = [oracle.bfs(g, s) for s in srcs]
    exp_m = oracle.reach(g, srcs)
    for rep in range(3):
        _say(f"concurrent batch + reach rep {rep}")
        dist.fill_(-7)
        mask.fill_(0)
        torch.cuda.synchronize()
        pg.reach(d, srcs, label_out=mask, stream=sb, asynchronous=True, **HALF)
        b.run()
        torch.cuda.synchronize()
        got = dist.view(16, n).cpu().numpy()
        for j in range(16):
            assert np.array_equal(got[j], exp_d[j]), (rep, j)
        assert np.array_equal(mask.cpu().numpy().view(np.uint64), exp_m), rep
    b.close()


def test_two_asynchronous_bfs_calls_overlap(pg):
    g1, g2 = gg.road(150, 3), gg.grid(120, 200)
    d1, d2 = pg.DeviceGraph.from_graph(g1), pg.DeviceGraph.from_graph(g2)
    o1 = torch.empty(g1.n, dtype=torch.int32, device="cuda")
    o2 = torch.empty(g2.n, dtype=torch.int32, device="cuda")
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        s1, s2 = int(gg.sources(g1, 1, rep)[0]), int(gg.sources(g2, 1, rep)[0])
        _say(f"two async bfs rep {rep}")
        torch.cuda.synchronize()
        pg.bfs(d1, s1, dist_out=o1, stream=sa, asynchronous=True, **HALF)
        pg.bfs(d2, s2, dist_out=o2, stream=sb, asynchronous=True, **HALF)
        torch.cuda.synchronize()
        assert np.array_equal(o1.cpu().numpy(), oracle.bfs(g1, s1)), rep
        assert np.array_equal(o2.cpu().numpy(), oracle.bfs(g2, s2)), rep


def test_async_timeout_reported_by_wait_and_next_call(pg):
    """Status of asynchronous launches (PASGAL_FLAG_ASYNC): a launch whose
    bounded waits expire (timeout 1 ms on a traversal of about 1,600 tau-1
    rounds, each ending at a grid barrier) still returns PASGAL_OK at once;
    pasgal_wait on its stream then reports PASGAL_ETIMEOUT, and a second wait
    reports OK. When nobody waits, the next call on that stream reports the
    timeout instead of running; the call after it runs normally. Every kernel
    exits through its own bounded wait."""
    g = gg.knn(2_000_000, 5, 2)
    d = pg.DeviceGraph.from_graph(g)
    src = int(gg.sources(g, 1, 31)[0])
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    quick = dict(stream=s, asynchronous=True, timeout_ms=1, tau=1, window=0)
    _say("async timeout, then wait")
    pg.bfs(d, src, dist_out=out, **quick)
    with pytest.raises(pg.PasgalError) as ei:
        pg.wait(s)
    assert ei.value.code == -7
    pg.wait(s)
    _say("async timeout, then the next call")
    pg.bfs(d, src, dist_out=out, **quick)
    with pytest.raises(pg.PasgalError) as ei:
        pg.bfs(d, src, dist_out=out, stream=s)
    assert ei.value.code == -7
    got = pg.bfs(d, src, dist_out=out, stream=s).cpu().numpy()
    assert np.array_equal(got, oracle.bfs(g, src))
    # an asynchronous launch that finishes in time reports OK
    pg.bfs(d, src, dist_out=out, stream=s, asynchronous=True)
    pg.wait(s)
    assert np.array_equal(out.cpu().numpy(), got)


def test_shutdown_then_calls_work_again(pg):
    """pasgal_shutdown releases every workspace; later calls re-create them."""
    g = gg.road(80, 9)
    d = pg.DeviceGraph.from_graph(g)
    srcs = gg.sources(g, 3, 12)
    before = pg.bfs(d, int(srcs[0])).cpu().numpy()
    pg.load().pasgal_shutdown()
    assert np.array_equal(pg.bfs(d, int(srcs[0])).cpu().numpy(), before)
    assert np.array_equal(pg.reach(d, srcs).cpu().numpy().view(np.uint64), oracle.reach(g, srcs))
    assert np.array_equal(before, oracle.bfs(g, int(srcs[0])))
