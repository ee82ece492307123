"""GPU parity of single-source shortest paths (VGC local searches with
delta-stepping rounds, Parallel SSSP paragraph) through the C ABI against the
oracle's Dijkstra.

Shortest-path distances with integer weights have exactly one correct value,
so every case is compared element by element, for every schedule parameter:
tau (1 = VGC off), the bucket width delta (default, given, none), frontier
capacity small enough to force the overflow path, heavy-row slices, and the
workgroup shape.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import pins

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


def _run(pg, d, w_dev, s, **kw):
    out, st = pg.sssp(d, w_dev, s, stats=True, **kw)
    u = out.cpu().numpy().view(np.uint32).astype(np.int64)
    u[u == 0xFFFFFFFF] = -1
    return u, st


def _wdev(w):
    return torch.from_numpy(np.ascontiguousarray(w).view(np.int32)).cuda()


CASES = [
    ("grid64_unit", lambda: gg.grid(64, 64), (1, 1)),
    ("knn20k", lambda: gg.knn(20000, 5, 7), (1, 1000)),
    ("road128", lambda: gg.road(128, 3), (1, 1000)),
    ("rmat12", lambda: gg.rmat(12, 8, 1), (1, 1000)),
    ("rmat12_dense", lambda: gg.rmat(12, 24, 4), (1, 1000)),  # m > 8n: default tau 1
    ("rand_zero_w", lambda: gg.random_graph(3000, 9000, 52), (0, 20)),
    ("dchain_w", lambda: gg.simple("dchain", 300), (0, 99)),
    ("empty", lambda: gg.simple("empty", 9), (1, 1)),
]


@pytest.mark.parametrize("name,make,wr", CASES, ids=[c[0] for c in CASES])
def test_sssp_families(pg, name, make, wr):
    g = make()
    w = gg.weights(g, 81, *wr)
    d, wd = pg.DeviceGraph.from_graph(g), _wdev(w)
    for s in sorted(set([0] + [int(x) for x in gg.sources(g, 2, 82)])):
        exp = oracle.sssp(g, w, s)
        _say(f"sssp {name} src={s}")
        got, _ = _run(pg, d, wd, s)
        assert np.array_equal(got, exp), s


@pytest.mark.parametrize("kw", [dict(mode="plain"), dict(tau=16), dict(tau=1024), dict(window=-1), dict(window=50),
                                dict(frontier_capacity=64), dict(heavy_arcs=16), dict(wg_size=256, blocks_per_cu=2),
                                dict(tau=1, window=-1, frontier_capacity=64), dict(prefetch=False),
                                dict(prefetch=False, frontier_capacity=64), dict(test_first=True)],
                         ids=["plain", "tau16", "tau1024", "nowindow", "delta50", "cap64", "heavy16", "wg256x2", "bellman",
                              "no_prefetch", "no_prefetch_cap64", "test_first"])
def test_sssp_schedules(pg, kw):
    for g, wr in [(gg.road(96, 5), (1, 1000)), (gg.rmat(11, 16, 3), (1, 100)), (gg.knn(8000, 5, 9), (0, 50))]:
        w = gg.weights(g, 83, *wr)
        d, wd = pg.DeviceGraph.from_graph(g), _wdev(w)
        s = int(gg.sources(g, 1, 84, min_degree=1)[0])
        _say(f"sssp {g.name} {kw}")
        got, _ = _run(pg, d, wd, s, **kw)
        assert np.array_equal(got, oracle.sssp(g, w, s)), kw


def test_sssp_unit_weights_equal_bfs_and_certificate(pg):
    g = gg.road(200, 7)
    d = pg.DeviceGraph.from_graph(g)
    ones = _wdev(np.ones(g.m, dtype=np.uint32))
    s = int(gg.sources(g, 1, 85, min_degree=1)[0])
    got, _ = _run(pg, d, ones, s)
    assert np.array_equal(got, pg.bfs(d, s).cpu().numpy().astype(np.int64))
    w = gg.weights(g, 86, 1, 5000)
    got, st = _run(pg, d, _wdev(w), s)
    assert pins.sssp_certificate_ok(g, w, s, got)
    assert st["rounds"] > 0


def test_sssp_argument_errors(pg):
    g = gg.road(32, 1)
    d = pg.DeviceGraph.from_graph(g)
    w = _wdev(gg.weights(g, 1))
    with pytest.raises(pg.PasgalError):
        pg.sssp(d, w, g.n)
    with pytest.raises(ValueError):
        pg.sssp(d, w[:-1], 0)
