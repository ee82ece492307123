"""GPU parity of the direction-optimizing BFS (top-down / bottom-up levels,
Parallel BFS paragraph) through the C ABI against the oracle's queue BFS.

Hop distances have exactly one correct value, so every case is compared
element by element, for the default switching thresholds and for schedules
forced to stay top-down or to go bottom-up from the first level.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import pins

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALWAYS_BU = dict(alpha=2**31 - 1, beta=-1)
NEVER_BU = dict(alpha=-1)


def _say(msg):
    sys.stdout.write(f"[case] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pg():
    import paper_2404_17101_amd as pg_
    pg_.load()
    assert torch.cuda.is_available()
    return pg_


SYMMETRIC = [
    ("rmat12", lambda: gg.rmat(12, 8, 1)),
    ("rmat16", lambda: gg.rmat(16, 16, 2)),
    ("grid64", lambda: gg.grid(64, 64)),
    ("uchain", lambda: gg.simple("uchain", 500)),
    ("ucycle", lambda: gg.simple("ucycle", 501)),
    ("complete", lambda: gg.simple("complete", 40)),
    ("star", lambda: gg.simple("star", 3000)),
    ("empty", lambda: gg.simple("empty", 7)),
    ("rand_sym", lambda: gg.random_graph(5000, 12000, 51, symmetric=True)),
]

DIRECTED = [
    ("knn20k", lambda: gg.knn(20000, 5, 7)),
    ("road128", lambda: gg.road(128, 3)),
    ("rand_dir", lambda: gg.random_graph(3000, 9000, 52)),
    ("dchain", lambda: gg.simple("dchain", 300)),
]


@pytest.mark.parametrize("name,make", SYMMETRIC, ids=[s[0] for s in SYMMETRIC])
def test_bfs_do_symmetric_graphs_without_transpose(pg, name, make):
    g = make()
    d = pg.DeviceGraph.from_graph(g)
    srcs = sorted(set([0, g.n - 1] + [int(s) for s in gg.sources(g, 3, 61)]))
    for s in srcs:
        exp = oracle.bfs(g, s)
        for kw in [dict(), ALWAYS_BU, NEVER_BU]:
            _say(f"bfs_do {name} src={s} {kw}")
            got = pg.bfs_do(d, s, **kw).cpu().numpy()
            assert np.array_equal(got, exp), (s, kw)


@pytest.mark.parametrize("name,make", DIRECTED, ids=[s[0] for s in DIRECTED])
def test_bfs_do_directed_graphs_with_transpose(pg, name, make):
    g = make()
    d = pg.DeviceGraph.from_graph(g)
    t = pg.transpose(d)
    for s in sorted(set([0] + [int(x) for x in gg.sources(g, 3, 62)])):
        exp = oracle.bfs(g, s)
        for kw in [dict(), ALWAYS_BU, NEVER_BU, dict(alpha=1, beta=1)]:
            _say(f"bfs_do {name} src={s} {kw}")
            got = pg.bfs_do(d, s, transpose=t, **kw).cpu().numpy()
            assert np.array_equal(got, exp), (s, kw)


def test_bfs_do_switches_both_ways_and_counts_levels(pg):
    g = gg.rmat(14, 16, 3)
    d = pg.DeviceGraph.from_graph(g)
    s = int(gg.sources(g, 1, 63, min_degree=1)[0])
    exp = oracle.bfs(g, s)
    got, st = pg.bfs_do(d, s, stats=True)
    assert np.array_equal(got.cpu().numpy(), exp)
    assert st["rounds"] == int(exp.max()) + 1
    _, st_td = pg.bfs_do(d, s, stats=True, **NEVER_BU)
    # bottom-up levels stop at the first frontier in-neighbour: fewer arcs
    assert st["arcs_scanned"] < st_td["arcs_scanned"]


def test_bfs_do_argument_errors(pg):
    g = gg.rmat(10, 8, 1)
    d = pg.DeviceGraph.from_graph(g)
    other = pg.DeviceGraph.from_graph(gg.rmat(9, 8, 1))
    for kw in [dict(transpose=other), dict(asynchronous=True)]:
        with pytest.raises(pg.PasgalError) as ei:
            pg.bfs_do(d, 0, **kw)
        assert ei.value.code == -1
    with pytest.raises(pg.PasgalError):
        pg.bfs_do(d, g.n)


# ---------------------------------------------- many sources at once ------

def _multi_check(pg, g, d, t, srcs, kw, name):
    k = len(srcs)
    dist = torch.empty(k * g.n, dtype=torch.int32, device="cuda")
    reach = torch.empty(g.n, dtype=torch.int64, device="cuda")
    _say(f"bfs_do_multi {name} k={k} {kw}")
    pg.bfs_do_multi(d, srcs, transpose=t, dist_out=dist, reach_out=reach, **kw)
    dd = dist.view(k, g.n).cpu().numpy()
    rr = reach.cpu().numpy().view(np.uint64)
    for q, s in enumerate(srcs):
        exp = oracle.bfs(g, s)
        assert np.array_equal(dd[q], exp), (name, q, s, kw)
        assert np.array_equal(((rr >> np.uint64(q)) & np.uint64(1)).astype(bool), exp >= 0), (name, q, s, kw)
    assert not np.any(rr >> np.uint64(k)) if k < 64 else True


MULTI = [
    ("rmat12", lambda: gg.rmat(12, 8, 1), True),
    ("grid64", lambda: gg.grid(64, 64), True),
    ("star", lambda: gg.simple("star", 3000), True),
    ("empty", lambda: gg.simple("empty", 7), True),
    ("rand_dir", lambda: gg.random_graph(3000, 9000, 52), False),
    ("road128", lambda: gg.road(128, 3), False),
    ("dchain", lambda: gg.simple("dchain", 300), False),
]


@pytest.mark.parametrize("name,make,symmetric", MULTI, ids=[m[0] for m in MULTI])
def test_bfs_do_multi_against_oracle(pg, name, make, symmetric):
    """Every source's distances and reach bit equal the oracle's single-source
    BFS, for 1, 5 (with a repeat) and 64 sources, under the default switching
    rule and schedules forced top-down or bottom-up from the first level."""
    g = make()
    d = pg.DeviceGraph.from_graph(g)
    t = None if symmetric else pg.transpose(d)
    many = [int(x) for x in gg.sources(g, min(64, g.n), 63)]
    many += [many[i % len(many)] for i in range(64 - len(many))]
    cases = [[0], [int(x) for x in gg.sources(g, min(4, g.n), 64)] + [0], many]
    for srcs in cases:
        for kw in [dict(), ALWAYS_BU, NEVER_BU]:
            _multi_check(pg, g, d, t, srcs, kw, name)


def test_bfs_do_multi_rejects_bad_arguments(pg):
    g = gg.grid(8, 8)
    d = pg.DeviceGraph.from_graph(g)
    for srcs in ([], [0] * 65, [64], [-1]):
        with pytest.raises(pg.PasgalError):
            pg.bfs_do_multi(d, srcs, reach_out=torch.empty(g.n, dtype=torch.int64, device="cuda"))


def test_bfs_do_multi_rmat24_full_size(pg):
    """The served RMAT-24 graph, 16 sources at once: four checked against the
    oracle element by element, every source's reach bit against its distances."""
    g = gg.rmat(24, 16, 5)
    d = pg.DeviceGraph.from_graph(g)
    pool = np.flatnonzero(np.diff(g.offsets) > 0)
    srcs = [int(pool[x]) for x in np.random.default_rng(7).integers(0, pool.size, size=16)]
    k = len(srcs)
    dist = torch.empty(k * g.n, dtype=torch.int32, device="cuda")
    reach = torch.empty(g.n, dtype=torch.int64, device="cuda")
    _say("bfs_do_multi rmat24 k=16")
    pg.bfs_do_multi(d, srcs, dist_out=dist, reach_out=reach)
    dv = dist.view(k, g.n)
    for q in range(k):
        bit = ((reach >> q) & 1).bool()
        assert torch.equal(bit, dv[q] >= 0), q
    for q in (0, 5, 10, 15):
        _say(f"bfs_do_multi rmat24 oracle source {q}")
        assert np.array_equal(dv[q].cpu().numpy(), oracle.bfs(g, srcs[q])), q
