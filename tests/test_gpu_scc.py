"""GPU parity of strongly connected components (batched forward/backward
reachability, Parallel SCC section) through the C ABI against the oracle.

The GPU call names each component by its smallest vertex, a labelling with
exactly one correct value, so every case is compared element by element with
oracle.scc_min_label (Tarjan, then the minimum vertex per component), for
every schedule parameter: tau (1 = one BFS level per round), trimming on and
off, a frontier capacity small enough to force the overflow path, and G^T
built inside the call or passed in.
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


def _scc(pg, g, **kw):
    d = pg.DeviceGraph.from_graph(g)
    comp, st = pg.scc(d, stats=True, **kw)
    return comp.cpu().numpy(), st


def _with_loops_and_duplicates(g):
    u = np.repeat(np.arange(g.n), np.diff(g.offsets))
    eu = np.concatenate([u, np.arange(0, g.n, 3), u[::4]])
    ew = np.concatenate([g.targets, np.arange(0, g.n, 3), g.targets[::4]])
    order = np.lexsort((ew, eu))
    off = np.zeros(g.n + 1, dtype=np.int64)
    np.add.at(off, eu + 1, 1)
    return gg.Graph(np.cumsum(off).astype(np.int32), ew[order].astype(np.int32))


def _disjoint_two_cycles(pairs):
    arcs = []
    for i in range(pairs):
        arcs += [(2 * i, 2 * i + 1), (2 * i + 1, 2 * i)]
    return pins.graph_from_arcs(2 * pairs, arcs)


SHAPES = [
    ("dcycle", lambda: gg.simple("dcycle", 1000)),
    ("dchain", lambda: gg.simple("dchain", 1000)),
    ("empty", lambda: gg.simple("empty", 10)),
    ("complete", lambda: gg.simple("complete", 50)),
    ("grid64", lambda: gg.grid(64, 64)),
    ("road128", lambda: gg.road(128, 3)),
    ("road256s5", lambda: gg.road(256, 5)),
    ("knn20k", lambda: gg.knn(20000, 5, 7)),
    ("rmat12", lambda: gg.rmat(12, 8, 1)),
    ("rand3k_sparse", lambda: gg.random_graph(3000, 3000, 41)),
    ("rand3k_mid", lambda: gg.random_graph(3000, 4500, 42)),
    ("rand3k_dense", lambda: gg.random_graph(3000, 9000, 43)),
    ("loops_dups", lambda: _with_loops_and_duplicates(gg.random_graph(2000, 3000, 44))),
]


@pytest.mark.parametrize("name,make", SHAPES, ids=[s[0] for s in SHAPES])
def test_scc_shapes_default(pg, name, make):
    g = make()
    exp = oracle.scc_min_label(g)
    _say(f"scc {name} n={g.n} m={g.m}")
    got, st = _scc(pg, g)
    assert np.array_equal(got, exp)
    assert st["components"] == np.unique(exp).size


@pytest.mark.parametrize("kw", [dict(trim_rounds=0), dict(mode="plain"), dict(tau=16), dict(tau=4096),
                                dict(frontier_capacity=64), dict(trim_rounds=0, frontier_capacity=64, tau=64),
                                dict(wg_size=256, blocks_per_cu=2), dict(prefetch=False),
                                dict(prefetch=False, test_first=True), dict(test_first=False)],
                         ids=["notrim", "plain", "tau16", "tau4096", "cap64", "notrim_cap64_tau64", "wg256x2",
                              "no_prefetch", "no_prefetch_test_first", "no_test_first"])
def test_scc_schedules(pg, kw):
    for g in [gg.road(128, 3), gg.random_graph(3000, 4500, 42), gg.rmat(11, 8, 3)]:
        exp = oracle.scc_min_label(g)
        _say(f"scc {g.name} n={g.n} {kw}")
        got, _ = _scc(pg, g, **kw)
        assert np.array_equal(got, exp)


def test_scc_transpose_passed_in(pg):
    g = gg.road(200, 11)
    d = pg.DeviceGraph.from_graph(g)
    t = pg.transpose(d)
    _say("scc road200 with G^T")
    got = pg.scc(d, transpose=t).cpu().numpy()
    assert np.array_equal(got, oracle.scc_min_label(g))


def test_scc_many_pivots_per_subproblem_repeat_batches(pg):
    """600 disjoint 2-cycles, no trimming and no weak-connectivity split: a
    batch of 512 positions holds far more than 64 unsettled vertices of the
    one initial subproblem, so batches must repeat until every draw got a
    bit. With the split every pair is its own subproblem after the first batch."""
    g = _disjoint_two_cycles(600)
    exp = oracle.scc_min_label(g)
    assert np.array_equal(exp, (np.arange(g.n) // 2 * 2).astype(np.int32))
    _say("scc 600 two-cycles no trim, no split")
    got, st = _scc(pg, g, trim_rounds=0, split=False)
    assert np.array_equal(got, exp)
    assert st["components"] == 600 and st["trimmed"] == 0
    assert st["batches"] > int(np.ceil(np.log2(g.n))) + 1
    _say("scc 600 two-cycles no trim, split")
    got, st = _scc(pg, g, trim_rounds=0)
    assert np.array_equal(got, exp)
    assert st["batches"] <= int(np.ceil(np.log2(g.n))) + 1


def test_scc_pivot_order_and_split_do_not_change_the_result(pg):
    for g in [gg.road(160, 8), gg.random_graph(4000, 6000, 45), gg.knn(8000, 5, 9)]:
        exp = oracle.scc_min_label(g)
        for kw in [dict(seed=1), dict(seed=0xDEADBEEF), dict(split=False), dict(split=False, trim_rounds=0, seed=7)]:
            _say(f"scc {g.name} n={g.n} {kw}")
            got, _ = _scc(pg, g, **kw)
            assert np.array_equal(got, exp), kw


def test_scc_tiny_and_degenerate(pg):
    cases = [pins.graph_from_arcs(1, []), pins.graph_from_arcs(1, [(0, 0)]), pins.graph_from_arcs(2, [(0, 1), (1, 0)]),
             pins.graph_from_arcs(3, [(2, 1), (1, 2), (0, 0)]), pins.graph_from_arcs(5, [(4, 3), (3, 2), (2, 4)])]
    for i, g in enumerate(cases):
        for kw in [dict(), dict(trim_rounds=0)]:
            _say(f"scc tiny case {i} {kw}")
            got, _ = _scc(pg, g, **kw)
            assert np.array_equal(got, oracle.scc_min_label(g)), (i, kw)


def test_scc_exhaustive_4_vertex_digraphs(pg):
    pairs = [(u, v) for u in range(4) for v in range(4) if u != v]
    for bits in range(0, 1 << 12, 37):
        g = pins.graph_from_arcs(4, [pairs[i] for i in range(12) if (bits >> i) & 1])
        got, _ = _scc(pg, g, trim_rounds=0)
        assert np.array_equal(got, oracle.scc_min_label(g)), bits


def test_scc_argument_errors(pg):
    g = gg.road(32, 1)
    d = pg.DeviceGraph.from_graph(g)
    other = pg.DeviceGraph.from_graph(gg.road(16, 1))
    with pytest.raises(pg.PasgalError) as ei:
        pg.scc(d, transpose=other)
    assert ei.value.code == -1
    with pytest.raises(pg.PasgalError) as ei:
        pg.scc(d, asynchronous=True)
    assert ei.value.code == -1
