"""Generator closed forms and determinism (input tooling, no GPU)."""
import json
import os

import numpy as np
import pytest

import graphgen as gg

HERE = os.path.dirname(os.path.abspath(__file__))


def _valid(g):
    assert g.offsets[0] == 0 and g.offsets[-1] == g.m
    assert np.all(np.diff(g.offsets) >= 0)
    assert g.m == 0 or (g.targets.min() >= 0 and g.targets.max() < g.n)
    u = np.repeat(np.arange(g.n), np.diff(g.offsets))
    assert not np.any(u == g.targets)
    for v in range(0, g.n, max(1, g.n // 200)):
        row = g.targets[g.offsets[v]: g.offsets[v + 1]]
        assert np.all(np.diff(row) > 0)


def test_grid_arc_counts():
    g = gg.grid(256, 256)
    assert (g.n, g.m) == (65536, 261120)
    _valid(g)
    for a, b in [(1, 1), (1, 9), (7, 3), (33, 64)]:
        g = gg.grid(a, b)
        assert g.m == 2 * (a * (b - 1) + b * (a - 1))
    t = gg.grid(6, 11, torus=True)
    assert t.m == 4 * 66
    _valid(t)


@pytest.mark.slow
def test_grid_8192_arc_count():
    g = gg.grid(8192, 8192)
    assert (g.n, g.m) == (67108864, 268402688)


def test_knn_out_degree_and_bruteforce():
    for n, k, seed in [(50, 5, 1), (777, 5, 2), (2000, 5, 3), (1500, 10, 4)]:
        for layout in ("draw", "morton"):
            g = gg.knn(n, k, seed, layout=layout)
            assert g.m == k * n
            assert np.all(np.diff(g.offsets) == k)
            _valid(g)
            xy = gg.points(n, seed, layout=layout).astype(np.int64)
            d = ((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1)
            np.fill_diagonal(d, np.iinfo(np.int64).max)
            idx = np.arange(n)
            for i in range(n):
                order = np.lexsort((idx, d[i]))[:k]
                assert np.array_equal(np.sort(order), g.targets[i * k:(i + 1) * k]), (n, k, i)


def test_knn_layouts_are_relabelings():
    a = gg.points(3000, 9, layout="draw")
    b = gg.points(3000, 9, layout="morton")
    assert sorted(map(tuple, a.tolist())) == sorted(map(tuple, b.tolist()))


def test_golden_knn_arc_count_ch5():
    with open(os.path.join(HERE, "golden", "paper_graph_table.json")) as f:
        row = json.load(f)["knn"]["rows"][0]
    assert row["m_directed"] == row["k"] * row["n"]
    g = gg.knn(row["n"], row["k"], 2)
    assert (g.n, g.m) == (row["n"], row["m_directed"])


def test_road_expected_counts():
    g = gg.road(512, 3)
    _valid(g)
    ne = 2 * 512 * 511
    # expected arcs: 0.7 * ne * (0.6*2 + 0.4) + diagonals
    exp = 0.7 * ne * 1.6 + 0.005 * 511 * 512 * 1.6
    assert abs(g.m - exp) < 0.01 * exp
    # every arc is a grid neighbour or a diagonal shortcut to the next/previous row
    u = np.repeat(np.arange(g.n), np.diff(g.offsets))
    dr = g.targets // 512 - u // 512
    dc = g.targets % 512 - u % 512
    assert np.all(np.abs(dr) + np.abs(dc) >= 1)
    assert np.all((np.abs(dr) <= 1) & (np.abs(dc) <= 1))


def test_rmat_symmetric_and_deduplicated():
    g = gg.rmat(12, 16, 5)
    _valid(g)
    assert g.n == 4096
    u = np.repeat(np.arange(g.n), np.diff(g.offsets))
    fwd = set(zip(u.tolist(), g.targets.tolist()))
    assert all((w, v) in fwd for v, w in fwd)


def test_determinism_and_thread_independence():
    a = gg.knn(20000, 5, 13)
    b = gg.knn(20000, 5, 13)
    assert np.array_equal(a.targets, b.targets)
    r1, r2 = gg.road(300, 8), gg.road(300, 8)
    assert np.array_equal(r1.targets, r2.targets) and np.array_equal(r1.offsets, r2.offsets)
    x1, x2 = gg.rmat(11, 8, 1), gg.rmat(11, 8, 1)
    assert np.array_equal(x1.targets, x2.targets)
    assert not np.array_equal(gg.road(300, 9).targets[:1000], r1.targets[:1000])


def test_batch_recipe_shape():
    rec = gg.batch_recipe()
    assert len(rec) == 256
    sides = [r[1] for r in rec if r[0] == "grid"]
    ns = [r[1] for r in rec if r[0] == "knn"]
    assert min(sides) >= 64 and max(sides) <= 2048
    assert min(ns) >= 10_000 and max(ns) <= 1_000_000
    small = gg.pack([gg.grid(3, 3), gg.knn(20, 5, 1), gg.simple("dchain", 4)])
    assert small.n == 9 + 20 + 4 and small.m == 24 + 100 + 3
    for i in range(3):
        sub = small.graph(i)
        _valid(sub)
