"""The CPU oracle against its pins (closed forms, brute force, certificates,
the paper's printed graph statistics). No GPU involved."""
import json
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import pins

HERE = os.path.dirname(os.path.abspath(__file__))


def test_bfs_grid_manhattan():
    pins.pin_bfs_grid(oracle.bfs)


def test_bfs_torus_closed_form():
    pins.pin_bfs_torus(oracle.bfs)


def test_bfs_families():
    pins.pin_bfs_families(oracle.bfs)


def test_bfs_floyd_warshall():
    pins.pin_bfs_bruteforce(oracle.bfs)


def test_bfs_exhaustive_4_vertex_digraphs():
    pins.pin_bfs_exhaustive4(oracle.bfs)


def test_bfs_certificate_and_undirected_lipschitz():
    pins.pin_bfs_certificates(oracle.bfs)


def test_reach_pins():
    pins.pin_reach(oracle.reach, oracle.bfs)


def test_scc_pins():
    pins.pin_scc(oracle.scc)


def test_scc_min_label_pins():
    pins.pin_scc_min_label(oracle.scc_min_label)


def test_sssp_pins():
    pins.pin_sssp(oracle.sssp, oracle.bfs)


def test_sssp_certificate_rejects_wrong_distances():
    g = gg.road(30, 4)
    w = gg.weights(g, 3, 1, 50)
    d = oracle.sssp(g, w, 0)
    assert pins.sssp_certificate_ok(g, w, 0, d)
    for v in [int(np.argmax(d)), int(np.flatnonzero(d > 0)[0])]:
        for delta in (-1, 1):
            bad = d.copy()
            bad[v] += delta
            assert not pins.sssp_certificate_ok(g, w, 0, bad), (v, delta)


def test_transpose_pins():
    pins.pin_transpose(oracle.transpose)


def test_self_loops_and_duplicate_arcs_change_nothing():
    g = gg.random_graph(200, 500, 31)
    u = np.repeat(np.arange(g.n), np.diff(g.offsets))
    # add every vertex's self-loop and duplicate every third arc
    extra_u = np.concatenate([u, np.arange(g.n), u[::3]])
    extra_w = np.concatenate([g.targets, np.arange(g.n), g.targets[::3]])
    order = np.lexsort((extra_w, extra_u))
    off = np.zeros(g.n + 1, dtype=np.int64)
    np.add.at(off, extra_u + 1, 1)
    g2 = gg.Graph(np.cumsum(off).astype(np.int32), extra_w[order].astype(np.int32))
    for s in [0, 7, 199]:
        assert np.array_equal(oracle.bfs(g, s), oracle.bfs(g2, s))
    assert np.array_equal(oracle.reach(g, [0, 7, 199]), oracle.reach(g2, [0, 7, 199]))
    assert pins.partition_equal(oracle.scc(g), oracle.scc(g2))


@pytest.mark.slow
def test_golden_rec_torus_diameter():
    """The paper prints n = 10^8, m = 4*10^8 and D = 50,500 for REC, a
    10^3 x 10^5 grid; a torus of that shape is vertex-transitive, so the
    eccentricity of vertex 0 is its diameter."""
    with open(os.path.join(HERE, "golden", "paper_graph_table.json")) as f:
        rec = json.load(f)["rec_torus"]
    g = gg.grid(rec["rows"], rec["cols"], torus=True)
    assert g.n == rec["n"] and g.m == rec["m"]
    d = oracle.bfs(g, 0)
    assert int(d.max()) == rec["D"]
    assert int(d.min()) == 0
    del g, d


# --------------------------------------------------------- mutation tests --
# Each mutation plants a plausible mistake in a private copy of oracle.c and
# checks that at least one pin catches it.

MUTATIONS = {
    # FIFO queue replaced by a LIFO stack: distances stop being BFS distances
    "lifo_queue": ("int32_t u = queue[head++];", "int32_t u = queue[--tail];", "bfs"),
    # off-by-one in the relaxation
    "dist_plus_two": ("dist[w] = dist[u] + 1;", "dist[w] = dist[u] + 2;", "bfs"),
    # last arc of every row skipped
    "skip_last_arc": ("for (int32_t e = offsets[u]; e < offsets[u + 1]; e++) {\n      int32_t w = targets[e];\n      if (dist[w] == -1)",
                      "for (int32_t e = offsets[u]; e < offsets[u + 1] - 1; e++) {\n      int32_t w = targets[e];\n      if (dist[w] == -1)", "bfs"),
    # reachability marks the wrong bit
    "reach_wrong_bit": ("const uint64_t bit = 1ULL << (i % 64);", "const uint64_t bit = 1ULL << ((i + 1) % 64);", "reach"),
    # source itself not marked
    "reach_no_source": ("mask[(size_t)s * words + word] |= bit;\n    stack[top++] = s;", "stack[top++] = s;", "reach"),
    # Tarjan without the on-stack test (cross arcs merge components)
    "tarjan_no_onstack": ("} else if (onstack[w] && index[w] < low[u]) {", "} else if (index[w] < low[u]) {", "scc"),
    # Dijkstra relaxes with weight 1 instead of the arc's weight
    "sssp_unit_weight": ("int64_t nd = it.key + (int64_t)weights[e];", "int64_t nd = it.key + 1;", "sssp"),
    # Dijkstra sets a distance only on first discovery (never lowers it)
    "sssp_first_visit_only": ("if (dist[w] < 0 || nd < dist[w]) {", "if (dist[w] < 0) {", "sssp"),
    # transpose keeps the original direction
    "transpose_same_dir": ("t_targets[cursor[targets[e]]++] = u;", "t_targets[cursor[targets[e]]++] = targets[e];", "transpose"),
}


def _mutant(tmpdir, old, new):
    with open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")) as f:
        src = f.read()
    assert old in src, "mutation site not found"
    src = src.replace(old, new, 1)
    c = os.path.join(tmpdir, "m.c")
    so = os.path.join(tmpdir, "libm.so")
    with open(c, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", so, c])
    return so


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    old, new, which = MUTATIONS[name]
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        so = _mutant(tmp, old, new)
        monkeypatch.setattr(oracle, "_LIB", so)
        monkeypatch.setattr(oracle, "_lib", None)
        caught = False
        try:
            if which == "bfs":
                for p in pins.ALL_BFS_PINS[:4]:
                    p(oracle.bfs)
            elif which == "reach":
                pins.pin_reach(oracle.reach, oracle.bfs)
            elif which == "scc":
                pins.pin_scc(oracle.scc)
            elif which == "sssp":
                pins.pin_sssp(oracle.sssp, oracle.bfs)
            else:
                pins.pin_transpose(oracle.transpose)
        except (AssertionError, ValueError, IndexError):
            caught = True
        assert caught, f"mutation {name} survived the pins"
    finally:
        monkeypatch.setattr(oracle, "_lib", None)
        shutil.rmtree(tmp, ignore_errors=True)
