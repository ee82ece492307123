"""Independent pins for the CPU oracle.

Each pin checks an oracle result against something other than the oracle:
a closed form, brute force written here with dense numpy matrices, or a
certificate that characterises the exact answer. The functions take the
oracle's entry points as arguments so the mutation tests can run the same pins
against deliberately broken builds of oracle.c.
"""
from __future__ import annotations

import itertools

import numpy as np

import graphgen as gg


# ----------------------------------------------------------------- helpers --

def dense_adj(g) -> np.ndarray:
    n = g.n
    a = np.zeros((n, n), dtype=bool)
    src = np.repeat(np.arange(n), np.diff(g.offsets))
    a[src, g.targets] = True
    return a


def floyd_warshall(adj: np.ndarray) -> np.ndarray:
    """All-pairs hop distances, -1 if unreachable (dense, O(n^3))."""
    n = adj.shape[0]
    inf = np.iinfo(np.int64).max // 4
    d = np.full((n, n), inf, dtype=np.int64)
    d[adj] = 1
    np.fill_diagonal(d, 0)
    for k in range(n):
        d = np.minimum(d, d[:, k : k + 1] + d[k : k + 1, :])
    d[d >= inf] = -1
    return d


def warshall_closure(adj: np.ndarray) -> np.ndarray:
    """Reflexive-transitive closure R[u, v] = u reaches v."""
    r = adj.copy()
    np.fill_diagonal(r, True)
    for k in range(adj.shape[0]):
        r = r | (r[:, k : k + 1] & r[k : k + 1, :])
    return r


def graph_from_arcs(n: int, arcs) -> gg.Graph:
    arcs = sorted(set((int(u), int(v)) for u, v in arcs))
    off = np.zeros(n + 1, dtype=np.int32)
    for u, _ in arcs:
        off[u + 1] += 1
    off = np.cumsum(off).astype(np.int32)
    tgt = np.array([v for _, v in arcs], dtype=np.int32)
    return gg.Graph(off, tgt)


def bfs_certificate_ok(g, src: int, dist: np.ndarray) -> bool:
    """dist is the exact hop distance from src iff
    (I1) dist[src] == 0,
    (I2) every arc (u,w) with dist[u] >= 0 has 0 <= dist[w] <= dist[u] + 1,
    (I3) every v != src with dist[v] >= 0 has an in-arc (u,v) with
         dist[u] == dist[v] - 1.
    I2 gives dist <= true distance on reached vertices and that the reached
    set is closed under arcs; I3 gives dist >= true distance."""
    n = g.n
    if dist.shape != (n,) or dist[src] != 0:
        return False
    u = np.repeat(np.arange(n), np.diff(g.offsets))
    w = g.targets
    du, dw = dist[u].astype(np.int64), dist[w].astype(np.int64)
    reached = du >= 0
    if np.any(dw[reached] < 0) or np.any(dw[reached] > du[reached] + 1):
        return False
    if np.any(dist < -1):
        return False
    has_parent = np.zeros(n, dtype=bool)
    ok = reached & (du == dw - 1)
    has_parent[w[ok]] = True
    need = dist > 0
    return bool(np.all(has_parent[need]))


def reach_closure_ok(g, sources, mask: np.ndarray) -> bool:
    """mask is the exact reachability closure iff bit i is set at sources[i],
    mask[w] contains mask[u] on every arc, and every set bit at v != source
    is supported by an in-arc carrying it (then set bits form a set closed
    under arcs that contains the source and whose members have in-paths
    from it -- the reachable set). Support is checked by the per-source BFS
    distances the caller cross-checks separately."""
    n = g.n
    u = np.repeat(np.arange(n), np.diff(g.offsets))
    w = g.targets
    for i, s in enumerate(sources):
        if not (int(mask[s, i // 64]) >> (i % 64)) & 1:
            return False
    return bool(np.all((mask[u] & ~mask[w]) == 0))


def partition_equal(a: np.ndarray, b: np.ndarray) -> bool:
    """Two labelings describe the same partition."""
    if a.shape != b.shape:
        return False
    pairs = set(zip(a.tolist(), b.tolist()))
    return len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


# --------------------------------------------------------------- the pins --

def pin_bfs_grid(bfs):
    for (a, b), srcs in [((1, 1), [0]), ((1, 7), [0, 3]), ((5, 3), [0, 7, 14]), ((32, 17), [0, 100, 543]),
                         ((256, 256), [0, 65535, 32896])]:
        g = gg.grid(a, b)
        r, c = np.divmod(np.arange(a * b), b)
        for s in srcs:
            r0, c0 = divmod(s, b)
            exp = np.abs(r - r0) + np.abs(c - c0)
            got = bfs(g, s)
            assert np.array_equal(got, exp), (a, b, s)


def pin_bfs_torus(bfs):
    for (a, b), srcs in [((3, 4), [0, 5]), ((7, 9), [0, 31]), ((40, 25), [0, 999, 517])]:
        g = gg.grid(a, b, torus=True)
        r, c = np.divmod(np.arange(a * b), b)
        for s in srcs:
            r0, c0 = divmod(s, b)
            dr, dc = np.abs(r - r0), np.abs(c - c0)
            exp = np.minimum(dr, a - dr) + np.minimum(dc, b - dc)
            assert np.array_equal(bfs(g, s), exp), (a, b, s)
            assert exp.max() == a // 2 + b // 2


def pin_bfs_families(bfs):
    n = 50
    idx = np.arange(n)
    for s in [0, 17, 49]:
        got = bfs(gg.simple("dchain", n), s)
        assert np.array_equal(got, np.where(idx >= s, idx - s, -1)), s
        assert np.array_equal(bfs(gg.simple("uchain", n), s), np.abs(idx - s))
        assert np.array_equal(bfs(gg.simple("dcycle", n), s), (idx - s) % n)
        d = np.abs(idx - s)
        assert np.array_equal(bfs(gg.simple("ucycle", n), s), np.minimum(d, n - d))
        exp = np.ones(n, dtype=np.int32)
        exp[s] = 0
        assert np.array_equal(bfs(gg.simple("complete", n), s), exp)
        exp = np.full(n, -1, dtype=np.int32)
        exp[s] = 0
        assert np.array_equal(bfs(gg.simple("empty", n), s), exp)
        star = bfs(gg.simple("star", n), s)
        exp = np.where(idx == 0, 1, 2) if s != 0 else np.ones(n, dtype=np.int32)
        exp = np.array(exp, dtype=np.int32)
        exp[s] = 0
        assert np.array_equal(star, exp)


def pin_bfs_bruteforce(bfs, count=40):
    for t in range(count):
        n = 2 + (t * 7) % 63
        m0 = int(n * (0.5 + (t % 5)))
        g = gg.random_graph(n, m0, seed=9000 + t)
        d = floyd_warshall(dense_adj(g))
        for s in range(n):
            assert np.array_equal(bfs(g, s), d[s]), (t, s)


def pin_bfs_exhaustive4(bfs):
    """Every digraph on 4 vertices without self-loops (2^12) from every source,
    against reachability by powers of the adjacency matrix."""
    pairs = [(u, v) for u in range(4) for v in range(4) if u != v]
    for bits in range(1 << 12):
        arcs = [pairs[i] for i in range(12) if (bits >> i) & 1]
        g = graph_from_arcs(4, arcs)
        a = dense_adj(g).astype(np.int64)
        exp = np.full((4, 4), -1, dtype=np.int64)
        p = np.eye(4, dtype=np.int64)
        for k in range(4):
            newly = (p > 0) & (exp < 0)
            exp[newly] = k
            p = np.minimum(p @ a, 1)
        for s in range(4):
            assert np.array_equal(bfs(g, s), exp[s]), (bits, s)


def pin_bfs_certificates(bfs):
    cases = [gg.knn(3000, 5, 7, layout="draw"), gg.road(64, 3), gg.rmat(10, 8, 5), gg.random_graph(500, 900, 77)]
    for g in cases:
        srcs = gg.sources(g, 3, 1)
        for s in srcs:
            d = bfs(g, int(s))
            assert bfs_certificate_ok(g, int(s), d), (g.name, s)
    # |d(u) - d(v)| <= 1 across every edge of an undirected graph
    for g in [gg.grid(40, 60), gg.rmat(9, 4, 3), gg.random_graph(300, 600, 5, symmetric=True)]:
        d = bfs(g, 0)
        u = np.repeat(np.arange(g.n), np.diff(g.offsets))
        both = (d[u] >= 0) & (d[g.targets] >= 0)
        assert np.all(np.abs(d[u][both] - d[g.targets][both]) <= 1)
        assert np.array_equal(d[u] >= 0, d[g.targets] >= 0)


def pin_reach(reach, bfs):
    n = 70
    ch = gg.simple("dchain", n)
    srcs = [0, 5, 69, 33]
    m = reach(ch, srcs)
    for i, s in enumerate(srcs):
        col = (m[:, 0] >> np.uint64(i)) & np.uint64(1)
        assert np.array_equal(col.astype(bool), np.arange(n) >= s)
    m = reach(gg.simple("dcycle", n), srcs)
    assert np.all(m[:, 0] == np.uint64((1 << len(srcs)) - 1))
    # Warshall closure on small random graphs, more than 64 sources (2 words)
    for t in range(12):
        nn = 8 + 7 * t
        g = gg.random_graph(nn, int(1.3 * nn), seed=500 + t)
        r = warshall_closure(dense_adj(g))
        k = min(nn, 70)
        srcs = np.array([(i * 13 + t) % nn for i in range(k)], dtype=np.int32)
        m = reach(g, srcs)
        for i, s in enumerate(srcs):
            col = ((m[:, i // 64] >> np.uint64(i % 64)) & np.uint64(1)).astype(bool)
            assert np.array_equal(col, r[s]), (t, i)
    # DFS reachability vs per-source BFS (different code paths of the oracle)
    for g in [gg.knn(2000, 5, 3, layout="draw"), gg.road(48, 9), gg.rmat(9, 8, 2)]:
        srcs = gg.sources(g, 64, 11)
        m = reach(g, srcs)
        assert reach_closure_ok(g, srcs, m)
        for i, s in enumerate(srcs):
            col = ((m[:, 0] >> np.uint64(i)) & np.uint64(1)).astype(bool)
            assert np.array_equal(col, bfs(g, int(s)) >= 0), (g.name, i)


def pin_scc(scc):
    n = 40
    assert len(set(scc(gg.simple("dcycle", n)).tolist())) == 1
    assert len(set(scc(gg.simple("dchain", n)).tolist())) == n
    assert len(set(scc(gg.grid(20, 30)).tolist())) == 1
    assert len(set(scc(gg.simple("empty", 9)).tolist())) == 9
    for t in range(25):
        nn = 3 + 3 * t
        g = gg.random_graph(nn, int(1.5 * nn), seed=700 + t)
        r = warshall_closure(dense_adj(g))
        mutual = r & r.T
        # canonical brute-force label: smallest vertex of the class
        bf = np.argmax(mutual, axis=1)
        assert partition_equal(scc(g), bf), t
    # exhaustive 4-vertex digraphs
    pairs = [(u, v) for u in range(4) for v in range(4) if u != v]
    for bits in range(0, 1 << 12, 3):
        g = graph_from_arcs(4, [pairs[i] for i in range(12) if (bits >> i) & 1])
        r = warshall_closure(dense_adj(g))
        assert partition_equal(scc(g), np.argmax(r & r.T, axis=1)), bits


def pin_scc_min_label(scc_min):
    """Exact labels, not just the partition: the brute-force class of v
    (mutual reachability by Warshall closure) named by its smallest vertex."""
    n = 40
    assert np.array_equal(scc_min(gg.simple("dcycle", n)), np.zeros(n, np.int32))
    assert np.array_equal(scc_min(gg.simple("dchain", n)), np.arange(n, dtype=np.int32))
    assert np.array_equal(scc_min(gg.simple("empty", 9)), np.arange(9, dtype=np.int32))
    assert np.array_equal(scc_min(gg.grid(20, 30)), np.zeros(600, np.int32))
    for t in range(25):
        nn = 3 + 3 * t
        g = gg.random_graph(nn, int(1.5 * nn), seed=900 + t)
        r = warshall_closure(dense_adj(g))
        assert np.array_equal(scc_min(g), np.argmax(r & r.T, axis=1).astype(np.int32)), t
    pairs = [(u, v) for u in range(4) for v in range(4) if u != v]
    for bits in range(1, 1 << 12, 5):
        g = graph_from_arcs(4, [pairs[i] for i in range(12) if (bits >> i) & 1])
        r = warshall_closure(dense_adj(g))
        assert np.array_equal(scc_min(g), np.argmax(r & r.T, axis=1).astype(np.int32)), bits


def pin_transpose(transpose):
    for g in [gg.random_graph(60, 200, 3), gg.road(20, 4), gg.knn(500, 5, 1, layout="draw"), gg.simple("empty", 5)]:
        t_off, t_tgt = transpose(g)
        assert t_off[0] == 0 and t_off[-1] == g.m
        a = dense_adj(g)
        tg = gg.Graph(t_off, t_tgt)
        assert np.array_equal(dense_adj(tg), a.T)
        for v in range(g.n):
            row = t_tgt[t_off[v] : t_off[v + 1]]
            assert np.all(np.diff(row) > 0)
        # involution
        o2, t2 = transpose(tg)
        assert np.array_equal(o2, g.offsets) and np.array_equal(t2, g.targets)


ALL_BFS_PINS = [pin_bfs_grid, pin_bfs_torus, pin_bfs_families, pin_bfs_bruteforce, pin_bfs_exhaustive4,
                pin_bfs_certificates]


def all_pairs_iter(n):
    return itertools.product(range(n), range(n))


# ------------------------------------------------------------------ SSSP ---

def sssp_certificate_ok(g, w, s, d) -> bool:
    """Exact characterisation of shortest-path distances for POSITIVE integer
    weights, checked arc by arc: (I1) d(s) = 0; (I2) every arc (u, v) with u
    reached has v reached and d(v) <= d(u) + w(u, v) (so d <= the true
    distance, by induction along a shortest path); (I3) every reached v != s
    has an in-arc (u, v) from a reached u with d(u) + w(u, v) = d(v) (so,
    following such arcs back, d(v) is the length of a real path, reaching s
    because d strictly decreases)."""
    d = np.asarray(d, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    if d[s] != 0:
        return False
    u = np.repeat(np.arange(g.n), np.diff(g.offsets))
    v = g.targets.astype(np.int64)
    ru = d[u] >= 0
    if np.any(ru & (d[v] < 0)):
        return False
    if np.any(ru & (d[v] > d[u] + w)):
        return False
    tight = ru & (d[u] + w == d[v])
    has = np.zeros(g.n, dtype=bool)
    has[v[tight]] = True
    need = (d >= 0)
    need[s] = False
    return bool(np.all(has[need]))


def weighted_floyd_warshall(g, w) -> np.ndarray:
    n = g.n
    inf = np.iinfo(np.int64).max // 4
    dm = np.full((n, n), inf, dtype=np.int64)
    np.fill_diagonal(dm, 0)
    u = np.repeat(np.arange(n), np.diff(g.offsets))
    for a, b, c in zip(u, g.targets, np.asarray(w, dtype=np.int64)):
        dm[a, b] = min(dm[a, b], c)
    for k in range(n):
        dm = np.minimum(dm, dm[:, k:k + 1] + dm[k:k + 1, :])
    dm[dm >= inf] = -1
    return dm


def pin_sssp(sssp, bfs):
    # unit weights: hop distances (an independent algorithm, FIFO BFS)
    for g in [gg.grid(30, 40), gg.knn(3000, 5, 4, layout="draw"), gg.road(40, 2), gg.rmat(10, 8, 3)]:
        ones = np.ones(g.m, dtype=np.uint32)
        for s in [0, g.n // 2]:
            assert np.array_equal(sssp(g, ones, s), bfs(g, s).astype(np.int64)), (g.name, s)
    # weighted directed chain: prefix sums from the source, -1 before it
    n = 50
    g = gg.simple("dchain", n)
    w = gg.weights(g, 5, 0, 99)
    pre = np.concatenate([[0], np.cumsum(w.astype(np.int64))])
    for s in [0, 17, n - 1]:
        exp = np.full(n, -1, dtype=np.int64)
        exp[s:] = pre[s:] - pre[s]
        assert np.array_equal(sssp(g, w, s), exp), s
    # brute force (Floyd-Warshall), zero weights included
    for t in range(20):
        nn = 4 + 2 * t
        g = gg.random_graph(nn, 3 * nn, seed=800 + t)
        w = gg.weights(g, 900 + t, 0, 20)
        dm = weighted_floyd_warshall(g, w)
        for s in range(0, nn, 3):
            assert np.array_equal(sssp(g, w, s), dm[s]), (t, s)
    # certificate with positive weights on larger graphs
    for g in [gg.knn(2000, 5, 3, layout="draw"), gg.road(48, 9), gg.rmat(9, 8, 2)]:
        w = gg.weights(g, 7, 1, 1000)
        for s in [int(x) for x in gg.sources(g, 3, 13)]:
            assert sssp_certificate_ok(g, w, s, sssp(g, w, s)), (g.name, s)
