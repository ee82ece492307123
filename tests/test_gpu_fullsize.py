"""GPU parity at the full configuration sizes, in the launch configurations
the benchmark times (tau 1024, window 32, 1024-thread workgroups, one per CU).

Where the oracle is too slow for every query at full size, the check is on
sampled queries against the oracle plus, for every query, a property that
holds at any size and characterises the exact answer (closed-form grid
distances, the BFS certificate, reachability closure).
"""
import sys
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import pins

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(300)]
torch = pytest.importorskip("torch")


def _say(msg):
    sys.stdout.write(f"[case] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pg():
    import paper_2404_17101_amd as pg_
    pg_.load()
    return pg_


@pytest.fixture(scope="module")
def knn10m():
    return gg.knn(10_000_000, 5, 2, layout="morton")


def test_c2_knn10m_batched16_and_reach16(pg, knn10m):
    g = knn10m
    srcs = [int(s) for s in gg.sources(g, 16, 1002)]
    d = pg.DeviceGraph.from_graph(g)
    n = g.n
    dist16 = torch.empty(16 * n, dtype=torch.int32, device="cuda")
    _say("c2 batched16")
    b = pg.Batch(d, np.array([0, n], np.int32), np.zeros(16, np.int32), np.array(srcs, np.int32),
                 np.arange(16, dtype=np.int64) * n, dist16)
    b.run()
    got = dist16.view(16, n).cpu().numpy()
    b.close()
    _say("c2 reach16")
    mask = pg.reach(d, srcs).cpu().numpy().view(np.uint64)[:, 0]
    for i in range(3):
        _say(f"c2 oracle source {i}")
        exp = oracle.bfs(g, srcs[i])
        assert np.array_equal(got[i], exp), i
        assert np.array_equal(((mask >> np.uint64(i)) & np.uint64(1)).astype(bool), exp >= 0), i
    for i in range(16):
        assert pins.bfs_certificate_ok(g, srcs[i], got[i]), i
        # reach bit i is exactly the BFS-reached set of source i
        assert np.array_equal(((mask >> np.uint64(i)) & np.uint64(1)).astype(bool), got[i] >= 0), i
    assert pins.reach_closure_ok(g, srcs, mask.reshape(-1, 1))


def test_c2_knn10m_single_source_calls(pg, knn10m):
    """Every tau the configuration names (64, 256, 1024, 4096), with the
    distance window off and at its default, and plain, for BFS and reach."""
    g = knn10m
    s = int(gg.sources(g, 16, 1002)[5])
    d = pg.DeviceGraph.from_graph(g)
    exp = oracle.bfs(g, s)
    cases = [dict(mode="plain")]
    for tau in (64, 256, 1024, 4096):
        cases += [dict(tau=tau), dict(tau=tau, window=0)]
    cases.append(dict(tau=4096, window=64))
    for kw in cases:
        _say(f"c2 single bfs {kw}")
        assert np.array_equal(pg.bfs(d, s, **kw).cpu().numpy(), exp), kw
    for kw in [dict(mode="plain"), dict(tau=64), dict(tau=256), dict(tau=1024), dict(tau=4096)]:
        _say(f"c2 single reach {kw}")
        got = pg.reach(d, [s], **kw).cpu().numpy().view(np.uint64)[:, 0]
        assert np.array_equal(got == 1, exp >= 0), kw
        assert np.all((got == 0) | (got == 1)), kw


def test_c2_knn10m_sssp_against_dijkstra(pg, knn10m):
    """Weighted shortest paths on the 10M-point 5-NN graph (weights uniform in
    [1, 1000], seed 2002) from one source, element by element."""
    g = knn10m
    w = gg.weights(g, 2002, 1, 1000)
    d = pg.DeviceGraph.from_graph(g)
    wd = torch.from_numpy(w.view(np.int32)).cuda()
    s = int(gg.sources(g, 16, 1002)[0])
    _say("c2 sssp dijkstra")
    exp = oracle.sssp(g, w, s)
    for kw in [dict(), dict(mode="plain")]:
        _say(f"c2 sssp {kw}")
        got = pg.sssp(d, wd, s, **kw).cpu().numpy().view(np.uint32).astype(np.int64)
        got[got == 0xFFFFFFFF] = -1
        assert np.array_equal(got, exp), kw


def test_c3_road4096_forward_backward_scc(pg):
    g = gg.road(4096, 3)
    d = pg.DeviceGraph.from_graph(g)
    _say("c3 transpose")
    t = pg.transpose(d)
    t_off, t_tgt = oracle.transpose(g)
    assert np.array_equal(t.offsets.cpu().numpy(), t_off)
    # every row as a set (the order inside a row is unspecified): sort the
    # (row, target) pairs of both sides
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(t_off))
    got_keys = np.sort(rows * g.n + t.targets.cpu().numpy().astype(np.int64))
    exp_keys = np.sort(rows * g.n + t_tgt.astype(np.int64))
    assert np.array_equal(got_keys, exp_keys)
    del rows, got_keys, exp_keys
    gt = gg.Graph(t_off, t_tgt)
    pivots = gg.sources(g, 64, 1003)
    _say("c3 forward/backward reach")
    fw = pg.reach(d, pivots).cpu().numpy().view(np.uint64)[:, 0]
    bw = pg.reach(t, pivots).cpu().numpy().view(np.uint64)[:, 0]
    # sampled pivots against the oracle, all pivots through closure + SCC partition
    for i in [0, 17, 63]:
        _say(f"c3 oracle pivot {i}")
        ef = oracle.bfs(g, int(pivots[i])) >= 0
        eb = oracle.bfs(gt, int(pivots[i])) >= 0
        assert np.array_equal(((fw >> np.uint64(i)) & np.uint64(1)).astype(bool), ef), i
        assert np.array_equal(((bw >> np.uint64(i)) & np.uint64(1)).astype(bool), eb), i
    assert pins.reach_closure_ok(g, pivots, fw.reshape(-1, 1))
    assert pins.reach_closure_ok(gt, pivots, bw.reshape(-1, 1))
    _say("c3 tarjan")
    comp = oracle.scc(g)
    both = fw & bw
    for i, p in enumerate(pivots):
        sel = ((both >> np.uint64(i)) & np.uint64(1)).astype(bool)
        assert np.array_equal(sel, comp == comp[p]), i


def test_c3_road4096_scc_against_tarjan(pg):
    """Whole SCC labelling of the 4096^2 road graph, element by element."""
    g = gg.road(4096, 3)
    d = pg.DeviceGraph.from_graph(g)
    _say("c3 scc oracle")
    exp = oracle.scc_min_label(g)
    t = pg.transpose(d)
    for kw in [dict(), dict(mode="plain"), dict(split=False, seed=3)]:
        _say(f"c3 scc {kw}")
        got, st = pg.scc(d, transpose=t, stats=True, **kw)
        assert np.array_equal(got.cpu().numpy(), exp), kw
        assert st["components"] == 1716206


@pytest.fixture(scope="module")
def c4():
    rec = gg.batch_recipe()
    _say("c4 generate")
    graphs = gg.batch_graphs(rec)
    packed = gg.pack(graphs)
    qg, qs, qo = [], [], []
    off = 0
    for gi, g in enumerate(graphs):
        for s in gg.sources(g, 4, 1004 + gi):
            qg.append(gi)
            qs.append(int(s))
            qo.append(off)
            off += g.n
    return rec, graphs, packed, np.array(qg), np.array(qs), np.array(qo, dtype=np.int64), off


def _check_c4(rec, graphs, qg, qs, qo, got):
    """Every query: grids by the closed form, 5-NN graphs by the oracle (the
    small ones and every 16th) or by the BFS certificate."""
    checked = 0
    for j in range(len(qg)):
        kind = rec[qg[j]]
        g = graphs[qg[j]]
        out = got[qo[j]:qo[j] + g.n]
        if kind[0] == "grid":
            side = kind[1]
            r, c = np.divmod(np.arange(g.n), side)
            r0, c0 = divmod(int(qs[j]), side)
            assert np.array_equal(out, np.abs(r - r0) + np.abs(c - c0)), j
        elif j % 16 == 0 or g.n < 30000:
            assert np.array_equal(out, oracle.bfs(g, int(qs[j]))), j
            checked += 1
        else:
            assert pins.bfs_certificate_ok(g, int(qs[j]), out), j
    assert checked > 0


def test_c4_batch_1024_queries_uneven_graphs(pg, c4):
    rec, graphs, packed, qg, qs, qo, total = c4
    pd = pg.DeviceGraph.from_numpy(packed.offsets, packed.targets)
    dist = torch.empty(total, dtype=torch.int32, device="cuda")
    _say(f"c4 batch of {len(qg)} queries, {packed.n} vertices, {packed.m} arcs")
    b = pg.Batch(pd, packed.vbase, qg, qs, qo, dist)
    b.run()
    got = dist.cpu().numpy()
    b.close()
    _check_c4(rec, graphs, qg, qs, qo, got)


def test_c4_batch_autotuned_every_query(pg, c4):
    """The configuration the c4 suite times: tau, workgroup size and frontier
    capacity chosen by the autotuner, the captured graph replayed twice (the
    second replay after eager work on the stream); every query checked."""
    rec, graphs, packed, qg, qs, qo, total = c4
    pd = pg.DeviceGraph.from_numpy(packed.offsets, packed.targets)
    dist = torch.empty(total, dtype=torch.int32, device="cuda")
    _say("c4 autotuned batch")
    b = pg.Batch(pd, packed.vbase, qg, qs, qo, dist, autotune=True)
    cfg = b.config()
    _say(f"c4 autotuned config {cfg}")
    b.run()
    got = dist.cpu().numpy()
    _check_c4(rec, graphs, qg, qs, qo, got)
    dist.fill_(-7)
    b.run()
    assert np.array_equal(dist.cpu().numpy(), got)
    b.close()


def test_c5_grid8192_closed_form_and_rmat24_sample(pg):
    side = 8192
    g = gg.grid(side, side)
    assert (g.n, g.m) == (67108864, 268402688)
    d = pg.DeviceGraph.from_graph(g)
    r, c = np.divmod(np.arange(g.n, dtype=np.int64), side)
    for s in [0, int(gg.sources(g, 1, 1005)[0])]:
        _say(f"c5 grid src={s}")
        got = pg.bfs(d, s).cpu().numpy()
        r0, c0 = divmod(s, side)
        assert np.array_equal(got, (np.abs(r - r0) + np.abs(c - c0)).astype(np.int32)), s
    del d, g, r, c
    torch.cuda.empty_cache()
    _say("c5 rmat24 generate")
    x = gg.rmat(24, 16, 5)
    dx = pg.DeviceGraph.from_graph(x)
    s = int(gg.sources(x, 1, 1005, min_degree=1)[0])
    _say(f"c5 rmat24 src={s} n={x.n} m={x.m}")
    exp = oracle.bfs(x, s)
    assert np.array_equal(pg.bfs(dx, s).cpu().numpy(), exp)
    assert np.array_equal(pg.bfs(dx, s, mode="plain").cpu().numpy(), exp)
    _say("c5 rmat24 direction-optimizing")
    assert np.array_equal(pg.bfs_do(dx, s).cpu().numpy(), exp)
    got = pg.reach(dx, [s]).cpu().numpy().view(np.uint64)[:, 0]
    assert np.array_equal(got == 1, exp >= 0)


def test_c5_served_full_size_state_past_2_32(pg):
    """The served configuration at full size: the 8192^2 grid and RMAT-24
    resident, 256 slots, a burst of requests whose state lies beyond 2^32
    elements of the arena (so 64-bit state and bitmap indices are used and the
    32-bit-keyed LDS filter is off). Grid BFS against the Manhattan closed form
    and grid reach against all bits set (the grid is connected), computed on
    the device; RMAT requests against the oracle."""
    side = 8192
    grid = gg.grid(side, side)
    _say("c5 served: generate rmat24")
    rmat = gg.rmat(24, 16, 5)
    dg, dr = pg.DeviceGraph.from_graph(grid), pg.DeviceGraph.from_graph(rmat)
    srv = pg.Server(max_slots=256)
    gid_g, gid_r = srv.add_graph(dg), srv.add_graph(dr)
    plan = []
    rng = np.random.default_rng(2025)
    # reach first: 40 x 8 B x 67M = 21.5 GB of arena, so the BFS requests
    # admitted after them (first fit, in arrival order, while the reach
    # requests are still resident) sit past 16 GiB = 2^32 4-byte elements
    for i in range(40):
        k = int(rng.integers(1, 65))
        srcs = [int(x) for x in rng.integers(0, grid.n, size=k)]
        plan.append(("grid", "reach", srcs, torch.empty(grid.n, dtype=torch.int64, device="cuda")))
    for i in range(24):
        plan.append(("grid", "bfs", [int(rng.integers(0, grid.n))], torch.empty(grid.n, dtype=torch.int32,
                                                                                 device="cuda")))
    pool = np.flatnonzero(np.diff(rmat.offsets) > 0)
    for i in range(3):
        kind = "reach" if i == 2 else "bfs"
        srcs = [int(pool[x]) for x in rng.integers(0, pool.size, size=(3 if kind == "reach" else 1))]
        plan.append(("rmat", kind, srcs, torch.empty(rmat.n, dtype=torch.int64 if kind == "reach" else torch.int32,
                                                     device="cuda")))
    torch.cuda.synchronize()
    reqs = [(where, kind, srcs, out, srv.submit(gid_g if where == "grid" else gid_r, kind, srcs, out=out))
            for where, kind, srcs, out in plan]
    assert all(r[4] is not None for r in reqs)
    _say(f"c5 served: {len(reqs)} requests submitted")
    most = 0
    done = []
    for _ in range(4000):
        most = max(most, srv.load_info()["bytes"])
        done += srv.poll(1000)
        if done:  # until the first completion
            break
        time.sleep(0.0005)
    # every grid reach request and at least one grid BFS request were resident together
    assert most >= 40 * 8 * grid.n + 4 * grid.n, most
    srv.drain(240000)
    comps = {c["id"]: c for c in done + srv.poll(1000)}
    assert len(comps) == len(reqs)
    assert all(c["status"] == 0 for c in comps.values())
    idx = torch.arange(grid.n, dtype=torch.int64, device="cuda")
    r, c = idx // side, idx % side
    del idx
    for where, kind, srcs, out, rid in reqs:
        if where != "grid":
            continue
        if kind == "bfs":
            r0, c0 = divmod(srcs[0], side)
            exp = ((r - r0).abs() + (c - c0).abs()).to(torch.int32)
            assert torch.equal(out, exp), (rid, srcs)
        else:
            want = int(np.array((1 << len(srcs)) - 1, dtype=np.uint64).view(np.int64))
            assert bool((out == want).all()), (rid, len(srcs))
    del r, c
    for where, kind, srcs, out, rid in reqs:
        if where != "rmat":
            continue
        _say(f"c5 served: rmat {kind} oracle")
        if kind == "bfs":
            assert np.array_equal(out.cpu().numpy(), oracle.bfs(rmat, srcs[0])), rid
        else:
            assert np.array_equal(out.cpu().numpy().view(np.uint64), oracle.reach(rmat, srcs)[:, 0]), rid
    srv.close()
