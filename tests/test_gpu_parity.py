"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every traversal result has exactly one correct value (hop distance / the
reachable set), so the bar is bit-exact equality on every case, for every
schedule parameter (tau, workgroup size, workgroups per CU, frontier
capacity down to a size that forces the overflow path).
"""
import os
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


def dev(pg, g):
    return pg.DeviceGraph.from_graph(g)


def np_dist(t):
    return t.cpu().numpy().astype(np.int32)


def np_mask(t):
    return t.cpu().numpy().view(np.uint64)


# ------------------------------------------------------------------ BFS ---

def test_c1_grid_plain_and_vgc_manhattan(pg):
    """256x256 grid from vertex 0: dist = r + c (511 levels)."""
    g = gg.grid(256, 256)
    d = dev(pg, g)
    r, c = np.divmod(np.arange(g.n), 256)
    exp = (r + c).astype(np.int32)
    _say("c1 plain")
    got, st = pg.bfs(d, 0, mode="plain", stats=True)
    assert np.array_equal(np_dist(got), exp)
    assert st["rounds"] == 511
    for tau in [1, 16, 64, 256, 1024, 4096]:
        _say(f"c1 vgc tau={tau}")
        got, st = pg.bfs(d, 0, tau=tau, stats=True)
        assert np.array_equal(np_dist(got), exp), tau
        if tau == 1:
            assert st["rounds"] == 511
        else:
            assert st["rounds"] < 511


@pytest.mark.parametrize("wg,bpc", [(64, 1), (256, 2), (512, 1), (1024, 1), (1024, 2)])
def test_bfs_launch_shapes(pg, wg, bpc):
    g = gg.knn(20000, 5, 2)
    d = dev(pg, g)
    for s in gg.sources(g, 3, 1002):
        _say(f"knn20k wg={wg} bpc={bpc} src={s}")
        exp = oracle.bfs(g, int(s))
        got = pg.bfs(d, int(s), tau=256, wg_size=wg, blocks_per_cu=bpc)
        assert np.array_equal(np_dist(got), exp)


@pytest.mark.parametrize("cap", [64, 200, 1000])
def test_bfs_tiny_frontier_forces_overflow_path(pg, cap):
    g = gg.road(128, 3)
    d = dev(pg, g)
    overflowed = 0
    for s in gg.sources(g, 2, 7):
        _say(f"road128 cap={cap} src={s}")
        exp = oracle.bfs(g, int(s))
        for tau in [1, 64, 1024]:
            got, st = pg.bfs(d, int(s), tau=tau, frontier_capacity=cap, stats=True)
            assert np.array_equal(np_dist(got), exp), (cap, tau)
            overflowed += st["overflow"]
    # a BFS level of this 128x128 road grid holds more than 64 vertices
    if cap == 64:
        assert overflowed > 0


def test_bfs_families_and_degenerate(pg):
    cases = [gg.simple("dchain", 3000), gg.simple("uchain", 1000), gg.simple("dcycle", 777),
             gg.simple("complete", 90), gg.simple("star", 5000), gg.simple("empty", 100), gg.simple("empty", 1),
             gg.grid(1, 1), gg.grid(1, 4097), gg.grid(3, 1000, torus=True), gg.random_graph(3000, 9000, 5)]
    for g in cases:
        d = dev(pg, g)
        srcs = sorted(set([0, g.n - 1, g.n // 2]))
        for s in srcs:
            exp = oracle.bfs(g, s)
            for mode, tau in [("plain", 0), ("vgc", 1), ("vgc", 64), ("vgc", 4096)]:
                _say(f"{g.name} src={s} {mode} tau={tau}")
                got = pg.bfs(d, s, mode=mode, tau=tau or 256)
                assert np.array_equal(np_dist(got), exp), (g.name, s, mode, tau)


def test_bfs_rmat_skewed_degrees(pg):
    g = gg.rmat(14, 16, 5)
    d = dev(pg, g)
    for s in gg.sources(g, 3, 9, min_degree=1):
        exp = oracle.bfs(g, int(s))
        for tau in [1, 256]:
            _say(f"rmat14 src={s} tau={tau}")
            assert np.array_equal(np_dist(pg.bfs(d, int(s), tau=tau)), exp)
        assert np.array_equal(np_dist(pg.bfs(d, int(s), mode="plain")), exp)


def test_bfs_metamorphic_relabel_and_duplicates(pg):
    g = gg.knn(5000, 5, 4, layout="draw")
    rng = np.random.default_rng(3)
    perm = rng.permutation(g.n).astype(np.int32)  # new id of old vertex
    inv = np.argsort(perm)
    u = np.repeat(np.arange(g.n), np.diff(g.offsets))
    nu, nw = perm[u], perm[g.targets]
    # duplicate every 4th arc and add self-loops
    nu = np.concatenate([nu, nu[::4], np.arange(g.n)])
    nw = np.concatenate([nw, nw[::4], np.arange(g.n)])
    order = np.lexsort((nw, nu))
    off = np.zeros(g.n + 1, dtype=np.int64)
    np.add.at(off, nu + 1, 1)
    g2 = gg.Graph(np.cumsum(off).astype(np.int32), nw[order].astype(np.int32))
    d1, d2 = dev(pg, g), dev(pg, g2)
    for s in [0, 17, 4999]:
        a = np_dist(pg.bfs(d1, s))
        b = np_dist(pg.bfs(d2, int(perm[s])))
        assert np.array_equal(a, b[perm]), s
        assert np.array_equal(a, oracle.bfs(g, s))
    _ = inv


@pytest.mark.parametrize("window,min_chunk", [(1, 1), (4, 1), (16, 8), (64, 64), (0, 32)])
def test_bfs_window_and_chunk(pg, window, min_chunk):
    for g in [gg.knn(30000, 5, 6), gg.road(100, 5), gg.simple("dchain", 2000), gg.rmat(12, 8, 4)]:
        d = dev(pg, g)
        for s in gg.sources(g, 2, 31, min_degree=1):
            exp = oracle.bfs(g, int(s))
            for tau, cap in [(16, 0), (256, 0), (64, 150)]:
                _say(f"{g.name} window={window} chunk={min_chunk} tau={tau} cap={cap} src={s}")
                got = pg.bfs(d, int(s), tau=tau, window=window, min_chunk=min_chunk, frontier_capacity=cap)
                assert np.array_equal(np_dist(got), exp), (g.name, window, min_chunk, tau, cap)


@pytest.mark.parametrize("prefetch,test_first", [(True, False), (False, False), (True, True), (False, True)])
def test_relax_variants(pg, prefetch, test_first):
    for g in [gg.knn(20000, 5, 3), gg.road(90, 7), gg.rmat(12, 8, 6)]:
        d = dev(pg, g)
        for s in gg.sources(g, 2, 77, min_degree=1):
            exp = oracle.bfs(g, int(s))
            for tau, window, cap in [(1, 0, 0), (256, 0, 0), (1024, 32, 0), (64, 8, 120)]:
                _say(f"{g.name} pf={prefetch} tf={test_first} tau={tau} w={window} cap={cap} src={s}")
                got = pg.bfs(d, int(s), tau=tau, window=window, frontier_capacity=cap, prefetch=prefetch,
                             test_first=test_first)
                assert np.array_equal(np_dist(got), exp)
        srcs = gg.sources(g, 20, 78)
        exp = oracle.reach(g, srcs)
        for tau in [1, 256, 4096]:
            got = pg.reach(d, srcs, tau=tau, prefetch=prefetch, test_first=test_first)
            assert np.array_equal(np_mask(got), exp)


def test_bfs_repeatable_across_schedules(pg):
    """Schedules change, the result does not (grid-size perturbation)."""
    g = gg.knn(30000, 5, 8)
    d = dev(pg, g)
    exp = oracle.bfs(g, 123)
    for wg in [64, 128, 192, 256, 320, 448, 640, 1024]:
        for tau in [3, 17, 100]:
            got = pg.bfs(d, 123, tau=tau, wg_size=wg)
            assert np.array_equal(np_dist(got), exp), (wg, tau)


# ---------------------------------------------------------------- reach ---

@pytest.mark.parametrize("k", [1, 5, 64, 70, 130])
def test_reach_matches_oracle(pg, k):
    g = gg.road(96, 11)
    d = dev(pg, g)
    srcs = gg.sources(g, k, 1003 + k)
    exp = oracle.reach(g, srcs)
    for mode, tau, cap in [("plain", 256, 0), ("vgc", 1, 0), ("vgc", 256, 0), ("vgc", 4096, 0), ("vgc", 64, 100)]:
        _say(f"reach road96 k={k} {mode} tau={tau} cap={cap}")
        got = pg.reach(d, srcs, mode=mode, tau=tau, frontier_capacity=cap)
        assert np.array_equal(np_mask(got), exp), (k, mode, tau, cap)


IMPL_GRAPHS = [("grid80x70", lambda: gg.grid(80, 70)), ("knn30k", lambda: gg.knn(30000, 5, 4)),
               ("road120", lambda: gg.road(120, 6)), ("rmat13", lambda: gg.rmat(13, 8, 3)),
               ("dchain3000", lambda: gg.simple("dchain", 3000)),
               ("dag4000", lambda: _dag(4000, 12000, 5))]


def _dag(n, m0, seed):
    """The arcs u -> w with u < w of a random digraph: a DAG."""
    r = gg.random_graph(n, m0, seed)
    u = np.repeat(np.arange(r.n), np.diff(r.offsets))
    keep = u < r.targets
    off = np.concatenate([[0], np.cumsum(np.bincount(u[keep], minlength=n))]).astype(np.int32)
    return gg.Graph(off, r.targets[keep].astype(np.int32), name=f"dag{n}")


@pytest.mark.parametrize("name,make", IMPL_GRAPHS, ids=[x[0] for x in IMPL_GRAPHS])
def test_reach_source_implications(pg, name, make):
    """Source implications (on by default for several sources): sources that
    reach each other (grids, the giant component of k-NN), one-way chains of
    implications (a directed chain, a DAG) and many small components (road);
    on and off, at several schedules, up to two mask words, and with
    repeated sources (which imply each other from the start)."""
    g = make()
    d = dev(pg, g)
    for k in [2, 16, 64, 100]:
        srcs = gg.sources(g, k, 2000 + k)
        if k == 16:
            srcs = np.concatenate([srcs, srcs[:3]])
        exp = oracle.reach(g, srcs)
        for kw in [dict(), dict(implications=False), dict(tau=1), dict(tau=64, frontier_capacity=100),
                   dict(test_first=True), dict(test_first=False, prefetch=False), dict(half_device=True, wg_size=512)]:
            _say(f"implications {name} k={len(srcs)} {kw}")
            assert np.array_equal(np_mask(pg.reach(d, srcs, **kw)), exp), (k, kw)


def test_reach_duplicate_sources_and_families(pg):
    for g in [gg.simple("dchain", 2000), gg.simple("dcycle", 300), gg.simple("empty", 50), gg.knn(3000, 5, 1)]:
        d = dev(pg, g)
        srcs = np.array([0, g.n - 1, 0, g.n // 3, g.n - 1], dtype=np.int32)
        exp = oracle.reach(g, srcs)
        for mode in ["plain", "vgc"]:
            _say(f"reach {g.name} {mode}")
            assert np.array_equal(np_mask(pg.reach(d, srcs, mode=mode)), exp)


def test_transpose_and_backward_reach_scc_partition(pg):
    g = gg.road(128, 3)
    d = dev(pg, g)
    _say("transpose road128")
    t = pg.transpose(d)
    t_off, t_tgt = oracle.transpose(g)
    got_off = t.offsets.cpu().numpy()
    got_tgt = t.targets.cpu().numpy()
    assert np.array_equal(got_off, t_off)
    for v in range(0, g.n, 97):
        assert np.array_equal(np.sort(got_tgt[got_off[v]:got_off[v + 1]]), t_tgt[t_off[v]:t_off[v + 1]])
    assert np.array_equal(np.sort(got_tgt), np.sort(t_tgt))
    gt = gg.Graph(t_off, t_tgt)
    pivots = gg.sources(g, 64, 1003)
    fw = np_mask(pg.reach(d, pivots))
    bw = np_mask(pg.reach(t, pivots))
    assert np.array_equal(fw, oracle.reach(g, pivots))
    assert np.array_equal(bw, oracle.reach(gt, pivots))
    comp = oracle.scc(g)
    for i, p in enumerate(pivots):
        both = ((fw[:, 0] & bw[:, 0]) >> np.uint64(i)) & np.uint64(1)
        assert np.array_equal(both.astype(bool), comp == comp[p]), i


def test_transpose_degenerate(pg):
    for g in [gg.simple("empty", 10), gg.simple("star", 3000), gg.rmat(12, 8, 1)]:
        d = dev(pg, g)
        t = pg.transpose(d)
        t_off, t_tgt = oracle.transpose(g)
        assert np.array_equal(t.offsets.cpu().numpy(), t_off)
        got = t.targets.cpu().numpy()
        for v in range(g.n):
            assert np.array_equal(np.sort(got[t_off[v]:t_off[v + 1]]), t_tgt[t_off[v]:t_off[v + 1]])


# --------------------------------------------------------------- errors ---

def test_error_paths_leave_outputs_untouched(pg):
    import ctypes
    from paper_2404_17101_amd import _lib as L
    lib = pg.load()
    g = gg.grid(8, 8)
    d = dev(pg, g)
    out = torch.full((g.n,), 12345, dtype=torch.int32, device="cuda")
    csr = d.csr()
    assert lib.pasgal_bfs(ctypes.byref(csr), -1, out.data_ptr()) == -1
    assert lib.pasgal_bfs(ctypes.byref(csr), g.n, out.data_ptr()) == -1
    assert lib.pasgal_bfs(ctypes.byref(csr), 0, None) == -1
    assert lib.pasgal_bfs(None, 0, out.data_ptr()) == -1
    bad = L.Csr(0, 0, csr.offsets, csr.targets)
    assert lib.pasgal_bfs(ctypes.byref(bad), 0, out.data_ptr()) == -1
    src = (ctypes.c_int32 * 2)(0, 64)
    lab = torch.full((g.n,), 7, dtype=torch.int64, device="cuda")
    assert lib.pasgal_reach(ctypes.byref(csr), src, 2, lab.data_ptr()) == -1
    assert lib.pasgal_reach(ctypes.byref(csr), src, 0, lab.data_ptr()) == -1
    torch.cuda.synchronize()
    assert int((out != 12345).sum()) == 0
    assert int((lab != 7).sum()) == 0
    # malformed CSR is caught with the validate flag
    off = g.offsets.copy()
    tgt = g.targets.copy()
    tgt[5] = g.n + 3
    bad_g = pg.DeviceGraph.from_numpy(off, tgt)
    assert not pg.validate(bad_g)
    assert pg.validate(d)
    with pytest.raises(pg.PasgalError) as ei:
        pg.bfs(bad_g, 0, validate=True)
    assert ei.value.code == -4
    off2 = g.offsets.copy()
    off2[3] = off2[4] + 1
    assert not pg.validate(pg.DeviceGraph.from_numpy(off2, g.targets))


# ---------------------------------------------------------------- batch ---

def _batch_inputs(pg, graphs, per_graph, seed):
    packed = gg.pack(graphs)
    pd = pg.DeviceGraph.from_numpy(packed.offsets, packed.targets)
    qg, qs, qo = [], [], []
    off = 0
    for gi, g in enumerate(graphs):
        srcs = gg.sources(g, min(per_graph, g.n), seed + gi)
        for s in srcs:
            qg.append(gi)
            qs.append(int(s))
            qo.append(off)
            off += g.n
    dist = torch.empty(off, dtype=torch.int32, device="cuda")
    return packed, pd, np.array(qg), np.array(qs), np.array(qo, dtype=np.int64), dist


def test_batch_matches_single_and_oracle(pg):
    graphs = [gg.grid(40, 70), gg.knn(3000, 5, 3), gg.road(50, 2), gg.simple("dchain", 500), gg.grid(1, 1),
              gg.knn(800, 5, 9), gg.rmat(10, 8, 3)]
    packed, pd, qg, qs, qo, dist = _batch_inputs(pg, graphs, 3, 100)
    for cap in [0, 300]:
        _say(f"batch cap={cap}")
        b = pg.Batch(pd, packed.vbase, qg, qs, qo, dist, tau=64, frontier_capacity=cap)
        for rep in range(3):
            dist.fill_(-7)
            b.run()
            got = dist.cpu().numpy()
            for j in range(len(qg)):
                g = graphs[qg[j]]
                exp = oracle.bfs(g, int(qs[j]))
                assert np.array_equal(got[qo[j]:qo[j] + g.n], exp), (cap, rep, j)
            # eager work between graph replays
            single = np_dist(pg.bfs(dev(pg, graphs[0]), int(qs[0])))
            assert np.array_equal(single, got[qo[0]:qo[0] + graphs[0].n])
        b.close()


def test_batch_autotune(pg):
    graphs = [gg.grid(30, 30), gg.knn(2000, 5, 5)]
    packed, pd, qg, qs, qo, dist = _batch_inputs(pg, graphs, 4, 7)
    b = pg.Batch(pd, packed.vbase, qg, qs, qo, dist, autotune=True)
    cfg = b.config()
    assert cfg["tau"] in (16, 64, 256, 1024, 4096)
    # the default capacity here is 2^20 entries; the tuner may shrink it 4x or 16x
    assert cfg["frontier_capacity"] in (1 << 20, 1 << 18, 1 << 16)
    for rep in range(2):
        dist.fill_(7)
        b.run()
        got = dist.cpu().numpy()
        for j in range(len(qg)):
            g = graphs[qg[j]]
            assert np.array_equal(got[qo[j]:qo[j] + g.n], oracle.bfs(g, int(qs[j]))), (rep, j)
    b.close()


# --------------------------------------------------------------- server ---

def test_server_results_equal_alone_and_in_mix(pg):
    g1, g2 = gg.grid(60, 60), gg.rmat(11, 8, 2)
    srv = pg.Server(max_slots=8, slice_rounds=4, tau=64)
    d1, d2 = dev(pg, g1), dev(pg, g2)
    ids = [srv.add_graph(d1), srv.add_graph(d2)]
    reqs = []
    for i in range(24):
        gid = ids[i % 2]
        g = g1 if gid == ids[0] else g2
        kind = "bfs" if i % 3 else "reach"
        if kind == "bfs":
            srcs = [int(gg.sources(g, 1, 500 + i, min_degree=1)[0])]
            out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        else:
            srcs = list(gg.sources(g, 1 + i % 5, 600 + i, min_degree=1))
            out = torch.empty(g.n, dtype=torch.int64, device="cuda")
        rid = srv.submit(gid, kind, srcs, out=out, tag=i)
        assert rid is not None
        reqs.append((rid, g, kind, srcs, out))
    srv.drain(60000)
    comps = {c["id"]: c for c in srv.poll(1000)}
    assert len(comps) == len(reqs)
    for rid, g, kind, srcs, out in reqs:
        assert comps[rid]["status"] == 0
        if kind == "bfs":
            assert np.array_equal(np_dist(out), oracle.bfs(g, srcs[0])), rid
        else:
            assert np.array_equal(np_mask(out)[:, None] if out.dim() == 1 else np_mask(out),
                                  oracle.reach(g, srcs)), rid
    srv.close()


def test_server_tiny_budget_queues_admission(pg):
    g = gg.grid(100, 100)
    per_req = 4 * g.n + 4 * ((g.n + 31) // 32) + 512
    srv = pg.Server(memory_budget=per_req + per_req // 2, max_slots=16, slice_rounds=8)
    gid = srv.add_graph(dev(pg, g))
    outs = []
    for i in range(6):
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        s = int(gg.sources(g, 1, 40 + i)[0])
        assert srv.submit(gid, "bfs", [s], out=out) is not None
        outs.append((s, out))
    srv.drain(60000)
    comps = srv.poll(100)
    assert len(comps) == 6 and all(c["status"] == 0 for c in comps)
    # only one request fits at a time: admissions are serialized
    comps.sort(key=lambda c: c["t_admit_ms"])
    for a, b in zip(comps, comps[1:]):
        assert b["t_admit_ms"] >= a["t_done_ms"] - 5.0
    for s, out in outs:
        assert np.array_equal(np_dist(out), oracle.bfs(g, s))
    srv.close()


@pytest.mark.parametrize("fixed", [False, True])
def test_server_lone_request_long_launch(pg, fixed):
    """A request served alone: by default one launch runs until it is done
    (no per-slice round trips); with fixed slices every launch stops after
    slice_rounds. Both give the oracle's results."""
    g = gg.grid(120, 90)
    srv = pg.Server(max_slots=8, slice_rounds=4, tau=64, fixed_slices=fixed)
    gid = srv.add_graph(dev(pg, g))
    for i, kind in enumerate(["bfs", "reach", "bfs"]):
        _say(f"lone request fixed={fixed} {kind}")
        src = int(gg.sources(g, 1, 700 + i)[0])
        out = torch.empty(g.n, dtype=torch.int32 if kind == "bfs" else torch.int64, device="cuda")
        assert srv.submit(gid, kind, [src], out=out, tag=i) is not None
        srv.drain(60000)
        (c,) = srv.poll(10)
        assert c["status"] == 0 and c["tag"] == i
        if kind == "bfs":
            assert np.array_equal(np_dist(out), oracle.bfs(g, src))
        else:
            assert np.array_equal(np_mask(out)[:, None], oracle.reach(g, [src]))
    srv.close()


def test_server_submission_ends_long_launch(pg):
    """A long launch for a lone request ends at the next round boundary once
    another request is submitted: the second (small) request is admitted and
    finishes while the first is still being traversed."""
    big, small = gg.grid(4096, 4096), gg.grid(32, 32)
    srv = pg.Server(max_slots=8, slice_rounds=8)
    gb, gs = srv.add_graph(dev(pg, big)), srv.add_graph(dev(pg, small))
    out_b = torch.empty(big.n, dtype=torch.int32, device="cuda")
    out_s = torch.empty(small.n, dtype=torch.int32, device="cuda")
    _say("long launch: big grid from corner 0")
    assert srv.submit(gb, "bfs", [0], out=out_b, tag=1) is not None
    import time
    t0 = time.perf_counter()
    while srv.load_info()["active"] == 0 and time.perf_counter() - t0 < 10:
        time.sleep(0.0002)
    time.sleep(0.002)
    _say("second request during the long launch")
    assert srv.submit(gs, "bfs", [5], out=out_s, tag=2) is not None
    srv.drain(60000)
    comps = {c["tag"]: c for c in srv.poll(10)}
    assert comps[1]["status"] == 0 and comps[2]["status"] == 0
    assert comps[2]["t_done_ms"] < comps[1]["t_done_ms"], comps
    r, c = np.divmod(np.arange(big.n), 4096)
    assert np.array_equal(np_dist(out_b), (r + c).astype(np.int32))
    assert np.array_equal(np_dist(out_s), oracle.bfs(small, 5))
    srv.close()


def test_server_lone_launch_hands_back_overflow(pg):
    """A lone request runs in the single-query kernel; with a frontier of
    1024 entries its overflow goes to the global-id dirty bitmap. A second
    submission ends the launch at a round boundary, and the frontier entries
    and dirty bits move to the request's own (multi-query) layout: both
    requests still give exact results. The big grid's second graph offset is
    not a multiple of 32, so the bitmap handover shifts words."""
    small, big = gg.grid(33, 33), gg.grid(2048, 2048)
    srv = pg.Server(max_slots=8, slice_rounds=8, frontier_capacity=1024)
    gs, gb = srv.add_graph(dev(pg, small)), srv.add_graph(dev(pg, big))
    assert small.n % 32 != 0
    out_b = torch.empty(big.n, dtype=torch.int32, device="cuda")
    out_s = torch.empty(small.n, dtype=torch.int32, device="cuda")
    _say("lone launch with a 1024-entry frontier: big grid from corner 0")
    assert srv.submit(gb, "bfs", [0], out=out_b, tag=1) is not None
    import time
    t0 = time.perf_counter()
    while srv.load_info()["active"] == 0 and time.perf_counter() - t0 < 10:
        time.sleep(0.0002)
    time.sleep(0.003)
    assert srv.submit(gs, "bfs", [7], out=out_s, tag=2) is not None
    srv.drain(120000)
    comps = {c["tag"]: c for c in srv.poll(10)}
    assert comps[1]["status"] == 0 and comps[2]["status"] == 0
    r, c = np.divmod(np.arange(big.n), 2048)
    assert np.array_equal(np_dist(out_b), (r + c).astype(np.int32))
    assert np.array_equal(np_dist(out_s), oracle.bfs(small, 7))
    srv.close()


@pytest.mark.parametrize("direction_optimizing", [True, False])
def test_server_dense_graph_bfs(pg, direction_optimizing):
    """BFS and single-source reach requests on a graph with mean out-degree
    above 8 are served by the direction-optimizing BFS by default (from the
    server's own copy of the graph and its transpose), reach requests with
    several sources by the batched launches; with direction optimization off
    everything is batched. Results as the oracle's, also for requests whose
    result is dropped (out=None) between others, and for a directed dense
    graph (transpose differs)."""
    gs = gg.rmat(11, 8, 3)
    gd = gg.random_graph(3000, 36000, 11, symmetric=False)
    assert gs.m > 8 * gs.n and gd.m > 8 * gd.n
    srv = pg.Server(max_slots=8, slice_rounds=4, direction_optimizing=direction_optimizing)
    ids = [srv.add_graph(dev(pg, gs)), srv.add_graph(dev(pg, gd))]
    reqs = []
    for i in range(16):
        gi = i % 2
        g = (gs, gd)[gi]
        kind = "reach" if i % 4 == 3 or i == 6 else "bfs"
        srcs = [int(x) for x in gg.sources(g, 3 if i % 8 == 7 else 1, 800 + i, min_degree=1)]
        out = None
        if i not in (5, 6):
            out = torch.empty(g.n, dtype=torch.int32 if kind == "bfs" else torch.int64, device="cuda")
        _say(f"dense server do={direction_optimizing} req {i} {kind} graph {gi} sources {len(srcs)}")
        assert srv.submit(ids[gi], kind, srcs, out=out, tag=i) is not None
        reqs.append((i, g, kind, srcs, out))
    srv.drain(60000)
    comps = {c["tag"]: c for c in srv.poll(100)}
    assert len(comps) == len(reqs)
    for i, g, kind, srcs, out in reqs:
        assert comps[i]["status"] == 0, i
        if out is None:
            continue
        if kind == "bfs":
            assert np.array_equal(np_dist(out), oracle.bfs(g, srcs[0])), i
        else:
            assert np.array_equal(np_mask(out)[:, None], oracle.reach(g, srcs)), i
    assert srv.load_info()["active"] == 0
    srv.close()


def test_server_dense_batches_split_at_64(pg):
    """More than 64 direction-optimizing requests queued on one dense graph
    (and a few on another) are served in several multi-source batches; every
    result equals the oracle's."""
    ga, gb = gg.rmat(10, 12, 4), gg.random_graph(1500, 18000, 13, symmetric=False)
    assert ga.m > 8 * ga.n and gb.m > 8 * gb.n
    srv = pg.Server(max_slots=8)
    ia, ib = srv.add_graph(dev(pg, ga)), srv.add_graph(dev(pg, gb))
    reqs = []
    srcs_a = [int(x) for x in gg.sources(ga, 80, 900, min_degree=1)]
    _say("dense batches: 80 + 6 direction-optimizing requests")
    for i, s in enumerate(srcs_a):
        kind = "bfs" if i % 3 else "reach"
        out = torch.empty(ga.n, dtype=torch.int32 if kind == "bfs" else torch.int64, device="cuda")
        assert srv.submit(ia, kind, [s], out=out, tag=i) is not None
        reqs.append((i, ga, kind, s, out))
    for j, s in enumerate(int(x) for x in gg.sources(gb, 6, 901, min_degree=1)):
        out = torch.empty(gb.n, dtype=torch.int32, device="cuda")
        assert srv.submit(ib, "bfs", [s], out=out, tag=1000 + j) is not None
        reqs.append((1000 + j, gb, "bfs", s, out))
    srv.drain(60000)
    comps = {c["tag"]: c for c in srv.poll(1000)}
    assert len(comps) == len(reqs)
    for tag, g, kind, s, out in reqs:
        assert comps[tag]["status"] == 0, tag
        if kind == "bfs":
            assert np.array_equal(np_dist(out), oracle.bfs(g, s)), tag
        else:
            assert np.array_equal(np_mask(out)[:, None], oracle.reach(g, [s])), tag
    srv.close()


# ------------------------------------------------------ heavy-row slices ---

def _hub_graph(n_leaves, extra_seed):
    """Symmetric star (hub 0, degree n_leaves) plus a sprinkle of random
    symmetric arcs among the leaves, so searches run on after the hub."""
    r = gg.random_graph(n_leaves + 1, 2 * n_leaves, extra_seed, symmetric=True)
    u = np.repeat(np.arange(r.n), np.diff(r.offsets))
    leaves = np.arange(1, n_leaves + 1)
    eu = np.concatenate([u, np.zeros(n_leaves, np.int64), leaves])
    ew = np.concatenate([r.targets, leaves, np.zeros(n_leaves, np.int64)])
    key = np.unique(eu.astype(np.int64) * (n_leaves + 1) + ew)
    eu, ew = key // (n_leaves + 1), key % (n_leaves + 1)
    off = np.zeros(n_leaves + 2, dtype=np.int64)
    np.add.at(off, eu + 1, 1)
    return gg.Graph(np.cumsum(off).astype(np.int32), ew.astype(np.int32))


@pytest.mark.parametrize("heavy", [16, 64, 1000])
def test_heavy_rows_cut_into_slices_bfs_reach(pg, heavy):
    """Rows longer than heavy_arcs are dealt out as slices; results stay exact
    (RMAT hubs, a star hub, and a slice buffer too small for the slices)."""
    for g in [gg.rmat(13, 16, 4), _hub_graph(20000, 71)]:
        d = dev(pg, g)
        srcs = [int(s) for s in gg.sources(g, 3, 72, min_degree=1)]
        for kw in [dict(heavy_arcs=heavy), dict(heavy_arcs=heavy, frontier_capacity=64),
                   dict(heavy_arcs=heavy, tau=16, window=0)]:
            for s in srcs:
                _say(f"heavy bfs {g.name} n={g.n} src={s} {kw}")
                assert np.array_equal(np_dist(pg.bfs(d, s, **kw)), oracle.bfs(g, s)), (s, kw)
            _say(f"heavy reach {g.name} {kw}")
            assert np.array_equal(np_mask(pg.reach(d, srcs, **kw)), oracle.reach(g, srcs)), kw


def test_heavy_rows_batch_scc_and_server(pg):
    g = _hub_graph(30000, 73)
    x = gg.rmat(12, 16, 6)
    graphs = [g, x]
    packed = gg.pack(graphs)
    pd = pg.DeviceGraph.from_numpy(packed.offsets, packed.targets)
    qg, qs, qo, off = [], [], [], 0
    for gi, gr in enumerate(graphs):
        for s in gg.sources(gr, 6, 74 + gi, min_degree=1):
            qg.append(gi)
            qs.append(int(s))
            qo.append(off)
            off += gr.n
    dist = torch.empty(off, dtype=torch.int32, device="cuda")
    for heavy in [32, 0]:
        _say(f"heavy batch heavy={heavy}")
        b = pg.Batch(pd, packed.vbase, np.array(qg), np.array(qs), np.array(qo, dtype=np.int64), dist,
                     heavy_arcs=heavy)
        b.run()
        got = dist.cpu().numpy()
        b.close()
        for j in range(len(qg)):
            gr = graphs[qg[j]]
            assert np.array_equal(got[qo[j]:qo[j] + gr.n], oracle.bfs(gr, qs[j])), (heavy, j)
    # SCC over a directed graph with hubs
    y = gg.rmat(12, 16, 7)
    keep = np.random.default_rng(75).random(y.m) < 0.6
    u = np.repeat(np.arange(y.n), np.diff(y.offsets))[keep]
    off2 = np.zeros(y.n + 1, dtype=np.int64)
    np.add.at(off2, u + 1, 1)
    yd = gg.Graph(np.cumsum(off2).astype(np.int32), y.targets[keep].astype(np.int32))
    for heavy in [8, 0]:
        _say(f"heavy scc heavy={heavy}")
        got = pg.scc(dev(pg, yd), heavy_arcs=heavy).cpu().numpy()
        assert np.array_equal(got, oracle.scc_min_label(yd)), heavy
    # the served form stops launches after slice_rounds (hub degree 30000 >
    # the default 4096); no slice may be left behind at a launch's end
    for rounds in [1, 2, 3]:
        _say(f"heavy server slice_rounds={rounds}")
        srv = pg.Server(max_slots=8, slice_rounds=rounds, tau=64)
        gid = srv.add_graph(dev(pg, g))
        reqs = []
        for i in range(6):
            s = int(gg.sources(g, 1, 76 + i, min_degree=1)[0])
            kind = "bfs" if i % 2 == 0 else "reach"
            out = torch.empty(g.n, dtype=torch.int32 if kind == "bfs" else torch.int64, device="cuda")
            assert srv.submit(gid, kind, [s], out=out) is not None
            reqs.append((s, kind, out))
        srv.drain(60000)
        comps = srv.poll(100)
        assert len(comps) == 6 and all(c["status"] == 0 for c in comps)
        for s, kind, out in reqs:
            if kind == "bfs":
                assert np.array_equal(np_dist(out), oracle.bfs(g, s)), (rounds, s)
            else:
                assert np.array_equal(np_mask(out)[:, None], oracle.reach(g, [s])), (rounds, s)
        srv.close()


@pytest.mark.parametrize("slots", [-1, 16, 4096])
def test_lds_filter_sizes_keep_results_exact(pg, slots):
    """The per-wavefront filter only skips relaxations that cannot win; any
    size (16 forces constant slot collisions, 4096 squeezes the ring) and off
    give the same exact results, single-query, batched and weighted."""
    g = gg.knn(30000, 5, 12)
    d = dev(pg, g)
    srcs = [int(s) for s in gg.sources(g, 3, 91)]
    for s in srcs:
        _say(f"filter {slots} bfs src={s}")
        assert np.array_equal(np_dist(pg.bfs(d, s, filter_slots=slots)), oracle.bfs(g, s))
    w = gg.weights(g, 92, 1, 300)
    wd = torch.from_numpy(w.view(np.int32)).cuda()
    got = pg.sssp(d, wd, srcs[0], filter_slots=slots).cpu().numpy().view(np.uint32).astype(np.int64)
    got[got == 0xFFFFFFFF] = -1
    assert np.array_equal(got, oracle.sssp(g, w, srcs[0]))
    graphs = [g, gg.grid(70, 90)]
    packed, pd, qg, qs, qo, dist = _batch_inputs(pg, graphs, 5, 93)
    b = pg.Batch(pd, packed.vbase, qg, qs, qo, dist, filter_slots=slots)
    b.run()
    out = dist.cpu().numpy()
    b.close()
    for j in range(len(qg)):
        gr = graphs[qg[j]]
        assert np.array_equal(out[qo[j]:qo[j] + gr.n], oracle.bfs(gr, int(qs[j]))), (slots, j)
