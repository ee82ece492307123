"""pasgal_bfs_noalloc (the entry point for callers that cannot allocate)
through the C ABI, against the existing entry point pasgal_bfs_ex: the same
distances element by element, on two calls in a row, the second on a smaller
graph (the fixed device array keeps the first call's contents, and
everything that must start at zero is cleared by the call), plus a frontier
capacity small enough to send entries to the dirty bitmap. The reference
distances are also the oracle's."""
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


def test_noalloc_matches_bfs_ex_two_calls_second_smaller(pg):
    cases = [(gg.knn(300_000, 5, 7), dict()), (gg.road(150, 5), dict()), (gg.grid(40, 30), dict(tau=1, window=0)),
             (gg.rmat(12, 8, 4), dict(heavy_arcs=16)), (gg.knn(50_000, 5, 9), dict(frontier_capacity=100))]
    for g, kw in cases:
        d = pg.DeviceGraph.from_graph(g)
        for s in gg.sources(g, 2, 91, min_degree=1):
            _say(f"noalloc {g.name} n={g.n} src={s} {kw}")
            ref = pg.bfs(d, int(s), **kw).cpu().numpy()
            out = torch.full((g.n,), 12345, dtype=torch.int32, device="cuda")
            got, st = pg.bfs_noalloc(d, int(s), dist_out=out, stats=True, **kw)
            assert np.array_equal(got.cpu().numpy(), ref), (g.name, s, kw)
            assert np.array_equal(ref, oracle.bfs(g, int(s))), (g.name, s)
            assert st["rounds"] >= 1


def test_noalloc_rejects_what_it_cannot_hold(pg):
    """n beyond the stated maximum: PASGAL_ECAPACITY before anything runs;
    asynchronous and plain calls: PASGAL_EINVAL."""
    import ctypes

    from paper_2404_17101_amd import _lib as L
    lib = pg.load()
    off = torch.zeros(4, dtype=torch.int32, device="cuda")
    out = torch.empty(4, dtype=torch.int32, device="cuda")
    big = L.Csr((1 << 28) + 1, 0, off.data_ptr(), off.data_ptr())
    assert lib.pasgal_bfs_noalloc(ctypes.byref(big), 0, out.data_ptr(), None, None) == -5
    g = gg.grid(2, 2)
    d = pg.DeviceGraph.from_graph(g)
    for kw in [dict(asynchronous=True), dict(mode="plain"), dict(validate=True)]:
        with pytest.raises(pg.PasgalError) as ei:
            pg.bfs_noalloc(d, 0, **kw)
        assert ei.value.code == -1
    assert np.array_equal(pg.bfs_noalloc(d, 0).cpu().numpy(), oracle.bfs(g, 0))
