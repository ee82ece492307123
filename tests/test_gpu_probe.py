"""GPU checks of the memory-latency probe (pasgal_probe_latency), the
measurement behind the latency floor that the bench reports beside each
single-source time. A dependent access cannot be faster than a few hundred
cycles or slower than a few microseconds on an idle device, a buffer held in
L2 must not be slower than one far larger than the last-level cache, and an
atomic round trip must not be faster than a plain cached load of an L2-held
buffer."""
import sys

import pytest

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


def test_probe_latency_ranges_and_order(pg):
    res = {}
    for nbytes in (1 << 20, 1 << 30):
        for kind in ("load", "coherent", "atomic"):
            _say(f"probe {nbytes} {kind}")
            ns = pg.probe_latency(nbytes, 4000, kind)
            res[(nbytes, kind)] = ns
            assert 20.0 < ns < 20000.0, (nbytes, kind, ns)
    assert res[(1 << 20, "load")] <= res[(1 << 30, "load")] * 1.05, res
    assert res[(1 << 20, "load")] <= res[(1 << 20, "atomic")] * 1.05, res


def test_probe_latency_smallest_buffer_and_errors(pg):
    _say("probe 4 KiB")
    assert pg.probe_latency(4096, 64, "load") >= 0.0  # 10 ns clock: a short walk may read 0
    with pytest.raises(pg.PasgalError) as ei:
        pg.probe_latency(100, 10, "load")
    assert ei.value.code == -1
