"""paper_2404_17101_amd -- VGC graph traversal on one AMD Instinct MI355X.

Thin Python binding over libpasgal.so (C ABI in include/pasgal.h). Every
function here only marshals arguments: torch tensors supply device memory and
the current HIP stream, and every step of the traversal runs in the library's
gfx950 kernels. There is no CPU fallback: if the library is missing, calls
raise.

Operations (PASGAL, SPAA'24): BFS hop distances with vertical granularity
control (Parallel BFS), multi-source reachability (Parallel SCC section), the
transpose G^T for backward reachability, strongly connected components by
batched forward/backward reachability (Parallel SCC section), a batched form
and a served form.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib as L

__all__ = ["DeviceGraph", "PasgalError", "bfs", "bfs_noalloc", "bfs_do", "sssp", "reach", "device_sources", "wait", "transpose",
           "validate", "scc", "Batch", "Server", "load"]

load = L.load


class PasgalError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = L.load()
        msg = lib.pasgal_strerror(code).decode()
        extra = f" (hipError {lib.pasgal_last_hip_error()})" if code == -3 else ""
        super().__init__(f"{where}: {L.ERRORS.get(code, code)} {msg}{extra}")
        self.code = code


def _check(rc: int, where: str):
    if rc != 0:
        raise PasgalError(rc, where)


def _torch():
    import torch

    return torch


@dataclass
class DeviceGraph:
    """int32 CSR resident on the GPU (torch tensors)."""

    offsets: "object"
    targets: "object"

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.targets.shape[0])

    @classmethod
    def from_numpy(cls, offsets: np.ndarray, targets: np.ndarray, device: str = "cuda") -> "DeviceGraph":
        torch = _torch()
        off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int32)).to(device)
        tgt = torch.from_numpy(np.ascontiguousarray(targets, dtype=np.int32))
        if tgt.numel() == 0:
            tgt = torch.zeros(1, dtype=torch.int32)
            out = cls(off, tgt.to(device)[:0])
            out._pad = tgt.to(device)
            return out
        return cls(off, tgt.to(device))

    @classmethod
    def from_graph(cls, g, device: str = "cuda") -> "DeviceGraph":
        return cls.from_numpy(g.offsets, g.targets, device)

    def csr(self) -> L.Csr:
        tp = self.targets.data_ptr() if self.m > 0 else getattr(self, "_pad", self.targets).data_ptr()
        return L.Csr(self.n, self.m, self.offsets.data_ptr(), tp)


def _stream_ptr(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _opts(mode="vgc", tau=0, wg_size=1024, blocks_per_cu=1, frontier_capacity=0, validate=False, timeout_ms=20000,
          stream=None, asynchronous=False, window=32, min_chunk=1, prefetch=None, test_first=None,
          heavy_arcs=0, filter_slots=0, chunks_per_wave=0, half_device=False, implications=True,
          device_share=0) -> L.Opts:
    """tau: local-search budget (0 = the entry point's default: 1024, SSSP and
    SCC on graphs of mean out-degree above 8: 1). window: BFS distance window per
    round (0 or negative = none).
    heavy_arcs: rows with more arcs are cut into slices dealt to all
    wavefronts (0 = default 512, negative = never). filter_slots: per-wavefront
    LDS filter of BFS/SSSP relaxations (0 = default 256, negative = off).
    half_device: the persistent launch takes half of every compute unit, so
    that a second such call on another stream runs beside it; device_share:
    the same with any percentage (1..99) of every compute unit. test_first:
    None = the entry point's default (on for reach with several sources on
    graphs of mean degree >= 4 and for SCC on graphs of mean degree > 8),
    True / False = always / never read before the atomic. prefetch: None =
    the entry point's default (on for single-source BFS, SSSP, reach and SCC), True / False = always /
    never carry arc ranges in the local queue."""
    o = L.Opts()
    L.load().pasgal_opts_default(ctypes.byref(o))
    o.mode = {"vgc": L.MODE_VGC, "plain": L.MODE_PLAIN}[mode]
    o.tau = int(tau)
    o.wg_size = int(wg_size)
    o.blocks_per_cu = int(blocks_per_cu)
    o.frontier_capacity = int(frontier_capacity)
    o.flags = ((L.FLAG_VALIDATE if validate else 0) | (L.FLAG_ASYNC if asynchronous else 0) |
               (0 if prefetch is None else (L.FLAG_PREFETCH if prefetch else L.FLAG_NO_PREFETCH)) |
               (0 if test_first is None else (L.FLAG_TEST_FIRST if test_first else L.FLAG_NO_TEST_FIRST)) |
               (L.FLAG_HALF_DEVICE if half_device else 0) | (0 if implications else L.FLAG_NO_IMPLICATIONS))
    o.timeout_ms = int(timeout_ms)
    o.stream = _stream_ptr(stream)
    o.window = int(window) if int(window) > 0 else -1
    o.min_chunk = int(min_chunk)
    o.heavy_arcs = int(heavy_arcs)
    o.filter_slots = int(filter_slots)
    o.chunks_per_wave = int(chunks_per_wave)
    o.device_share = int(device_share)
    return o


def bfs(g: DeviceGraph, src: int, dist_out=None, stats: bool = False, **opts):
    """Hop distances from src (int32 tensor, -1 = unreachable). With
    stats=True also returns the call's counters as a dict."""
    torch = _torch()
    if dist_out is None:
        dist_out = torch.empty(g.n, dtype=torch.int32, device=g.offsets.device)
    csr = g.csr()
    o = _opts(**opts)
    st = L.Stats()
    _check(L.load().pasgal_bfs_ex(ctypes.byref(csr), int(src), dist_out.data_ptr(), ctypes.byref(o),
                                  ctypes.byref(st)), "pasgal_bfs")
    return (dist_out, st.as_dict()) if stats else dist_out


def bfs_noalloc(g: DeviceGraph, src: int, dist_out=None, stats: bool = False, **opts):
    """pasgal_bfs_noalloc: the distances of bfs() with every library buffer
    taken from the library's fixed device array (no allocation inside the
    call; dist_out, when given, is the caller's)."""
    torch = _torch()
    if dist_out is None:
        dist_out = torch.empty(g.n, dtype=torch.int32, device=g.offsets.device)
    csr = g.csr()
    o = _opts(**opts)
    st = L.Stats()
    _check(L.load().pasgal_bfs_noalloc(ctypes.byref(csr), int(src), dist_out.data_ptr(), ctypes.byref(o),
                                       ctypes.byref(st)), "pasgal_bfs_noalloc")
    return (dist_out, st.as_dict()) if stats else dist_out


def bfs_do(g: DeviceGraph, src: int, transpose: DeviceGraph | None = None, dist_out=None, alpha: int = 0,
           beta: int = 0, stats: bool = False, **opts):
    """Direction-optimizing BFS (top-down / bottom-up levels). transpose: G^T;
    None only when g is symmetric. alpha / beta: switching thresholds (0 =
    defaults 100 / 24, negative = never switch that way). Same output as bfs."""
    torch = _torch()
    if dist_out is None:
        dist_out = torch.empty(g.n, dtype=torch.int32, device=g.offsets.device)
    csr = g.csr()
    tcsr = transpose.csr() if transpose is not None else None
    o = _opts(**opts)
    st = L.Stats()
    _check(L.load().pasgal_bfs_do(ctypes.byref(csr), ctypes.byref(tcsr) if tcsr is not None else None, int(src),
                                  dist_out.data_ptr(), int(alpha), int(beta), ctypes.byref(o), ctypes.byref(st)),
           "pasgal_bfs_do")
    return (dist_out, st.as_dict()) if stats else dist_out


def bfs_do_multi(g: DeviceGraph, sources, transpose: DeviceGraph | None = None, dist_out=None, reach_out=None,
                 alpha: int = 0, beta: int = 0, stats: bool = False, **opts):
    """Direction-optimizing BFS from up to 64 sources at once (one bit per
    source). dist_out: int32 tensor of k*n (row q: distances from sources[q])
    or None; reach_out: int64 tensor of n (bit q: sources[q] arrives) or
    None; with both None, dist_out is allocated. transpose as for bfs_do."""
    torch = _torch()
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
    if dist_out is None and reach_out is None:
        dist_out = torch.empty(src.size * g.n, dtype=torch.int32, device=g.offsets.device)
    csr = g.csr()
    tcsr = transpose.csr() if transpose is not None else None
    o = _opts(**opts)
    st = L.Stats()
    _check(L.load().pasgal_bfs_do_multi(ctypes.byref(csr), ctypes.byref(tcsr) if tcsr is not None else None,
                                        int(src.size), _i32p(src),
                                        dist_out.data_ptr() if dist_out is not None else None,
                                        reach_out.data_ptr() if reach_out is not None else None,
                                        int(alpha), int(beta), ctypes.byref(o), ctypes.byref(st)),
           "pasgal_bfs_do_multi")
    out = dist_out if reach_out is None else (reach_out if dist_out is None else (dist_out, reach_out))
    return (out, st.as_dict()) if stats else out


def sssp(g: DeviceGraph, weights, src: int, dist_out=None, stats: bool = False, **opts):
    """Shortest-path distances with non-negative integer arc weights (a device
    tensor of m int32/uint32, parallel to g.targets). Returns an int32 tensor
    holding uint32 distances (0xFFFFFFFF, i.e. -1, = unreachable). window is
    the bucket width delta (0 = 8 x mean weight, negative = none)."""
    torch = _torch()
    if dist_out is None:
        dist_out = torch.empty(g.n, dtype=torch.int32, device=g.offsets.device)
    if weights.numel() != g.m:
        raise ValueError("one weight per arc")
    csr = g.csr()
    delta = int(opts.pop("window", 0))
    o = _opts(**opts)
    o.window = delta if delta >= 0 else -1
    st = L.Stats()
    wp = weights.data_ptr() if g.m > 0 else None
    _check(L.load().pasgal_sssp(ctypes.byref(csr), wp, int(src), dist_out.data_ptr(), ctypes.byref(o),
                                ctypes.byref(st)), "pasgal_sssp")
    return (dist_out, st.as_dict()) if stats else dist_out


def device_sources(sources, device, stream=None):
    """The int32 device array of source ids that pasgal_reach takes: a CUDA
    tensor is used as it is (converted to contiguous int32 if needed), host
    data is copied on `stream` (default: the current stream), so that the
    library, reading it on that stream, sees the copy."""
    torch = _torch()
    if isinstance(sources, torch.Tensor) and sources.is_cuda:
        return sources.to(torch.int32).contiguous().view(-1)
    src = torch.from_numpy(np.ascontiguousarray(np.asarray(sources, dtype=np.int32).ravel()))
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
        return src.to(device)


def reach(g: DeviceGraph, sources, label_out=None, stats: bool = False, **opts):
    """Reachability masks: int64 tensor [n, ceil(k/64)]; bit i%64 of word i/64
    of row v is set iff sources[i] reaches v. sources: a CUDA int32 tensor
    (passed to the library as it is) or host ids (copied to the device on the
    call's stream)."""
    torch = _torch()
    src = device_sources(sources, g.offsets.device, opts.get("stream"))
    k = int(src.numel())
    words = max(1, (k + 63) // 64)
    if label_out is None:
        label_out = torch.empty((g.n, words), dtype=torch.int64, device=g.offsets.device)
    csr = g.csr()
    o = _opts(**opts)
    st = L.Stats()
    _check(L.load().pasgal_reach_ex(ctypes.byref(csr), ctypes.cast(src.data_ptr(), ctypes.POINTER(ctypes.c_int32)), k,
                                    label_out.data_ptr(), ctypes.byref(o), ctypes.byref(st)), "pasgal_reach")
    return (label_out, st.as_dict()) if stats else label_out


def wait(stream=None):
    """pasgal_wait: wait for the library's work on the stream (default: the
    current one); raises PasgalError (ETIMEOUT) if an asynchronous launch there
    timed out."""
    _check(L.load().pasgal_wait(_stream_ptr(stream)), "pasgal_wait")


def transpose(g: DeviceGraph, **opts) -> DeviceGraph:
    """G^T on the device (row order inside a row unspecified)."""
    torch = _torch()
    t_off = torch.empty(g.n + 1, dtype=torch.int32, device=g.offsets.device)
    t_tgt = torch.empty(max(g.m, 1), dtype=torch.int32, device=g.offsets.device)
    csr = g.csr()
    o = _opts(**opts)
    _check(L.load().pasgal_transpose(ctypes.byref(csr), t_off.data_ptr(), t_tgt.data_ptr(), ctypes.byref(o)),
           "pasgal_transpose")
    out = DeviceGraph(t_off, t_tgt[: g.m])
    if g.m == 0:
        out._pad = t_tgt
    return out


PROBE_KINDS = {"load": 0, "coherent": 1, "atomic": 2}


def probe_latency(nbytes: int, steps: int = 20000, kind: str = "load", **opts) -> float:
    """Mean ns of one dependent device-memory access over a buffer of about
    nbytes (a random single cycle walked by one lane): the per-level floor of
    a traversal. kind: "load" (cached), "coherent" (agent-scope load) or
    "atomic" (agent-scope atomic add of 0)."""
    ns = ctypes.c_double()
    o = _opts(**opts)
    _check(L.load().pasgal_probe_latency(int(nbytes), int(steps), PROBE_KINDS[kind], ctypes.byref(ns), ctypes.byref(o)),
           "pasgal_probe_latency")
    return ns.value


def validate(g: DeviceGraph, **opts) -> bool:
    csr = g.csr()
    o = _opts(**opts)
    rc = L.load().pasgal_validate(ctypes.byref(csr), ctypes.byref(o))
    if rc == -4:
        return False
    _check(rc, "pasgal_validate")
    return True


def scc(g: DeviceGraph, transpose: DeviceGraph | None = None, comp_out=None, trim_rounds: int = -1,
        split: bool = True, seed: int = 0, stats: bool = False, **opts):
    """Strongly connected components: int32 tensor [n], entry v = the smallest
    vertex of v's component. transpose: G^T if already built (else built
    inside the call). trim_rounds < 0 selects the default, 0 disables
    trimming; split=False keeps subproblems whole (no weak-connectivity cut);
    seed keys the random pivot order (0 = default; the result does not depend
    on it). With stats=True also returns the call's counters as a dict."""
    torch = _torch()
    if comp_out is None:
        comp_out = torch.empty(g.n, dtype=torch.int32, device=g.offsets.device)
    csr = g.csr()
    tcsr = transpose.csr() if transpose is not None else None
    o = _opts(**opts)
    so = L.SccOpts(int(trim_rounds), 0 if split else L.SCC_NO_SPLIT, int(seed) & 0xFFFFFFFF, 0)
    st = L.SccStats()
    _check(L.load().pasgal_scc(ctypes.byref(csr), ctypes.byref(tcsr) if tcsr is not None else None,
                               comp_out.data_ptr(), ctypes.byref(so), ctypes.byref(o), ctypes.byref(st)),
           "pasgal_scc")
    return (comp_out, st.as_dict()) if stats else comp_out


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Batch:
    """Many BFS queries over a packed CSR in one hipGraph-captured persistent
    launch. q_out[j] is the element offset of query j's distances in dist."""

    def __init__(self, packed: DeviceGraph, vbase: np.ndarray, q_graph, q_source, q_out, dist, autotune: bool = False,
                 **opts):
        self._keep = [np.ascontiguousarray(vbase, dtype=np.int32), np.ascontiguousarray(q_graph, dtype=np.int32),
                      np.ascontiguousarray(q_source, dtype=np.int32), np.ascontiguousarray(q_out, dtype=np.int64)]
        vb, qg, qs, qo = self._keep
        self.packed = packed
        self.dist = dist
        d = L.BatchDesc()
        d.packed = packed.csr()
        d.ngraphs = int(vb.size - 1)
        d.vbase = _i32p(vb)
        d.nqueries = int(qg.size)
        d.q_graph = _i32p(qg)
        d.q_source = _i32p(qs)
        d.q_out = qo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        d.dist_out = dist.data_ptr()
        d.dist_len = int(dist.numel())
        o = _opts(**opts)
        h = ctypes.c_void_p()
        _check(L.load().pasgal_batch_create(ctypes.byref(d), ctypes.byref(o), L.BATCH_AUTOTUNE if autotune else 0,
                                            ctypes.byref(h)), "pasgal_batch_create")
        self._h = h

    def run(self) -> dict:
        st = L.Stats()
        _check(L.load().pasgal_batch_run(self._h, ctypes.byref(st)), "pasgal_batch_run")
        return st.as_dict()

    def config(self) -> dict:
        o = L.Opts()
        _check(L.load().pasgal_batch_config(self._h, ctypes.byref(o)), "pasgal_batch_config")
        return {"tau": o.tau, "wg_size": o.wg_size, "blocks_per_cu": o.blocks_per_cu,
                "frontier_capacity": o.frontier_capacity}

    def close(self):
        if getattr(self, "_h", None):
            L.load().pasgal_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop over resident graphs (see
    pasgal_server_* in include/pasgal.h)."""

    def __init__(self, memory_budget: int = 0, max_slots: int = 0, slice_rounds: int = 0, tau: int = 0,
                 wg_size: int = 0, blocks_per_cu: int = 0, frontier_capacity: int = 0, timeout_ms: int = 0,
                 window: int = 0, test_first=None, fixed_slices: bool = False, direction_optimizing: bool = True):
        """test_first: None = the server's default (on in a launch holding a
        request on a graph with mean out-degree above 8), True / False =
        always / never. fixed_slices:
        every launch runs at most slice_rounds rounds, also for a request
        served alone. direction_optimizing: BFS requests on graphs with mean
        out-degree above 8 are served by the direction-optimizing BFS (False:
        by the batched launches, like every other request)."""
        flags = 0 if test_first is None else (L.FLAG_TEST_FIRST if test_first else L.FLAG_NO_TEST_FIRST)
        if fixed_slices:
            flags |= L.SERVER_FIXED_SLICES
        if not direction_optimizing:
            flags |= L.SERVER_NO_DIRECTION_OPT
        so = L.ServerOpts(int(memory_budget), int(max_slots), int(slice_rounds), int(tau), int(wg_size),
                          int(blocks_per_cu), int(frontier_capacity), int(timeout_ms), int(window), flags, 0)
        h = ctypes.c_void_p()
        _check(L.load().pasgal_server_create(ctypes.byref(so), ctypes.byref(h)), "pasgal_server_create")
        self._h = h
        self._graphs = {}

    def add_graph(self, g: DeviceGraph) -> int:
        gid = ctypes.c_int32()
        csr = g.csr()
        _check(L.load().pasgal_server_add_graph(self._h, ctypes.byref(csr), ctypes.byref(gid)),
               "pasgal_server_add_graph")
        self._graphs[gid.value] = (g.n, g.m)
        return gid.value

    def submit(self, graph: int, kind: str, sources, out=None, tag: int = 0):
        """Queue a request; returns its id, or None when the queue is full."""
        r = L.Request()
        r.graph = int(graph)
        r.kind = {"bfs": L.REQ_BFS, "reach": L.REQ_REACH}[kind]
        src = list(np.asarray(sources, dtype=np.int64).ravel())
        r.nsources = len(src)
        for i, s in enumerate(src[:64]):
            r.sources[i] = int(s)
        r.out = out.data_ptr() if out is not None else None
        r.tag = int(tag)
        rid = ctypes.c_int64()
        rc = L.load().pasgal_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid))
        if rc == -6:
            return None
        _check(rc, "pasgal_server_submit")
        return rid.value

    def poll(self, max_items: int = 1024) -> list:
        buf = (L.Completion * max_items)()
        cnt = ctypes.c_int32()
        _check(L.load().pasgal_server_poll(self._h, buf, max_items, ctypes.byref(cnt)), "pasgal_server_poll")
        return [{k: getattr(buf[i], k) for k, _ in L.Completion._fields_} for i in range(cnt.value)]

    def drain(self, timeout_ms: int = 60000):
        _check(L.load().pasgal_server_drain(self._h, int(timeout_ms)), "pasgal_server_drain")

    def load_info(self) -> dict:
        q, a, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(L.load().pasgal_server_load(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(b)),
               "pasgal_server_load")
        return {"queued": q.value, "active": a.value, "bytes": b.value}

    def close(self):
        if getattr(self, "_h", None):
            L.load().pasgal_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
