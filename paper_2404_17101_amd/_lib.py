"""ctypes declarations of libpasgal.so (mirrors include/pasgal.h)."""
from __future__ import annotations

import atexit
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpasgal.so")

PASGAL_OK = 0
ERRORS = {
    -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ECSR", -5: "ECAPACITY", -6: "EAGAIN", -7: "ETIMEOUT",
    -8: "ENOTFOUND", -9: "EINTERNAL",
}
MODE_VGC, MODE_PLAIN = 0, 1
FLAG_VALIDATE, FLAG_ASYNC, FLAG_PREFETCH, FLAG_TEST_FIRST, FLAG_HALF_DEVICE, FLAG_NO_TEST_FIRST = 1, 2, 4, 8, 32, 64
FLAG_NO_PREFETCH = 128
FLAG_NO_IMPLICATIONS = 256
SERVER_FIXED_SLICES = 65536
SERVER_NO_DIRECTION_OPT = 131072
BATCH_AUTOTUNE = 1
REQ_BFS, REQ_REACH = 0, 1

# every function include/pasgal.h declares
EXPORTS = [
    "pasgal_opts_default", "pasgal_strerror", "pasgal_last_hip_error", "pasgal_version", "pasgal_wait",
    "pasgal_shutdown",
    "pasgal_bfs", "pasgal_bfs_ex", "pasgal_bfs_noalloc", "pasgal_bfs_do", "pasgal_bfs_do_multi", "pasgal_sssp", "pasgal_reach", "pasgal_reach_ex", "pasgal_transpose", "pasgal_validate",
    "pasgal_probe_latency",
    "pasgal_scc", "pasgal_batch_create", "pasgal_batch_run", "pasgal_batch_config", "pasgal_batch_destroy",
    "pasgal_server_create", "pasgal_server_add_graph", "pasgal_server_submit", "pasgal_server_poll",
    "pasgal_server_drain", "pasgal_server_load", "pasgal_server_destroy",
]


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("offsets", ctypes.c_void_p),
                ("targets", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tau", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("frontier_capacity", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("timeout_ms", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("window", ctypes.c_int32), ("min_chunk", ctypes.c_int32), ("heavy_arcs", ctypes.c_int32),
                ("filter_slots", ctypes.c_int32), ("chunks_per_wave", ctypes.c_int32),
                ("device_share", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("expansions", ctypes.c_int64), ("arcs_scanned", ctypes.c_int64),
                ("relax_success", ctypes.c_int64), ("published", ctypes.c_int64), ("overflow", ctypes.c_int64),
                ("stale", ctypes.c_int64), ("max_frontier", ctypes.c_int64), ("device_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("steps", ctypes.c_int64), ("filtered", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


SCC_NO_SPLIT = 1


class SccOpts(ctypes.Structure):
    _fields_ = [("trim_rounds", ctypes.c_int32), ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint32),
                ("reserved", ctypes.c_int32)]


class SccStats(ctypes.Structure):
    _fields_ = [("components", ctypes.c_int64), ("trimmed", ctypes.c_int64), ("pivots", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("rounds", ctypes.c_int64), ("arcs_scanned", ctypes.c_int64),
                ("device_ms", ctypes.c_double), ("reach_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchDesc(ctypes.Structure):
    _fields_ = [("packed", Csr), ("ngraphs", ctypes.c_int32), ("vbase", ctypes.POINTER(ctypes.c_int32)),
                ("nqueries", ctypes.c_int32), ("q_graph", ctypes.POINTER(ctypes.c_int32)),
                ("q_source", ctypes.POINTER(ctypes.c_int32)), ("q_out", ctypes.POINTER(ctypes.c_int64)),
                ("dist_out", ctypes.c_void_p), ("dist_len", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_int64), ("max_slots", ctypes.c_int32), ("slice_rounds", ctypes.c_int32),
                ("tau", ctypes.c_int32), ("wg_size", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("frontier_capacity", ctypes.c_int64), ("timeout_ms", ctypes.c_int32), ("window", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("kind", ctypes.c_int32), ("nsources", ctypes.c_int32),
                ("sources", ctypes.c_int32 * 64), ("out", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("rounds", ctypes.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpasgal.so not found at {path}: build it with "
                           f"`python -m paper_2404_17101_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    c_int, i32, i64, vp = ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.pasgal_opts_default.argtypes = [P(Opts)]
    lib.pasgal_opts_default.restype = None
    lib.pasgal_strerror.argtypes = [c_int]
    lib.pasgal_strerror.restype = ctypes.c_char_p
    lib.pasgal_last_hip_error.restype = c_int
    lib.pasgal_version.restype = c_int
    lib.pasgal_wait.argtypes = [vp]
    lib.pasgal_wait.restype = c_int
    lib.pasgal_shutdown.argtypes = []
    lib.pasgal_shutdown.restype = None
    lib.pasgal_bfs.argtypes = [P(Csr), i32, vp]
    lib.pasgal_bfs_ex.argtypes = [P(Csr), i32, vp, P(Opts), P(Stats)]
    lib.pasgal_bfs_noalloc.argtypes = [P(Csr), i32, vp, P(Opts), P(Stats)]
    lib.pasgal_bfs_do.argtypes = [P(Csr), P(Csr), i32, vp, i32, i32, P(Opts), P(Stats)]
    lib.pasgal_bfs_do_multi.argtypes = [P(Csr), P(Csr), i32, P(i32), vp, vp, i32, i32, P(Opts), P(Stats)]
    lib.pasgal_sssp.argtypes = [P(Csr), vp, i32, vp, P(Opts), P(Stats)]
    lib.pasgal_reach.argtypes = [P(Csr), P(i32), i32, vp]
    lib.pasgal_reach_ex.argtypes = [P(Csr), P(i32), i32, vp, P(Opts), P(Stats)]
    lib.pasgal_transpose.argtypes = [P(Csr), vp, vp, P(Opts)]
    lib.pasgal_validate.argtypes = [P(Csr), P(Opts)]
    lib.pasgal_probe_latency.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double), P(Opts)]
    lib.pasgal_scc.argtypes = [P(Csr), P(Csr), vp, P(SccOpts), P(Opts), P(SccStats)]
    lib.pasgal_batch_create.argtypes = [P(BatchDesc), P(Opts), ctypes.c_uint32, P(vp)]
    lib.pasgal_batch_run.argtypes = [vp, P(Stats)]
    lib.pasgal_batch_config.argtypes = [vp, P(Opts)]
    lib.pasgal_batch_destroy.argtypes = [vp]
    lib.pasgal_batch_destroy.restype = None
    lib.pasgal_server_create.argtypes = [P(ServerOpts), P(vp)]
    lib.pasgal_server_add_graph.argtypes = [vp, P(Csr), P(i32)]
    lib.pasgal_server_submit.argtypes = [vp, P(Request), P(i64)]
    lib.pasgal_server_poll.argtypes = [vp, P(Completion), i32, P(i32)]
    lib.pasgal_server_drain.argtypes = [vp, i32]
    lib.pasgal_server_load.argtypes = [vp, P(i32), P(i32), P(i64)]
    lib.pasgal_server_destroy.argtypes = [vp]
    lib.pasgal_server_destroy.restype = None
    for f in ("pasgal_bfs", "pasgal_bfs_ex", "pasgal_bfs_noalloc", "pasgal_bfs_do", "pasgal_bfs_do_multi", "pasgal_sssp", "pasgal_reach", "pasgal_reach_ex", "pasgal_transpose",
              "pasgal_validate", "pasgal_probe_latency", "pasgal_scc", "pasgal_batch_create", "pasgal_batch_run",
              "pasgal_batch_config",
              "pasgal_server_create", "pasgal_server_add_graph", "pasgal_server_submit", "pasgal_server_poll",
              "pasgal_server_drain", "pasgal_server_load"):
        getattr(lib, f).restype = c_int
    _lib = lib
    # release the library's workspaces before the HIP runtime tears down
    atexit.register(lib.pasgal_shutdown)
    return lib
