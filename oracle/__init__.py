"""CPU oracle for the traversal results -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package. The GPU library (paper_2404_17101_amd) never imports it, and it
never imports the GPU library: the two share no code. Inputs come from the
seeded generators in ``graphgen``, which hold none of the traversal arithmetic.

What each function computes (plain definitions; see oracle.c):
  bfs(g, src)          hop distance from src along out-arcs, -1 if unreachable;
                       the sequential FIFO-queue BFS the paper uses as its BFS
                       baseline (Experimental Results; BFS time table).
  reach(g, sources)    uint64 masks [n, ceil(k/64)]: bit i set iff sources[i]
                       reaches v (reachability search, Parallel SCC section);
                       iterative DFS per source.
  scc(g)               Tarjan's SCC labels (the paper's SCC baseline).
  scc_min_label(g)     the same components, each named by its smallest
                       vertex (a unique labelling, the form the GPU SCC
                       call returns).
  transpose(g)         G^T with rows sorted ascending (stable counting sort).
  sssp(g, w, src)      shortest-path distances with non-negative integer arc
                       weights w (parallel to g.targets), int64, -1 if
                       unreachable; Dijkstra with a binary heap (Parallel
                       SSSP paragraph).

Parity status of each function is recorded in tests/test_oracle.py: every one
is pinned against closed forms, brute force or an independent certificate.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c (plain C, single-threaded) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_I32P = ctypes.POINTER(ctypes.c_int32)
_U64P = ctypes.POINTER(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_bfs.argtypes = [ctypes.c_int32, _I32P, _I32P, ctypes.c_int32, _I32P]
        lib.oracle_reach.argtypes = [ctypes.c_int32, _I32P, _I32P, ctypes.c_int32, _I32P, ctypes.c_int32, _U64P]
        lib.oracle_scc.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P]
        lib.oracle_transpose.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P, _I32P]
        lib.oracle_sssp.argtypes = [ctypes.c_int32, _I32P, _I32P, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int64)]
        for f in ("oracle_bfs", "oracle_reach", "oracle_scc", "oracle_transpose", "oracle_sssp"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _csr(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int32)
    tgt = np.ascontiguousarray(g.targets, dtype=np.int32)
    if tgt.size == 0:
        tgt = np.zeros(1, dtype=np.int32)
    return off, tgt


def _p(a, t=_I32P):
    return a.ctypes.data_as(t)


def bfs(g, src: int) -> np.ndarray:
    off, tgt = _csr(g)
    n = off.size - 1
    dist = np.empty(n, dtype=np.int32)
    rc = _load().oracle_bfs(n, _p(off), _p(tgt), int(src), _p(dist))
    if rc != 0:
        raise ValueError(f"oracle_bfs failed ({rc})")
    return dist


def reach(g, sources) -> np.ndarray:
    off, tgt = _csr(g)
    n = off.size - 1
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.size)
    words = (k + 63) // 64
    mask = np.empty((n, words), dtype=np.uint64)
    rc = _load().oracle_reach(n, _p(off), _p(tgt), k, _p(src), words, _p(mask, _U64P))
    if rc != 0:
        raise ValueError(f"oracle_reach failed ({rc})")
    return mask


def scc(g) -> np.ndarray:
    off, tgt = _csr(g)
    n = off.size - 1
    comp = np.empty(n, dtype=np.int32)
    rc = _load().oracle_scc(n, _p(off), _p(tgt), _p(comp))
    if rc < 0:
        raise ValueError(f"oracle_scc failed ({rc})")
    return comp


def sssp(g, weights, src: int) -> np.ndarray:
    off, tgt = _csr(g)
    n = off.size - 1
    w = np.ascontiguousarray(weights, dtype=np.uint32)
    if w.size != int(off[-1]):
        raise ValueError("one weight per arc")
    if w.size == 0:
        w = np.zeros(1, dtype=np.uint32)
    dist = np.empty(n, dtype=np.int64)
    rc = _load().oracle_sssp(n, _p(off), _p(tgt), w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), int(src),
                             dist.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle_sssp failed ({rc})")
    return dist


def scc_min_label(g) -> np.ndarray:
    """Strongly connected components (Parallel SCC section) with each vertex
    labelled by the smallest vertex of its component: Tarjan's component
    numbers, then the minimum vertex id per component."""
    comp = scc(g)
    n = comp.size
    _, idx = np.unique(comp, return_inverse=True)
    smallest = np.full(idx.max() + 1 if n else 0, n, dtype=np.int64)
    np.minimum.at(smallest, idx, np.arange(n, dtype=np.int64))
    return smallest[idx].astype(np.int32)


def transpose(g):
    """Returns (t_offsets, t_targets) of G^T, rows ascending."""
    off, tgt = _csr(g)
    n = off.size - 1
    m = int(off[-1])
    t_off = np.empty(n + 1, dtype=np.int32)
    t_tgt = np.empty(max(m, 1), dtype=np.int32)
    rc = _load().oracle_transpose(n, _p(off), _p(tgt), _p(t_off), _p(t_tgt))
    if rc != 0:
        raise ValueError(f"oracle_transpose failed ({rc})")
    return t_off, t_tgt[:m].copy()
