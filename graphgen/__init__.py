"""Seeded synthetic graph generators (int32 CSR), shared input tooling.

This module only draws inputs: grids, tori, chains, cycles, k-NN graphs of
uniform 2D points, road-like grids, RMAT graphs and random digraphs, plus the
packer that lays many graphs out as one CSR. It computes nothing the traversal
computes (no distances, reachability or transposition), so both the CPU oracle
tests and the GPU path can consume its output without sharing any method code.

Graph sizes follow the paper's notation (Preliminaries): n vertices, m arcs;
undirected graphs are stored symmetrised, so an undirected edge counts as two
arcs, as the paper's m does for symmetrised graphs (Table of tested graphs).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")


def build(force: bool = True) -> str:
    """Compile graphgen.c into libgraphgen.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _GG(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("offsets", ctypes.POINTER(ctypes.c_int32)),
        ("targets", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_GG)
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        lib.gg_grid.argtypes = [i64, i64, ctypes.c_int, P]
        lib.gg_simple.argtypes = [i32, i64, P]
        lib.gg_random.argtypes = [i64, i64, ctypes.c_int, u64, P]
        lib.gg_knn.argtypes = [i64, i32, u64, ctypes.c_int, P]
        lib.gg_road.argtypes = [i64, dbl, dbl, dbl, u64, P]
        lib.gg_rmat.argtypes = [i32, i32, dbl, dbl, dbl, u64, P]
        lib.gg_points_ordered.argtypes = [i64, u64, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]
        lib.gg_points_ordered.restype = None
        lib.gg_weights.argtypes = [i64, u64, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        lib.gg_weights.restype = None
        lib.gg_free.argtypes = [P]
        lib.gg_free.restype = None
        lib.gg_rng64.argtypes = [u64, u64, u64]
        lib.gg_rng64.restype = u64
        for f in ("gg_grid", "gg_simple", "gg_random", "gg_knn", "gg_road", "gg_rmat"):
            getattr(lib, f).restype = ctypes.c_int
        lib.gg_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Graph:
    """int32 CSR: offsets[n+1], targets[m]; rows sorted, no self-loops/duplicates."""

    offsets: np.ndarray
    targets: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.targets.shape[0])


def _take(fn, *args, name="", **meta) -> Graph:
    lib = _load()
    g = _GG()
    rc = getattr(lib, fn)(*args, ctypes.byref(g))
    if rc != 0:
        raise RuntimeError(f"{fn}{args} failed with code {rc}")
    try:
        n, m = int(g.n), int(g.m)
        off = np.ctypeslib.as_array(g.offsets, shape=(n + 1,)).copy()
        tgt = np.ctypeslib.as_array(g.targets, shape=(max(m, 1),))[:m].copy()
    finally:
        lib.gg_free(ctypes.byref(g))
    return Graph(off, tgt, name=name, meta=dict(meta))


def weights(g: Graph, seed: int, lo: int = 1, hi: int = 1000) -> np.ndarray:
    """uint32 weight per arc of g (parallel to g.targets), uniform integers in
    [lo, hi] from counter-based stream 70 of `seed`."""
    if not (0 <= lo <= hi < 2**32):
        raise ValueError("weights need 0 <= lo <= hi < 2^32")
    w = np.empty(max(g.m, 1), dtype=np.uint32)
    _load().gg_weights(g.m, seed, lo, hi, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return w[:g.m]


def grid(a: int, b: int, torus: bool = False) -> Graph:
    """a x b 4-neighbour undirected grid (torus if requested); id = r*b + c."""
    return _take("gg_grid", a, b, 1 if torus else 0, name=f"{'torus' if torus else 'grid'}{a}x{b}", a=a, b=b)


SIMPLE = {"dchain": 0, "uchain": 1, "dcycle": 2, "ucycle": 3, "complete": 4, "star": 5, "empty": 6}


def simple(kind: str, n: int) -> Graph:
    """Closed-form families: dchain, uchain, dcycle, ucycle, complete, star, empty."""
    return _take("gg_simple", SIMPLE[kind], n, name=f"{kind}{n}")


def random_graph(n: int, m0: int, seed: int, symmetric: bool = False) -> Graph:
    """m0 uniform arcs (self-loops and repeats then removed)."""
    return _take("gg_random", n, m0, 1 if symmetric else 0, seed, name=f"rand{n}_{m0}_{seed}")


LAYOUTS = {"draw": 0, "morton": 1}


def knn(n: int, k: int, seed: int, layout: str = "morton") -> Graph:
    """Directed k-NN graph of n uniform points in [0,1)^2 (24-bit coordinates).

    layout 'draw' numbers vertices in draw order (ids carry no locality);
    'morton' renumbers the drawn points along the Z-order curve.
    """
    return _take("gg_knn", n, k, seed, LAYOUTS[layout], name=f"knn{n}_k{k}_s{seed}_{layout}", layout=layout)


def points(n: int, seed: int, layout: str = "morton") -> np.ndarray:
    """The (n, 2) int32 integer coordinates (units of 2^-24) knn() uses."""
    lib = _load()
    xy = np.empty(2 * n, dtype=np.int32)
    lib.gg_points_ordered(n, seed, LAYOUTS[layout], xy.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return xy.reshape(n, 2)


def road(side: int, seed: int, p_del: float = 0.3, p_both: float = 0.6, p_diag: float = 0.005) -> Graph:
    """side x side road-like directed grid (deletions, one-way edges, diagonal shortcuts)."""
    return _take("gg_road", side, p_del, p_both, p_diag, seed, name=f"road{side}_s{seed}")


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19, c: float = 0.19) -> Graph:
    """Symmetrised, deduplicated, relabelled RMAT graph with 2^scale vertices."""
    return _take("gg_rmat", scale, edge_factor, a, b, c, seed, name=f"rmat{scale}_ef{edge_factor}_s{seed}")


def rng64(seed: int, stream: int, i: int) -> int:
    """The generators' counter-based 64-bit draw (SplitMix64 finaliser)."""
    return int(_load().gg_rng64(seed, stream, i))


def u01(seed: int, stream: int, i: int) -> float:
    return (rng64(seed, stream, i) >> 11) * (1.0 / 9007199254740992.0)


def sources(g: Graph, count: int, seed: int, min_degree: int = 0) -> np.ndarray:
    """count distinct vertices drawn with the counter-based stream 50; when
    min_degree > 0 only vertices with out-degree >= min_degree qualify."""
    deg = np.diff(g.offsets)
    out = []
    seen = set()
    i = 0
    limit = 1000 * count + 10 * g.n
    while len(out) < count and i < limit:
        v = rng64(seed, 50, i) % g.n
        i += 1
        if v in seen or deg[v] < min_degree:
            continue
        seen.add(v)
        out.append(v)
    if len(out) < count:
        raise ValueError("not enough qualifying vertices")
    return np.asarray(out, dtype=np.int32)


@dataclass
class Packed:
    """Many graphs laid out as one CSR over the disjoint union of their vertex
    sets: graph g owns global vertices [vbase[g], vbase[g+1]) and arcs
    [ebase[g], ebase[g+1]); targets hold global vertex ids."""

    offsets: np.ndarray
    targets: np.ndarray
    vbase: np.ndarray
    ebase: np.ndarray
    names: list

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.targets.shape[0])

    @property
    def ngraphs(self) -> int:
        return int(self.vbase.shape[0] - 1)

    def graph(self, g: int) -> Graph:
        v0, v1 = int(self.vbase[g]), int(self.vbase[g + 1])
        e0, e1 = int(self.ebase[g]), int(self.ebase[g + 1])
        return Graph((self.offsets[v0 : v1 + 1] - e0).astype(np.int32), (self.targets[e0:e1] - v0).astype(np.int32),
                     name=self.names[g])


def pack(graphs: list) -> Packed:
    ns = np.array([g.n for g in graphs], dtype=np.int64)
    ms = np.array([g.m for g in graphs], dtype=np.int64)
    vbase = np.zeros(len(graphs) + 1, dtype=np.int64)
    ebase = np.zeros(len(graphs) + 1, dtype=np.int64)
    vbase[1:] = np.cumsum(ns)
    ebase[1:] = np.cumsum(ms)
    if vbase[-1] >= 2**31 or ebase[-1] >= 2**31:
        raise ValueError("packed graph exceeds int32 ids")
    off = np.empty(int(vbase[-1]) + 1, dtype=np.int32)
    tgt = np.empty(int(ebase[-1]), dtype=np.int32)
    for i, g in enumerate(graphs):
        v0, e0 = int(vbase[i]), int(ebase[i])
        off[v0 : v0 + g.n] = g.offsets[:-1] + e0
        tgt[e0 : e0 + g.m] = g.targets + v0
    off[-1] = int(ebase[-1])
    return Packed(off, tgt, vbase.astype(np.int32), ebase.astype(np.int32), [g.name for g in graphs])


def batch_recipe(ngrids: int = 128, nknn: int = 128, seed: int = 4, grid_lo: int = 64, grid_hi: int = 2048,
                 knn_lo: int = 10_000, knn_hi: int = 1_000_000, k: int = 5) -> list:
    """Uneven-size graph mix: grids with side round(lo * (hi/lo)^U) and k-NN
    graphs with n = round(lo * (hi/lo)^U), U uniform in [0,1) (stream 60 for
    grids, 61 for k-NN); the k-NN graph j uses seed*1000003 + j."""
    out = []
    for j in range(ngrids):
        u = u01(seed, 60, j)
        side = int(round(grid_lo * (grid_hi / grid_lo) ** u))
        out.append(("grid", side))
    for j in range(nknn):
        u = u01(seed, 61, j)
        n = int(round(knn_lo * (knn_hi / knn_lo) ** u))
        out.append(("knn", n, seed * 1000003 + j))
    return out


def batch_graphs(recipe: list, layout: str = "morton") -> list:
    gs = []
    for item in recipe:
        if item[0] == "grid":
            gs.append(grid(item[1], item[1]))
        else:
            gs.append(knn(item[1], 5, item[2], layout=layout))
    return gs


def threads() -> int:
    return int(_load().gg_num_threads())
