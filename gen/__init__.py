"""Seeded synthetic graph inputs (shared by tests, benchmark and oracle checks).

This package makes inputs only; it contains none of the BFS / matvec
arithmetic. Large graphs come from ``gen.cpp`` (OpenMP, counter-based
SplitMix64 so results do not depend on the thread count); small hand-made
graphs are built here with numpy.

Every graph is returned as a :class:`HostGraph`: int32 CSR of A (row u lists
the out-neighbours v of u, edge u->v) and int32 CSC of A (column v lists the
in-neighbours u of v). Rows are sorted and duplicate-free. For undirected
graphs the two are the same arrays.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import json
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB = os.path.join(_HERE, "libgen.so")

# R-MAT quadrant probabilities used by the paper's generated graphs' family
# (Graph500 values; d = 1 - a - b - c = 0.05).
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def build(force: bool = False) -> str:
    """Compile gen.cpp into libgen.so (g++ -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.gen_rmat.restype = vp
        lib.gen_rmat.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, u64, ctypes.c_int]
        lib.gen_lattice3d.restype = vp
        lib.gen_lattice3d.argtypes = [i32, dbl, u64]
        lib.gen_grid2d.restype = vp
        lib.gen_grid2d.argtypes = [i32, i32]
        lib.gen_graph_nv.restype = i32
        lib.gen_graph_nv.argtypes = [vp]
        lib.gen_graph_nnz.restype = i64
        lib.gen_graph_nnz.argtypes = [vp]
        lib.gen_graph_copy.restype = ctypes.c_int
        lib.gen_graph_copy.argtypes = [vp, vp, vp]
        lib.gen_graph_free.restype = None
        lib.gen_graph_free.argtypes = [vp]
        lib.gen_rmat_edges.restype = None
        lib.gen_rmat_edges.argtypes = [ctypes.c_int, dbl, dbl, dbl, u64, i64, i64, vp, vp]
        lib.gen_sample.restype = i64
        lib.gen_sample.argtypes = [vp, i64, i64, u64, vp]
        lib.gen_transpose.restype = None
        lib.gen_transpose.argtypes = [i32, i64, vp, vp, vp, vp]
        lib.gen_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclasses.dataclass
class HostGraph:
    """Host-side CSR(A) + CSC(A), int32, rows sorted and duplicate-free."""

    name: str
    V: int
    rowptr: np.ndarray  # CSR(A): out-neighbours
    colind: np.ndarray
    csc_colptr: np.ndarray  # CSC(A): in-neighbours
    csc_rowind: np.ndarray
    symmetric: bool
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colind.size)

    def out_degree(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def in_degree(self) -> np.ndarray:
        return np.diff(self.csc_colptr.astype(np.int64))


def _from_handle(h, name: str, meta: dict) -> HostGraph:
    lib = _load()
    if not h:
        raise ValueError("generator rejected its parameters: %s %r" % (name, meta))
    try:
        V = lib.gen_graph_nv(h)
        nnz = lib.gen_graph_nnz(h)
        rowptr = np.empty(V + 1, dtype=np.int32)
        colind = np.empty(nnz, dtype=np.int32)
        if lib.gen_graph_copy(h, _ptr(rowptr), _ptr(colind)) != 0:
            raise ValueError("graph %s has more than 2^31-1 edges" % name)
    finally:
        lib.gen_graph_free(h)
    return HostGraph(name, V, rowptr, colind, rowptr, colind, True, meta)


def _cached(key: dict, make):
    """Optional on-disk cache (directory in $DOBFS_GRAPH_CACHE), npz without pickle."""
    cache = os.environ.get("DOBFS_GRAPH_CACHE")
    if not cache:
        return make()
    tag = hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:16]
    path = os.path.join(cache, "%s_%s.npz" % (key["kind"], tag))
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
            rp, ci = z["rowptr"], z["colind"]
            return HostGraph(meta["name"], int(rp.size - 1), rp, ci, rp, ci, True, meta["meta"])
    g = make()
    os.makedirs(cache, exist_ok=True)
    tmp = path + ".tmp%d.npz" % os.getpid()
    np.savez(tmp, rowptr=g.rowptr, colind=g.colind,
             meta=np.array(json.dumps({"name": g.name, "meta": g.meta})))
    os.replace(tmp, path)
    return g


def rmat(scale: int, edgefactor: int = 16, a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C,
         seed: int = 1, relabel: bool = True) -> HostGraph:
    """Undirected simple R-MAT graph: 2^scale vertices, edgefactor*2^scale generated edges,
    self-loops and duplicates removed, vertex ids relabelled by a seeded permutation."""
    key = dict(kind="rmat", scale=scale, ef=edgefactor, a=a, b=b, c=c, seed=seed, relabel=bool(relabel))

    def make():
        t0 = time.time()
        h = _load().gen_rmat(scale, edgefactor, a, b, c, seed, int(bool(relabel)))
        meta = dict(key, gen_seconds=None)
        g = _from_handle(h, "rmat%d_ef%d" % (scale, edgefactor), meta)
        g.meta["gen_seconds"] = round(time.time() - t0, 3)
        return g

    return _cached(key, make)


def lattice3d(n: int, del_frac: float = 0.05, seed: int = 3) -> HostGraph:
    """n^3 7-point lattice with floor(del_frac * 3 n^2 (n-1)) undirected edges deleted."""
    key = dict(kind="lattice3d", n=n, del_frac=del_frac, seed=seed)
    return _cached(key, lambda: _from_handle(_load().gen_lattice3d(n, del_frac, seed),
                                             "lattice%d" % n, key))


def grid2d(nx: int, ny: int) -> HostGraph:
    """nx x ny 4-connected grid."""
    key = dict(kind="grid2d", nx=nx, ny=ny)
    return _cached(key, lambda: _from_handle(_load().gen_grid2d(nx, ny), "grid%dx%d" % (nx, ny), key))


def rmat_raw_edges(scale: int, count: int, seed: int = 1, start: int = 0,
                   a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C):
    """The generator's raw directed R-MAT pairs (before permutation and cleaning)."""
    src = np.empty(count, dtype=np.int32)
    dst = np.empty(count, dtype=np.int32)
    _load().gen_rmat_edges(scale, a, b, c, seed, start, count, _ptr(src), _ptr(dst))
    return src, dst


def transpose(V: int, rowptr: np.ndarray, colind: np.ndarray):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    trp = np.empty(V + 1, dtype=np.int32)
    tci = np.empty(colind.size, dtype=np.int32)
    _load().gen_transpose(V, colind.size, _ptr(rowptr), _ptr(colind), _ptr(trp), _ptr(tci))
    return trp, tci


def from_edges(V: int, src, dst, directed: bool = False, keep_self_loops: bool = False,
               keep_duplicates: bool = False, name: str = "edges") -> HostGraph:
    """Small graphs from an explicit edge list (numpy). Undirected graphs get both directions."""
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= V or dst.max() >= V):
        raise ValueError("edge endpoint out of range")
    if not directed:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    if not keep_self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    key = src * V + dst
    if keep_duplicates:
        order = np.argsort(key, kind="stable")
        key = key[order]
    else:
        key = np.unique(key)
    s, d = key // V, key % V
    rowptr = np.zeros(V + 1, dtype=np.int64)
    np.add.at(rowptr, s + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    colind = d.astype(np.int32)
    if directed:
        cp, ri = transpose(V, rowptr, colind)
        return HostGraph(name, V, rowptr, colind, cp, ri, False, {"kind": "edges"})
    return HostGraph(name, V, rowptr, colind, rowptr, colind, True, {"kind": "edges"})


def sample_sources(g: HostGraph, k: int, seed: int) -> np.ndarray:
    """k distinct sources drawn uniformly among vertices with out-degree > 0."""
    cand = np.nonzero(g.out_degree() > 0)[0].astype(np.int32)
    out = np.empty(min(k, cand.size), dtype=np.int32)
    n = _load().gen_sample(_ptr(cand), cand.size, k, seed, _ptr(out))
    return out[:n]


def max_degree_vertex(g: HostGraph) -> int:
    """Vertex of largest out-degree; ties go to the smallest id."""
    return int(np.argmax(g.out_degree()))


def num_threads() -> int:
    return int(_load().gen_num_threads())


# Workloads of the method's evaluation, as synthetic stand-ins (sizes are the
# ones the benchmark and full-size tests use).
def workload(name: str) -> HostGraph:
    if name == "rmat10":
        return rmat(10, 16, seed=1)
    if name == "rmat22":
        return rmat(22, 16, seed=1)
    if name == "rmat20":
        return rmat(20, 16, seed=1)
    if name == "lattice256":
        return lattice3d(256, 0.05, seed=3)
    raise KeyError(name)
