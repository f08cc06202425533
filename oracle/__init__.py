"""CPU oracle for direction-optimized BFS as Boolean matvec.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the GPU library and its Python
binding never import, link or call it, and share no code with it.

What it computes (each function cites the passage it follows):

* :func:`bfs` -- textbook FIFO-queue BFS (Section 2.1), C in ``oracle.c``.
* :func:`validate` -- Graph500-style checks of a (depth, parent) pair.
* :func:`mxv` -- y = (A^T x) .* m over ({0,1}, OR, AND, 0) with structural
  complement and OR-accumulate (Equations 4-5, Section 3.2).
* :func:`first_parent` -- the parent a first-hit pull reports (Section 5.3).
* :func:`schedule` -- the push/pull direction sequence of the Section 6.3 rule.
* :func:`schedule_edges` -- the same under Beamer's edge-count rule (Section 6.3).
* :func:`level_work` -- per-level frontier sizes and the work of Table 1.

Parity unpinned: parents chosen on push levels (any in-neighbour one level up
is correct, so only validity is checked).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PUSH, PULL = 0, 1


def build(force: bool = False) -> str:
    """Compile oracle.c (plain C, gcc -O2, single thread) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.oracle_bfs.restype = ctypes.c_int
        lib.oracle_bfs.argtypes = [i32, vp, vp, i32, vp, vp]
        lib.oracle_validate.restype = ctypes.c_int
        lib.oracle_validate.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, ctypes.POINTER(i64)]
        lib.oracle_mxv.restype = None
        lib.oracle_mxv.argtypes = [i32, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
        lib.oracle_first_parent.restype = None
        lib.oracle_first_parent.argtypes = [i32, vp, vp, vp, i32, vp]
        lib.oracle_pull_checks.restype = i64
        lib.oracle_pull_checks.argtypes = [i32, vp, vp, vp, i32]
        _lib = lib
    return _lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a) != 0, dtype=np.uint8)


def bfs(g, source: int):
    """(depth, parent) of a FIFO-queue BFS over CSR(A) (Section 2.1)."""
    depth = np.empty(g.V, dtype=np.int32)
    parent = np.empty(g.V, dtype=np.int32)
    rp, ci = _i32(g.rowptr), _i32(g.colind)
    rc = _load().oracle_bfs(g.V, rp.ctypes.data, ci.ctypes.data, int(source),
                            depth.ctypes.data, parent.ctypes.data)
    if rc == -1:
        raise ValueError("source %d out of range [0, %d)" % (source, g.V))
    if rc != 0:
        raise MemoryError("oracle_bfs")
    return depth, parent


VALIDATE_MESSAGES = {
    1: "source must have depth 0 and be its own parent",
    2: "only the source may have depth 0; depths must be >= -1",
    3: "depth -1 must coincide with parent -1",
    4: "parent must be an in-neighbour exactly one level closer",
    5: "an edge from a reached vertex leads to an unreached or too-deep vertex",
}


def validate(g, source: int, depth, parent):
    """(code, vertex): code 0 when (depth, parent) is a valid BFS result, else the failed check."""
    depth, parent = _i32(depth), _i32(parent)
    bad = ctypes.c_int64(-1)
    arrs = [_i32(x) for x in (g.rowptr, g.colind, g.csc_colptr, g.csc_rowind)]
    code = _load().oracle_validate(g.V, *[a.ctypes.data for a in arrs], int(source),
                                   depth.ctypes.data, parent.ctypes.data, ctypes.byref(bad))
    return code, bad.value


def mxv(g, x, mask=None, complement: bool = False, accum: bool = False, y_old=None) -> np.ndarray:
    """y = (A^T x) .* m over the Boolean semiring (Equations 4-5), one byte per vertex."""
    x = _u8(x)
    y = _u8(y_old) if (accum and y_old is not None) else np.zeros(g.V, dtype=np.uint8)
    m = _u8(mask) if mask is not None else None
    rp, ci = _i32(g.rowptr), _i32(g.colind)
    _load().oracle_mxv(g.V, rp.ctypes.data, ci.ctypes.data, x.ctypes.data,
                       m.ctypes.data if m is not None else None, int(bool(complement)),
                       int(bool(accum)), y.ctypes.data)
    return y


def first_parent(g, depth, source: int) -> np.ndarray:
    """First in-neighbour (stored CSC order) one level closer: the parent a first-hit pull reports."""
    depth = _i32(depth)
    out = np.empty(g.V, dtype=np.int32)
    cp, ri = _i32(g.csc_colptr), _i32(g.csc_rowind)
    _load().oracle_first_parent(g.V, cp.ctypes.data, ri.ctypes.data, depth.ctypes.data,
                                int(source), out.ctypes.data)
    return out


def pull_checks(g, depth, level: int) -> int:
    """In-neighbour checks of a level-`level` pull with mask, early exit and the visited set as input."""
    depth = _i32(depth)
    cp, ri = _i32(g.csc_colptr), _i32(g.csc_rowind)
    return int(_load().oracle_pull_checks(g.V, cp.ctypes.data, ri.ctypes.data, depth.ctypes.data,
                                          int(level)))


def level_sizes(depth) -> list:
    """nnz(f) entering each level: level L expands the vertices of depth L. The last level
    (the one that discovers nothing) has the deepest layer as its frontier."""
    depth = np.asarray(depth)
    reached = depth[depth >= 0]
    if reached.size == 0:
        return []
    return np.bincount(reached).astype(np.int64).tolist()


def schedule(sizes, V: int, alpha: float = 0.01, beta: float = 0.01, start: int = PUSH) -> list:
    """Direction used at each level under the rule of Section 6.3.

    r = nnz(f)/M. After a level that turned a frontier of size nf into one of
    size nn: push -> pull when r increased (nn > nf) and nn > alpha*M;
    pull -> push when r decreased (nn < nf) and nn < beta*M. The traversal
    starts in push. `sizes` are the frontier sizes entering each level; the
    level after the last one discovers nothing.
    """
    alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    dirs = []
    d = start
    n = len(sizes)
    for L in range(n):
        dirs.append(d)
        nf = sizes[L]
        nn = sizes[L + 1] if L + 1 < n else 0
        if d == PUSH and nn > nf and nn > alpha * V:
            d = PULL
        elif d == PULL and nn < nf and nn < beta * V:
            d = PUSH
    return dirs


def schedule_edges(g, depth, alpha: float = 1 / 14, beta: float = 1 / 24, start: int = PUSH) -> list:
    """Direction used at each level under Beamer's edge-count rule as Section 6.3 states it.

    After level L (which found the vertices of depth L+1): in push, switch to pull when
    nnz(m_f) > alpha * nnz(m_u), where m_f is the out-edges of the new frontier (depth L+1)
    and m_u the in-edges of the vertices still unvisited (no depth yet, or depth > L+1); in
    pull, switch back when nnz(f)/M < beta, f being the new frontier (M = number of rows).
    alpha and beta are taken as float32 (the options store them so) and compared in double.
    """
    alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    depth = np.asarray(depth)
    sizes = level_sizes(depth)
    outdeg = g.out_degree().astype(np.int64)
    indeg = g.in_degree().astype(np.int64)
    V = int(depth.size)
    dirs = []
    d = start
    for L in range(len(sizes)):
        dirs.append(d)
        new = depth == L + 1
        nn = int(new.sum())
        m_f = int(outdeg[new].sum())
        m_u = int(indeg[(depth < 0) | (depth > L + 1)].sum())
        if d == PUSH:
            d = PULL if float(m_f) > alpha * float(m_u) else PUSH
        else:
            d = PUSH if float(nn) < beta * float(V) else PULL
    return dirs


def level_work(g, depth, dirs):
    """Per-level reference statistics for a BFS run with direction sequence `dirs`
    (full method: mask, early exit, visited set as pull input).

    For each level L: frontier size nf, discovered n_new, and the edges touched:
    push -- nnz(m_f^+) = sum of out-degrees over the frontier (Table 1, column-based);
    pull -- in-neighbour checks with early exit (:func:`pull_checks`)."""
    depth = np.asarray(depth)
    sizes = level_sizes(depth)
    outdeg = g.out_degree()
    rows = []
    for L, d in enumerate(dirs):
        nf = sizes[L]
        nn = sizes[L + 1] if L + 1 < len(sizes) else 0
        if d == PUSH:
            work = int(outdeg[depth == L].sum())
        else:
            work = pull_checks(g, depth, L)
        rows.append(dict(level=L, dir=d, nf=nf, n_new=nn, edges=work))
    return rows


def table1_counts(g, x=None, mask=None, complement: bool = False) -> dict:
    """Memory accesses into A of the four matvec variants (Table 1), counted exactly:
    row-based unmasked touches every nonzero; row-based masked the in-edges of rows that
    pass the mask (no early exit); column-based the out-edges of nonzeros of x."""
    indeg, outdeg = g.in_degree(), g.out_degree()
    out = {"row": int(g.nnz)}
    if mask is not None:
        passing = (np.asarray(mask) != 0) ^ bool(complement)
        out["row_masked"] = int(indeg[passing].sum())
    if x is not None:
        out["col"] = int(outdeg[np.asarray(x) != 0].sum())
    return out


def teps_edges(g, depth) -> dict:
    """Edge counts for TEPS: 'graph500' = undirected edges with a reached endpoint
    (sum of reached out-degrees / 2 on a symmetric graph); 'paper' = nnz(A), the whole
    symmetrized graph, which matches the figures printed in Section 7."""
    depth = np.asarray(depth)
    reached = int(g.out_degree()[depth >= 0].sum())
    return {"graph500": reached // 2 if g.symmetric else reached, "paper": int(g.nnz)}
