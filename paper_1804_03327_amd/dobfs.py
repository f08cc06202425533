"""Python binding of libdobfs (include/dobfs.h): same names as the C entry points, argument
marshalling only. Every step of BFS and mxv runs in the library's HIP kernels; torch
provides device memory and streams. There is no fallback: if the library is missing or the
GPU is unavailable, calls raise."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdobfs.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "dobfs.h")

# status codes
OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_WORKSPACE_TOO_SMALL, ERR_UNSUPPORTED, \
    ERR_INTERNAL, ERR_TIMEOUT = range(8)
UPLOAD_VALIDATE = 1
UPLOAD_HUBS_FIRST = 2
DIR_PUSH, DIR_PULL = 0, 1
MODE_FULL, MODE_PUSH_ONLY, MODE_PULL_UNMASKED, MODE_PULL_MASKED, MODE_PULL_MASKED_EE, \
    MODE_PULL_ONLY, MODE_PUSH_SORT, MODE_PUSH_SORT_KEYS = range(8)
MODES = {"full": MODE_FULL, "push_only": MODE_PUSH_ONLY, "pull_unmasked": MODE_PULL_UNMASKED,
         "pull_masked": MODE_PULL_MASKED, "pull_masked_ee": MODE_PULL_MASKED_EE,
         "pull_only": MODE_PULL_ONLY, "push_sort": MODE_PUSH_SORT, "push_sort_keys": MODE_PUSH_SORT_KEYS}
HEUR_RATIO, HEUR_EDGES = 0, 1
OPT_TIME_KERNELS = 1
OPT_PERSISTENT = 2
MXV_EARLY_EXIT, MXV_ACCUM_OR = 1, 2


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("heuristic", ctypes.c_int32),
                ("alpha", ctypes.c_float), ("beta", ctypes.c_float),
                ("forced_dirs", ctypes.c_void_p), ("n_forced", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("pull_mid", ctypes.c_int32), ("bitmap_rows", ctypes.c_int32),
                ("local_unit", ctypes.c_int32), ("local_chunks", ctypes.c_int32)]


class LevelStats(ctypes.Structure):
    _fields_ = [("dir", ctypes.c_int32), ("nf", ctypes.c_int32), ("n_new", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("edges", ctypes.c_int64), ("m_f", ctypes.c_int64),
                ("ms_main", ctypes.c_float), ("ms_aux", ctypes.c_float)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("cap", ctypes.c_int32),
                ("level", ctypes.POINTER(LevelStats)), ("ms_total", ctypes.c_float),
                ("ms_init", ctypes.c_float), ("reached", ctypes.c_int64),
                ("launches_main", ctypes.c_int32), ("launches_aux", ctypes.c_int32),
                ("ms_main_all", ctypes.c_float), ("ms_aux_all", ctypes.c_float),
                ("edges_g500", ctypes.c_int64)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("mem_budget", ctypes.c_size_t), ("opt", Options)]


class QueryInfo(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("source", ctypes.c_int32),
                ("batch_size", ctypes.c_int32), ("status", ctypes.c_int32),
                ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double)]


class DobfsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_status_name(status), message))
        self.status = status


_lib = None


def _status_name(s: int) -> str:
    try:
        return load().dobfs_status_string(s).decode()
    except Exception:  # library not loadable: still report the number
        return "status %d" % s


def load():
    """Load libdobfs.so from the package directory (built by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdobfs.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sz = ctypes.c_size_t
    sigs = {
        "dobfs_graph_upload": (i32, [i32, i64, vp, vp, vp, vp, i32, u32, ctypes.POINTER(vp)]),
        "dobfs_graph_wrap_device": (i32, [i32, i64, vp, vp, vp, vp, i32, u32, vp, ctypes.POINTER(vp)]),
        "dobfs_graph_destroy": (i32, [vp]),
        "dobfs_graph_info": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "dobfs_options_default": (i32, [ctypes.POINTER(Options)]),
        "dobfs_next_direction": (i32, [ctypes.POINTER(Options), i32, i64, i64, i64, i64, i64]),
        "dobfs_bfs_workspace_bytes": (i32, [vp, ctypes.POINTER(Options), ctypes.POINTER(sz)]),
        "dobfs_bfs": (i32, [vp, i32, ctypes.POINTER(Options), vp, vp, vp, sz, vp, ctypes.POINTER(Stats)]),
        "dobfs_bfs_static": (i32, [vp, i32, ctypes.POINTER(Options), vp, vp, vp, ctypes.POINTER(Stats)]),
        "dobfs_bfs_batch_workspace_bytes": (i32, [vp, i32, ctypes.POINTER(sz)]),
        "dobfs_bfs_batch": (i32, [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(Options), vp, vp, sz, vp,
                                  ctypes.POINTER(Stats)]),
        "dobfs_mxv_workspace_bytes": (i32, [vp, ctypes.POINTER(sz)]),
        "dobfs_mxv": (i32, [vp, vp, vp, i32, vp, i32, i32, u32, vp, vp, vp, ctypes.POINTER(i32), vp,
                            sz, vp]),
        "dobfs_server_options_default": (i32, [ctypes.POINTER(ServerOptions)]),
        "dobfs_server_create": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(ServerOptions),
                                      ctypes.POINTER(vp)]),
        "dobfs_server_submit": (i32, [vp, i32, i32, vp, ctypes.POINTER(ctypes.c_uint64)]),
        "dobfs_server_wait": (i32, [vp, ctypes.c_uint64, i32, ctypes.POINTER(QueryInfo)]),
        "dobfs_server_destroy": (i32, [vp]),
        "dobfs_status_string": (ctypes.c_char_p, [i32]),
        "dobfs_last_error": (ctypes.c_char_p, []),
        "dobfs_version": (i32, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    _lib = lib
    return lib


def header_functions() -> list:
    """Names of the functions include/dobfs.h declares."""
    with open(HEADER_PATH) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(dobfs_[a-z_0-9]+)\s*\(", text)))


def _check(status: int):
    if status != OK:
        raise DobfsError(status, load().dobfs_last_error().decode())


def _dptr(t, dtype, n, name):
    """Device pointer of a contiguous torch CUDA tensor with at least n elements."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < n:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), n))
    return t.data_ptr()


def _stream(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Graph:
    """Handle of a device-resident graph (dobfs_graph). Destroyed on garbage collection."""

    def __init__(self, handle, V: int, nnz: int, device: int, keepalive=None):
        self.handle = handle
        self.V, self.nnz, self.device = V, nnz, device
        self._keepalive = keepalive

    @property
    def nwords(self) -> int:
        return (self.V + 31) // 32

    def __del__(self):
        try:
            if self.handle:
                graph_destroy(self)
        except Exception:
            pass


def graph_upload(V, nnz, csr_rowptr, csr_colind, csc_colptr, csc_rowind, device=0, flags=0) -> Graph:
    """dobfs_graph_upload: host int32 arrays -> library-owned device copy."""
    lib = load()
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (csr_rowptr, csr_colind)]
    if csc_colptr is csr_rowptr and csc_rowind is csr_colind:
        arrs += arrs  # same host arrays: uploaded once
    else:
        arrs += [np.ascontiguousarray(a, dtype=np.int32) for a in (csc_colptr, csc_rowind)]
    h = ctypes.c_void_p()
    _check(lib.dobfs_graph_upload(int(V), int(nnz), *[a.ctypes.data for a in arrs], int(device),
                                  int(flags), ctypes.byref(h)))
    return Graph(h.value, int(V), int(nnz), int(device))


def graph_wrap_device(V, nnz, csr_rowptr, csr_colind, csc_colptr, csc_rowind, device=0, flags=0,
                      stream=None) -> Graph:
    """dobfs_graph_wrap_device: borrow int32 CUDA tensors (kept alive by the returned Graph)."""
    import torch
    lib = load()
    ptrs = [_dptr(t, torch.int32, n, nm) for t, n, nm in
            ((csr_rowptr, V + 1, "csr_rowptr"), (csr_colind, nnz, "csr_colind"),
             (csc_colptr, V + 1, "csc_colptr"), (csc_rowind, nnz, "csc_rowind"))]
    h = ctypes.c_void_p()
    _check(lib.dobfs_graph_wrap_device(int(V), int(nnz), *ptrs, int(device), int(flags),
                                       _stream(stream, device), ctypes.byref(h)))
    return Graph(h.value, int(V), int(nnz), int(device),
                 keepalive=(csr_rowptr, csr_colind, csc_colptr, csc_rowind))


def graph_destroy(g: Graph):
    h, g.handle = g.handle, None
    if h:
        _check(load().dobfs_graph_destroy(h))


def graph_info(g: Graph):
    V, nnz, dev = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
    _check(load().dobfs_graph_info(g.handle, ctypes.byref(V), ctypes.byref(nnz), ctypes.byref(dev)))
    return V.value, nnz.value, dev.value


def options_default() -> Options:
    o = Options()
    _check(load().dobfs_options_default(ctypes.byref(o)))
    return o


SCHED_FIELDS = ("pull_mid", "bitmap_rows", "local_unit", "local_chunks")


def make_options(mode="full", heuristic=HEUR_RATIO, alpha=0.01, beta=0.01, forced_dirs=None,
                 time_kernels=False, persistent=False, sched=None) -> Options:
    """An Options struct; forced_dirs (list of DIR_*) is kept alive on the struct; sched: a dict
    of schedule settings (SCHED_FIELDS; missing or 0 = the library's default)."""
    o = options_default()
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.heuristic = int(heuristic)
    o.alpha, o.beta = float(alpha), float(beta)
    if forced_dirs is not None:
        buf = np.ascontiguousarray(forced_dirs, dtype=np.int8)
        o._forced = buf
        o.forced_dirs = buf.ctypes.data
        o.n_forced = buf.size
    o.flags = (OPT_TIME_KERNELS if time_kernels else 0) | (OPT_PERSISTENT if persistent else 0)
    for k, v in (sched or {}).items():
        if k not in SCHED_FIELDS:
            raise ValueError("unknown schedule setting %r" % k)
        setattr(o, k, int(v))
    return o


def next_direction(opt, dir, V, nf, n_new, m_f=0, m_u=0) -> int:
    return int(load().dobfs_next_direction(ctypes.byref(opt) if opt is not None else None, int(dir),
                                           int(V), int(nf), int(n_new), int(m_f), int(m_u)))


def bfs_workspace_bytes(g: Graph, opt=None) -> int:
    n = ctypes.c_size_t()
    _check(load().dobfs_bfs_workspace_bytes(g.handle, ctypes.byref(opt) if opt else None,
                                            ctypes.byref(n)))
    return n.value


def bfs_batch_workspace_bytes(g: Graph, k: int) -> int:
    n = ctypes.c_size_t()
    _check(load().dobfs_bfs_batch_workspace_bytes(g.handle, int(k), ctypes.byref(n)))
    return n.value


def mxv_workspace_bytes(g: Graph) -> int:
    n = ctypes.c_size_t()
    _check(load().dobfs_mxv_workspace_bytes(g.handle, ctypes.byref(n)))
    return n.value


def make_stats(cap: int = 0) -> Stats:
    st = Stats()
    st.cap = int(cap)
    if cap:
        st._levels = (LevelStats * cap)()
        st.level = ctypes.cast(st._levels, ctypes.POINTER(LevelStats))
    return st


def stats_levels(st: Stats) -> list:
    n = min(st.levels, st.cap)
    return [dict(dir=st.level[k].dir, nf=st.level[k].nf, n_new=st.level[k].n_new,
                 edges=st.level[k].edges, m_f=st.level[k].m_f, ms_main=st.level[k].ms_main,
                 ms_aux=st.level[k].ms_aux, variant=st.level[k].variant) for k in range(n)]


def bfs(g: Graph, source: int, depth, parent=None, opt=None, workspace=None, ws_bytes=None,
        stream=None, stats=None):
    """dobfs_bfs: depth/parent are int32 CUDA tensors of V elements; workspace a uint8 CUDA
    tensor (or None for the library's own)."""
    import torch
    lib = load()
    d = _dptr(depth, torch.int32, g.V, "depth")
    p = _dptr(parent, torch.int32, g.V, "parent")
    w = _dptr(workspace, torch.uint8, 0, "workspace")
    nbytes = workspace.numel() if workspace is not None else 0
    if ws_bytes is not None:
        nbytes = int(ws_bytes)
    _check(lib.dobfs_bfs(g.handle, int(source), ctypes.byref(opt) if opt is not None else None,
                         d, p, w, nbytes, _stream(stream, g.device),
                         ctypes.byref(stats) if stats is not None else None))
    return stats


def bfs_static(g: Graph, source: int, depth, parent=None, opt=None, stream=None, stats=None):
    """dobfs_bfs_static: dobfs_bfs with the library's static device scratch as its workspace
    (no allocation inside the call); depth/parent are int32 CUDA tensors of V elements."""
    import torch
    lib = load()
    d = _dptr(depth, torch.int32, g.V, "depth")
    p = _dptr(parent, torch.int32, g.V, "parent")
    _check(lib.dobfs_bfs_static(g.handle, int(source), ctypes.byref(opt) if opt is not None else None,
                                d, p, _stream(stream, g.device),
                                ctypes.byref(stats) if stats is not None else None))
    return stats


def bfs_batch(g: Graph, sources, depth, opt=None, workspace=None, ws_bytes=None, stream=None,
              stats=None):
    """dobfs_bfs_batch: `sources` a host sequence of k ints (1 <= k <= 64); depth an int32 CUDA
    tensor of k*V elements (row b = depths from sources[b]); workspace a uint8 CUDA tensor or None."""
    import torch
    lib = load()
    src = [int(x) for x in sources]
    k = len(src)
    arr = (ctypes.c_int32 * max(k, 1))(*src)
    d = _dptr(depth, torch.int32, k * g.V, "depth")
    w = _dptr(workspace, torch.uint8, 0, "workspace")
    nbytes = workspace.numel() if workspace is not None else 0
    if ws_bytes is not None:
        nbytes = int(ws_bytes)
    _check(lib.dobfs_bfs_batch(g.handle, arr, k, ctypes.byref(opt) if opt is not None else None, d, w,
                               nbytes, _stream(stream, g.device),
                               ctypes.byref(stats) if stats is not None else None))
    return stats


class Server:
    """Handle of a query server (dobfs_server) over device-resident graphs; destroyed by close()
    or on garbage collection. Keeps the graphs and every submitted depth buffer alive until the
    server is gone."""

    def __init__(self, graphs, slots=4, max_batch=64, mem_budget=0, opt=None):
        lib = load()
        so = ServerOptions()
        _check(lib.dobfs_server_options_default(ctypes.byref(so)))
        so.slots, so.max_batch, so.mem_budget = int(slots), int(max_batch), int(mem_budget)
        if opt is not None:
            so.opt = opt
        self.graphs = list(graphs)
        arr = (ctypes.c_void_p * len(self.graphs))(*[g.handle for g in self.graphs])
        h = ctypes.c_void_p()
        _check(lib.dobfs_server_create(arr, len(self.graphs), ctypes.byref(so), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, graph: int, source: int, depth) -> int:
        """Queue a BFS; depth is an int32 CUDA tensor of the graph's V elements. The server's
        slots run on streams of their own, not ordered after torch's: work queued on any stream
        that writes depth (a fill, say) must be complete before the call."""
        import torch
        g = self.graphs[graph] if 0 <= graph < len(self.graphs) else self.graphs[0]
        d = _dptr(depth, torch.int32, g.V, "depth")
        qid = ctypes.c_uint64()
        _check(load().dobfs_server_submit(self.handle, int(graph), int(source), d, ctypes.byref(qid)))
        self._keep[qid.value] = depth
        return qid.value

    def wait(self, qid: int, timeout_ms: int = -1) -> dict:
        """Block until query qid is done (DobfsError with ERR_TIMEOUT past timeout_ms)."""
        info = QueryInfo()
        _check(load().dobfs_server_wait(self.handle, int(qid), int(timeout_ms), ctypes.byref(info)))
        self._keep.pop(int(qid), None)
        return dict(graph=info.graph, source=info.source, batch_size=info.batch_size,
                    status=info.status, t_submit_ms=info.t_submit_ms, t_start_ms=info.t_start_ms,
                    t_done_ms=info.t_done_ms)

    def close(self):
        if self.handle:
            _check(load().dobfs_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mxv(g: Graph, y_bits, x_bits=None, x_idx=None, x_nnz=None, mask_bits=None, complement=False,
        direction=DIR_PULL, flags=0, y_idx=None, y_witness=None, want_nnz=True, workspace=None,
        stream=None):
    """dobfs_mxv: bit vectors are int32 CUDA tensors of ceil(V/32) words (uint32 bit patterns);
    x_idx / y_idx / y_witness int32 CUDA tensors. Returns nnz(y) when want_nnz."""
    import torch
    lib = load()
    nw = g.nwords
    xb = _dptr(x_bits, torch.int32, nw, "x_bits")
    xi = _dptr(x_idx, torch.int32, 0, "x_idx")
    n = int(x_nnz if x_nnz is not None else (x_idx.numel() if x_idx is not None else 0))
    mb = _dptr(mask_bits, torch.int32, nw, "mask_bits")
    yb = _dptr(y_bits, torch.int32, nw, "y_bits")
    yi = _dptr(y_idx, torch.int32, g.V, "y_idx")
    yw = _dptr(y_witness, torch.int32, g.V, "y_witness")
    w = _dptr(workspace, torch.uint8, 0, "workspace")
    nbytes = workspace.numel() if workspace is not None else 0
    out = ctypes.c_int32(-1)
    _check(lib.dobfs_mxv(g.handle, xb, xi, n, mb, int(bool(complement)), int(direction), int(flags),
                         yb, yi, yw, ctypes.byref(out) if want_nnz else None, w, nbytes,
                         _stream(stream, g.device)))
    return out.value if want_nnz else None


def status_string(s: int) -> str:
    return load().dobfs_status_string(int(s)).decode()


def last_error() -> str:
    return load().dobfs_last_error().decode()


def version() -> int:
    return int(load().dobfs_version())
