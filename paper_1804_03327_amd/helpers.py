"""Conveniences around the binding: graph upload from host arrays, bit-vector packing and a
runner that keeps depth / parent / workspace tensors allocated across BFS calls. Plumbing
only: no BFS or matvec arithmetic happens here."""
from __future__ import annotations

import numpy as np

from . import dobfs


def pack_bits(mask) -> np.ndarray:
    """bool[V] -> int32[ceil(V/32)]: bit i is bit (i & 31) of word i >> 5."""
    mask = np.asarray(mask).astype(bool).ravel()
    nw = (mask.size + 31) // 32
    padded = np.zeros(nw * 32, dtype=np.uint8)
    padded[:mask.size] = mask
    return np.packbits(padded, bitorder="little").view("<u4").view(np.int32)


def unpack_bits(words, V: int) -> np.ndarray:
    """int32/uint32 words -> bool[V]."""
    w = np.ascontiguousarray(np.asarray(words)).view(np.uint32).astype("<u4")
    return np.unpackbits(w.view(np.uint8), bitorder="little")[:V].astype(bool)


def upload(hg, device: int = 0, validate: bool = False, hubs_first: bool = False) -> dobfs.Graph:
    """Upload a host graph with CSR(A) (rowptr, colind) and CSC(A) (csc_colptr, csc_rowind);
    hubs_first keeps each row's in-neighbours ordered by decreasing out-degree on the device."""
    flags = (dobfs.UPLOAD_VALIDATE if validate else 0) | (dobfs.UPLOAD_HUBS_FIRST if hubs_first else 0)
    return dobfs.graph_upload(hg.V, hg.nnz, hg.rowptr, hg.colind, hg.csc_colptr, hg.csc_rowind,
                              device=device, flags=flags)



class BfsRunner:
    """Repeated dobfs_bfs calls on one graph with caller-owned outputs and workspace."""

    def __init__(self, g: dobfs.Graph, with_parent: bool = True, stats_cap: int = 4096):
        import torch
        self.g = g
        dev = torch.device("cuda", g.device)
        self.depth = torch.empty(g.V, dtype=torch.int32, device=dev)
        self.parent = torch.empty(g.V, dtype=torch.int32, device=dev) if with_parent else None
        self.ws = torch.empty(dobfs.bfs_workspace_bytes(g), dtype=torch.uint8, device=dev)
        self.stats = dobfs.make_stats(stats_cap)

    def run(self, source: int, mode="full", heuristic=dobfs.HEUR_RATIO, alpha=0.01, beta=0.01,
            forced_dirs=None, time_kernels=False, stream=None, opt=None, persistent=False):
        if opt is None:
            opt = dobfs.make_options(mode, heuristic, alpha, beta, forced_dirs, time_kernels, persistent)
        dobfs.bfs(self.g, source, self.depth, self.parent, opt, self.ws, stream=stream,
                  stats=self.stats)
        return self.stats

    def result(self):
        """(depth, parent) as host numpy arrays (synchronizes)."""
        d = self.depth.cpu().numpy()
        p = self.parent.cpu().numpy() if self.parent is not None else None
        return d, p

    def levels(self) -> list:
        return dobfs.stats_levels(self.stats)
