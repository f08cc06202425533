"""Autotuner for the per-level direction rule (Section 6.3).

The rule's constants decide, level by level, between the push and the pull; the paper tuned
alpha = beta = 0.01 of its ratio form by hand on its GPU. This tuner measures instead: it times
the traversal on a set of tuning sources for every candidate (rule, alpha, beta) and keeps the
fastest. Depths do not depend on the choice (every schedule computes the same level sets), so
the tuner only ever trades time. Tuning sources should be disjoint from the ones a result is
reported on.
"""
from __future__ import annotations

import itertools
import time

from . import dobfs

# Candidate constants: the ratio form around the paper's 0.01, and the edge-count form around
# Beamer's alpha = 1/14, beta = 1/24 (push -> pull when m_f > alpha * m_u; back when
# n_new < beta * V).
RATIO_GRID = [0.002, 0.005, 0.01, 0.02, 0.05]
EDGES_ALPHA = [1 / 40, 1 / 28, 1 / 20, 1 / 14, 1 / 10, 1 / 6, 1 / 3]
EDGES_BETA = [1 / 96, 1 / 48, 1 / 24, 1 / 12]


def candidates():
    """Every (heuristic, alpha, beta) the tuner tries."""
    out = [(dobfs.HEUR_RATIO, a, a) for a in RATIO_GRID]
    out += [(dobfs.HEUR_EDGES, a, b) for a, b in itertools.product(EDGES_ALPHA, EDGES_BETA)]
    return out


def _time_single(g, sources, opt, ws, depth, parent, reps):
    import torch
    for s in sources[:2]:
        dobfs.bfs(g, s, depth, parent, opt, ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        for s in sources:
            dobfs.bfs(g, s, depth, parent, opt, ws)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / (reps * len(sources))


def tune_single(g, sources, reps: int = 2, mode: str = "full"):
    """Fastest direction rule for single-source traversals of graph g over `sources`.

    Returns a dict: heuristic, alpha, beta, ms (mean per traversal), and `table`, every
    candidate's mean time in ms."""
    import torch
    dev = torch.device("cuda", g.device)
    depth = torch.empty(g.V, dtype=torch.int32, device=dev)
    parent = torch.empty(g.V, dtype=torch.int32, device=dev)
    ws = torch.empty(dobfs.bfs_workspace_bytes(g), dtype=torch.uint8, device=dev)
    table = []
    for heur, a, b in candidates():
        opt = dobfs.make_options(mode, heur, a, b)
        table.append((heur, a, b, 1e3 * _time_single(g, sources, opt, ws, depth, parent, reps)))
    heur, a, b, ms = min(table, key=lambda r: r[3])
    return dict(heuristic=heur, alpha=a, beta=b, ms=ms, table=table)


def tune_batch(g, sources, reps: int = 2):
    """Fastest direction rule for one multi-source launch over `sources` (up to 64)."""
    import torch
    dev = torch.device("cuda", g.device)
    k = len(sources)
    depth = torch.empty(k * g.V, dtype=torch.int32, device=dev)
    ws = torch.empty(dobfs.bfs_batch_workspace_bytes(g, k), dtype=torch.uint8, device=dev)
    table = []
    for heur, a, b in candidates():
        opt = dobfs.make_options("full", heur, a, b)
        dobfs.bfs_batch(g, sources, depth, opt=opt, workspace=ws)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            dobfs.bfs_batch(g, sources, depth, opt=opt, workspace=ws)
        torch.cuda.synchronize()
        table.append((heur, a, b, 1e3 * (time.perf_counter() - t) / reps))
    heur, a, b, ms = min(table, key=lambda r: r[3])
    return dict(heuristic=heur, alpha=a, beta=b, ms=ms, table=table)


def describe(result) -> str:
    name = "edges" if result["heuristic"] == dobfs.HEUR_EDGES else "ratio"
    return "%s alpha=%.4g beta=%.4g" % (name, result["alpha"], result["beta"])
