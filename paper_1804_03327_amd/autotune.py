"""Autotuner for the direction rule (Section 6.3) and the schedule settings of the kernels.

The rule's constants decide, level by level, between the push and the pull; the paper tuned
alpha = beta = 0.01 of its ratio form by hand on its GPU. This tuner measures instead: it times
the traversal on a set of tuning sources for every candidate (rule, alpha, beta) and keeps the
fastest, then walks the schedule settings of the single-source kernels one at a time (the
pull's thread-to-wave cut-over, the row limit of the block-local push over a pull's bits, the
local push's unit size and its chunk limit), keeping a value only when it beats the best so far
by more than the measured noise. Every candidate is timed as `reps` separate passes over the
sources; the noise band of a comparison is twice the combined standard error of the two means.
Depths do not depend on any choice (every schedule computes the same level sets), so the tuner
only ever trades time. Tuning sources should be disjoint from the ones a result is reported on.
"""
from __future__ import annotations

import itertools
import math
import time

from . import dobfs

# Candidate constants: the ratio form around the paper's 0.01, and the edge-count form around
# Beamer's alpha = 1/14, beta = 1/24 (push -> pull when m_f > alpha * m_u; back when
# n_new < beta * V).
RATIO_GRID = [0.002, 0.005, 0.01, 0.02, 0.05]
EDGES_ALPHA = [1 / 40, 1 / 28, 1 / 20, 1 / 14, 1 / 10, 1 / 6, 1 / 3]
EDGES_BETA = [1 / 96, 1 / 48, 1 / 24, 1 / 12]

# Schedule settings and the values tried (the library's defaults: 32, 512, 128, 4).
SCHED_GRID = {
    "pull_mid": [8, 16, 32, 64, 128],
    "bitmap_rows": [0, 128, 256, 512, 1024, 2048, 4096],
    "local_unit": [32, 64, 128, 256],
    "local_chunks": [1, 2, 4, 8, 16],
}
SCHED_DEFAULT = {"pull_mid": 32, "bitmap_rows": 512, "local_unit": 128, "local_chunks": 4}


def candidates():
    """Every (heuristic, alpha, beta) the tuner tries."""
    out = [(dobfs.HEUR_RATIO, a, a) for a in RATIO_GRID]
    out += [(dobfs.HEUR_EDGES, a, b) for a, b in itertools.product(EDGES_ALPHA, EDGES_BETA)]
    return out


class _Timer:
    """Times passes of single-source traversals over fixed sources with caller-owned buffers."""

    def __init__(self, g, sources, mode):
        import torch
        dev = torch.device("cuda", g.device)
        self.g, self.sources, self.mode = g, list(sources), mode
        self.depth = torch.empty(g.V, dtype=torch.int32, device=dev)
        self.parent = torch.empty(g.V, dtype=torch.int32, device=dev)
        self.ws = torch.empty(dobfs.bfs_workspace_bytes(g), dtype=torch.uint8, device=dev)

    def passes(self, heur, a, b, sched, reps):
        """Mean ms per traversal of each of `reps` passes over the sources (after a warm-up)."""
        import torch
        opt = dobfs.make_options(self.mode, heur, a, b, sched=sched)
        for s in self.sources[:2]:
            dobfs.bfs(self.g, s, self.depth, self.parent, opt, self.ws)
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            t = time.perf_counter()
            for s in self.sources:
                dobfs.bfs(self.g, s, self.depth, self.parent, opt, self.ws)
            torch.cuda.synchronize()
            out.append(1e3 * (time.perf_counter() - t) / len(self.sources))
        return out


def _mean_se(xs):
    m = sum(xs) / len(xs)
    if len(xs) < 2:
        return m, 0.0
    var = sum((x - m) ** 2 for x in xs) / (len(xs) - 1)
    return m, math.sqrt(var / len(xs))


def _band(se_a, se_b):
    """Noise band of a difference of two means: twice their combined standard error."""
    return 2.0 * math.sqrt(se_a * se_a + se_b * se_b)


def tune_single(g, sources, reps: int = 3, mode: str = "full"):
    """Fastest direction rule for single-source traversals of graph g over `sources`.

    Returns a dict: heuristic, alpha, beta, ms (mean per traversal), se (its standard error) and
    `table`, every candidate's mean time in ms."""
    tm = _Timer(g, sources, mode)
    table = []
    for heur, a, b in candidates():
        m, se = _mean_se(tm.passes(heur, a, b, None, reps))
        table.append((heur, a, b, m, se))
    heur, a, b, ms, se = min(table, key=lambda r: r[3])
    return dict(heuristic=heur, alpha=a, beta=b, ms=ms, se=se, table=[r[:4] for r in table])


def tune_schedule(g, sources, reps: int = 3, mode: str = "full", rule=None):
    """The direction rule (tune_single, unless `rule` = (heuristic, alpha, beta) is given), then
    the schedule settings one at a time, each value tried with the others at their best so far;
    a value replaces the best only when its mean is lower by more than the noise band.

    Returns heuristic, alpha, beta, sched (every setting), ms and se of the result, default_ms
    and default_se (the same rule with the default settings), and `steps`: for every setting,
    the mean ms of every value tried."""
    tm = _Timer(g, sources, mode)
    if rule is None:
        r = tune_single(g, sources, reps, mode)
        rule = (r["heuristic"], r["alpha"], r["beta"])
    heur, a, b = rule
    best = dict(SCHED_DEFAULT)
    best_m, best_se = _mean_se(tm.passes(heur, a, b, best, reps))
    default_m, default_se = best_m, best_se
    steps = {}
    for name, values in SCHED_GRID.items():
        tried = {}
        for v in values:
            if v == best[name]:
                tried[v] = round(best_m, 5)
                continue
            cand = dict(best, **{name: v})
            m, se = _mean_se(tm.passes(heur, a, b, cand, reps))
            tried[v] = round(m, 5)
            if best_m - m > _band(se, best_se):
                best, best_m, best_se = cand, m, se
        steps[name] = tried
    return dict(heuristic=heur, alpha=a, beta=b, sched=best, ms=best_m, se=best_se,
                default_ms=default_m, default_se=default_se, steps=steps)


def tune_batch(g, sources, reps: int = 3):
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
        xs = []
        for _ in range(reps):
            t = time.perf_counter()
            dobfs.bfs_batch(g, sources, depth, opt=opt, workspace=ws)
            torch.cuda.synchronize()
            xs.append(1e3 * (time.perf_counter() - t))
        m, se = _mean_se(xs)
        table.append((heur, a, b, m, se))
    heur, a, b, ms, se = min(table, key=lambda r: r[3])
    return dict(heuristic=heur, alpha=a, beta=b, ms=ms, se=se, table=[r[:4] for r in table])


def describe(result) -> str:
    name = "edges" if result["heuristic"] == dobfs.HEUR_EDGES else "ratio"
    out = "%s alpha=%.4g beta=%.4g" % (name, result["alpha"], result["beta"])
    if "sched" in result:
        out += " " + " ".join("%s=%d" % kv for kv in sorted(result["sched"].items()))
    return out
