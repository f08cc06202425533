"""Benchmark: single-source direction-optimized BFS on RMAT scale 22 (edge factor 16) on one
MI355X, through the C ABI.

A step is one BFS from each of the 64 seeded sources (vertices with degree > 0). The metric
is GTEPS with the Graph500 edge count (undirected edges with a reached endpoint); the
paper-convention figure (nnz(A) / time) is reported beside it. Prints one JSON line.

Also reported: the HBM roofline of the dominant kernel (algorithmic bytes per launch over its
average execution time, from each kernel's own start/end events in a repeat of the timed
steps), the CPU oracle on a bounded sample of the same workload, the Table 2 ablation modes,
the other direction rule, the autotuner, the 256^3 lattice, the paper's own scale-22 graph (edge
factor 64) beside its published figure, the multi-source measurement (64 sources per launch on
RMAT-20 against the same 64 queries run one at a time) and the query server (four graphs,
Poisson arrivals from 0.5x to 16x the sequential capacity, p50/p99 latency against first-in
first-out plain DOBFS).

--profile-steps / --profile-batched / --profile-lattice run only the BFS launches (for rocprofv3); --copy-mb adds
one device copy of known size as the reference for scaling the PMC byte counters.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ATOMIC_CEILING_PER_S = 27e9  # device atomics on distinct words, measured on MI355X
METRIC = "GTEPS DOBFS RMAT-22 (1 GPU)"
KERNEL_DIR = os.path.join(ROOT, "paper_1804_03327_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the sources the single-source kernels (k_bfs_init, k_step) are compiled from: kernels.hip and
# the headers it includes (the multi-source, sort and host files do not change them); the
# multi-source kernels likewise come from batch.hip and the same headers
SINGLE_SOURCE_KERNEL_FILES = ("kernels.hip", "device_common.h", "dobfs_internal.h", "dobfs.h")
MULTI_SOURCE_KERNEL_FILES = ("batch.hip", "device_common.h", "dobfs_internal.h", "dobfs.h")


def kernel_source_hash(files=SINGLE_SOURCE_KERNEL_FILES) -> str:
    """SHA-256 (16 hex digits) over the sources of a group of kernels."""
    h = hashlib.sha256()
    for name in files:
        path = os.path.join(KERNEL_DIR, name)
        if not os.path.exists(path):
            path = os.path.join(ROOT, "include", name)
        with open(path, "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


# ------------------------------------------------------------- byte model
# Algorithmic bytes each kernel must move (int32 indices; random bit lookups into the
# L2-resident visited / frontier bitmaps count 0).
def bytes_push_scan(nf):
    return 4 * nf + 8 * nf + 8 * nf  # frontier ids, rowptr pair, (scan, row start) written


def bytes_push_expand(nf, m_f, n_new):
    return 12 * nf + 4 * m_f + 12 * n_new  # (scan, start, id) per vertex, adjacency, depth/parent/queue


def bytes_pull(V, n_cand, checks, n_new):
    # visited + nonzero-row words read, new visited words written, colptr pair per candidate
    # row, one index per in-neighbour checked, depth + parent per discovery
    return 3 * V / 8 + 8 * n_cand + 4 * checks + 8 * n_new


def bytes_d2s(V, n):
    return 2 * V / 8 + 4 * n


def bytes_local_expand(nf, m_f, n_new):
    return 12 * nf + 4 * m_f + 12 * n_new  # (id, offset pair) per vertex, adjacency, depth/parent/queue


def bytes_mu_recount(V):
    return 2 * V / 8  # nz and visited words (edge-count rule, first push after a pull)


def bytes_init(V):
    return 8 * V + V / 8


def candidates_per_level(depth, indeg_nz):
    """Rows a level-L pull lists: in-degree > 0 and not visited at level start (depth <= L)."""
    d = depth[indeg_nz]
    reached = d[d >= 0]
    cnt = np.bincount(reached) if reached.size else np.zeros(1, dtype=np.int64)
    total = int(indeg_nz.sum())
    return total - np.cumsum(cnt)  # index L -> candidates at level L


def load_traffic(kernel: str, workload: str = "rmat22"):
    """HBM traffic per launch from committed rocprofv3 PMC summaries, or None when absent or
    taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def load_mb_traffic(levels):
    """HBM traffic per push or pull step of k_mb_step (scan steps and the steps past the end
    left out, as in the batched roofline) from the committed PMC summary of one 64-source
    RMAT-20 launch, or None when absent, taken on other kernel sources, or when that launch's
    level directions differ from `levels`."""
    path = os.path.join(ROOT, "profiles", "traffic_mb_step_rmat20.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256_16") != kernel_source_hash(MULTI_SOURCE_KERNEL_FILES):
        return None
    if t.get("levels") != list(levels):
        return None
    return t.get("bytes_per_push_or_pull_step")


def step_roofline(V, heur, runs, cand_tables, traffic):
    """Per-kernel table and the roofline of the dominant kernel from timed traversals.

    runs: (source, stats) of traversals made with DOBFS_OPT_TIME_KERNELS; cand_tables[source]:
    the rows each level's pull lists (from the oracle's depths). The kernels are k_bfs_init and
    k_step (one launch per level, two for a push level that needs the global degree scan); the
    push / pull split of the steps' time (scan steps apart) is reported beside them. Returns
    (roofline, kernel table, per-BFS ms)."""
    from paper_1804_03327_amd import dobfs
    kinds = {k: {"ms": 0.0, "launches": 0, "bytes": 0.0} for k in
             ("step", "init", "push", "push_scan", "pull")}
    push_edges, push_big = 0, {"edges": 0, "ms": 0.0, "levels": 0}

    def add(kind, ms, nbytes, launches=1):
        kinds[kind]["ms"] += ms
        kinds[kind]["launches"] += launches
        kinds[kind]["bytes"] += nbytes

    bfs_ms = []
    for s, st in runs:
        if st.levels > st.cap:
            raise RuntimeError("level stats truncated: %d levels > cap %d" % (st.levels, st.cap))
        bfs_ms.append(st.ms_total)
        add("init", st.ms_init, bytes_init(V))
        prev = dobfs.DIR_PUSH
        step_bytes = 0
        for L, lv in enumerate(dobfs.stats_levels(st)):
            if lv["dir"] == dobfs.DIR_PUSH:
                after_pull = prev == dobfs.DIR_PULL
                mu = bytes_mu_recount(V) if (after_pull and heur == dobfs.HEUR_EDGES) else 0
                if lv["variant"] == 0:  # scan step, then expansion step
                    scan = bytes_push_scan(lv["nf"]) + (bytes_d2s(V, lv["nf"]) + mu if after_pull else 0)
                    main = bytes_push_expand(lv["nf"], lv["m_f"], lv["n_new"])
                    add("push_scan", lv["ms_aux"], scan)
                    step_bytes += scan
                elif lv["variant"] == 1:  # block-local over the frontier list
                    main = bytes_local_expand(lv["nf"], lv["m_f"], lv["n_new"])
                else:  # block-local over the bits the pull found
                    main = V / 8 + mu + bytes_local_expand(lv["nf"], lv["m_f"], lv["n_new"]) - 4 * lv["nf"]
                add("push", lv["ms_main"], main)
                # the push's adjacency entries, each one plain load of a visited word and, when the
                # target still looks unvisited, one atomic claim: against the atomic rate
                push_edges += lv["edges"]
                if lv["edges"] >= 1 << 15:  # the pushes large enough to keep the atomics busy
                    push_big["edges"] += lv["edges"]
                    push_big["ms"] += lv["ms_main"] + lv["ms_aux"]
                    push_big["levels"] += 1
            else:
                nc = cand_tables[s][L] if L < len(cand_tables[s]) else cand_tables[s][-1]
                main = bytes_pull(V, int(nc), lv["edges"], lv["n_new"])
                add("pull", lv["ms_main"], main)
            step_bytes += main
            prev = lv["dir"]
        # every launch of the step kernel, as a profiler counts them: the levels' steps,
        # the step that finds the end and those enqueued past it (no work, no bytes)
        add("step", st.ms_main_all, step_bytes, st.launches_main)
    dom = max(("step", "init"), key=lambda k: kinds[k]["ms"])
    kd = kinds[dom]
    avg_ms = kd["ms"] / max(1, kd["launches"])
    per_launch = kd["bytes"] / max(1, kd["launches"])
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": "k_" + dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic if dom == "step" else None,
                "algorithmic_bytes_per_launch": round(per_launch),
                "avg_launch_us": round(avg_ms * 1e3, 3), "launches": kd["launches"]}
    kernel_table = {k: {"total_ms": round(v["ms"], 3), "launches": v["launches"],
                        "avg_us": round(1e3 * v["ms"] / max(1, v["launches"]), 3),
                        "GBps": round(v["bytes"] / max(1e-12, v["ms"] * 1e-3) / 1e9, 1)}
                    for k, v in kinds.items()}
    # push levels against the atomic ceiling (27 G/s for atomics on distinct words, measured on
    # the box): edges per second, each at most one claim
    kernel_table["push"]["edges_per_s"] = round(push_edges / max(1e-12, kinds["push"]["ms"] * 1e-3), 0)
    kernel_table["push"]["large_levels_edges_per_s"] = round(
        push_big["edges"] / max(1e-12, push_big["ms"] * 1e-3), 0)
    kernel_table["push"]["large_levels"] = push_big["levels"]
    kernel_table["push"]["atomic_ceiling_per_s"] = ATOMIC_CEILING_PER_S
    return roofline, kernel_table, bfs_ms


def validate_sources(hg, sources, run):
    """Runs run(s) -> (depth, parent) host arrays for every source on the GPU, one after another,
    and checks each against the oracle in a thread pool (the C oracle runs outside the GIL):
    depths equal, parents valid (parent None: depths only). Returns {source: oracle depth};
    exits on a mismatch."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle

    def check(s, d, p):
        want, _ = oracle.bfs(hg, s)
        if not np.array_equal(d, want):
            return s, None, "%d depths differ" % int((d != want).sum())
        if p is not None:
            code, at = oracle.validate(hg, s, d, p)
            if code:
                return s, None, "parent check %d failed at %d" % (code, at)
        return s, want, ""

    workers = max(1, min(16, os.cpu_count() or 1))
    out = {}
    with ThreadPoolExecutor(workers) as ex:
        futs = []
        for s in sources:
            d, p = run(s)
            futs.append(ex.submit(check, s, d, p))
        for f in futs:
            s, want, err = f.result()
            if err:
                raise SystemExit("bench: GPU result differs from the oracle on source %d: %s" % (s, err))
            out[s] = want
    return out


def loop_costs(g, srcs, heur, alpha, beta, reps, stream):
    """Mean ms per BFS and us per level of the two forms of the single-source level loop (one
    launch per step; the persistent kernel with a grid barrier between steps) over `srcs`."""
    import torch
    from paper_1804_03327_amd import dobfs
    from paper_1804_03327_amd.helpers import BfsRunner
    r = BfsRunner(g, with_parent=True)
    out = {}
    for name, pers in (("step_launches", False), ("persistent", True)):
        opt = dobfs.make_options("full", heur, alpha, beta, persistent=pers)
        st = dobfs.make_stats(0)
        levels = 0
        for s in srcs:
            dobfs.bfs(g, s, r.depth, r.parent, opt, r.ws, stream=stream, stats=st)
            levels += st.levels
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            for s in srcs:
                dobfs.bfs(g, s, r.depth, r.parent, opt, r.ws, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        out[name] = {"ms_per_bfs": round(1e3 * dt / len(srcs), 4), "us_per_level": round(1e6 * dt / levels, 2)}
    return out


def measure_lattice(args, heur, alpha, beta):
    """The high-diameter configuration: a 256^3 7-point lattice with 5% of its undirected edges
    deleted (seed 3), 16 sources (seed 4, degree > 0), in the benchmarked mode and rule. Every
    source is checked against the oracle; ms per BFS, GTEPS in both edge counts, the roofline of
    the dominant kernel and the single-core oracle on two of the sources."""
    import torch
    import gen
    import oracle
    from paper_1804_03327_amd import dobfs
    from paper_1804_03327_amd.helpers import BfsRunner, upload

    hl = gen.lattice3d(args.lattice_n, 0.05, seed=3)
    srcs = [int(x) for x in gen.sample_sources(hl, 16, seed=4)]
    gl = upload(hl, device=0, hubs_first=not args.stored_order)
    r = BfsRunner(gl, with_parent=True)
    stream = torch.cuda.current_stream()
    opt = dobfs.make_options("full", heur, alpha, beta)
    opt_t = dobfs.make_options("full", heur, alpha, beta, time_kernels=True)

    def run_one(s):
        r.run(s, opt=opt, stream=stream)
        return r.result()

    want = validate_sources(hl, srcs, run_one)
    edges = {s: oracle.teps_edges(hl, want[s])["graph500"] for s in srcs}
    cand = {s: candidates_per_level(want[s], hl.in_degree() > 0) for s in srcs}
    reps = 3
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        for s in srcs:
            dobfs.bfs(gl, s, r.depth, r.parent, opt, r.ws, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    n = reps * len(srcs)
    stats = [dobfs.make_stats(4096) for _ in srcs]
    for s, st in zip(srcs, stats):
        dobfs.bfs(gl, s, r.depth, r.parent, opt_t, r.ws, stream=stream, stats=st)
    torch.cuda.synchronize()
    roof, table, _ = step_roofline(hl.V, heur, list(zip(srcs, stats)), cand,
                                   load_traffic("step", "lattice%d" % args.lattice_n))
    levels = [st.levels for st in stats]
    loops = loop_costs(gl, srcs[:4], heur, alpha, beta, 1, stream)
    tuned = None
    if not args.no_autotune:  # the rule and schedule settings tuned on 4 other sources
        from paper_1804_03327_amd import autotune
        pool = [int(x) for x in gen.sample_sources(hl, 40, seed=5)]
        tsrc = [x for x in pool if x not in set(srcs)][:4]
        rt = autotune.tune_schedule(gl, tsrc, reps=2)
        ot = dobfs.make_options("full", rt["heuristic"], rt["alpha"], rt["beta"], sched=rt["sched"])
        passes = {"tuned": [], "fixed": []}
        for _ in range(2):
            for name, o in (("fixed", opt), ("tuned", ot)):
                t1 = time.perf_counter()
                for s in srcs[:8]:
                    dobfs.bfs(gl, s, r.depth, r.parent, o, r.ws, stream=stream)
                torch.cuda.synchronize()
                passes[name].append(1e3 * (time.perf_counter() - t1) / 8)
        tuned = {"settings": autotune.describe(rt), "ms_per_bfs": round(float(np.mean(passes["tuned"])), 4),
                 "ms_per_bfs_fixed_same_passes": round(float(np.mean(passes["fixed"])), 4),
                 "passes": 2, "timed_sources": 8, "tuning_sources": len(tsrc)}
        log("lattice autotuned:", json.dumps(tuned))
    cpu_src = srcs[:2]
    tc = 0.0
    for s in cpu_src:
        t2 = time.perf_counter()
        oracle.bfs(hl, s)
        tc += time.perf_counter() - t2
    res = {"workload": "lattice%d^3, 5%% of undirected edges deleted (seed 3), 16 sources (seed 4)" % args.lattice_n,
           "vertices": hl.V, "directed_edges": hl.nnz,
           "gteps": round(sum(edges.values()) * reps / dt / 1e9, 3),
           "gteps_paper_convention": round(hl.nnz * n / dt / 1e9, 3),
           "ms_per_bfs": round(1e3 * dt / n, 4),
           "levels_mean": round(float(np.mean(levels)), 1),
           "us_per_level": round(1e6 * dt / reps / max(1, sum(levels)), 3),
           "validated_sources": len(want),
           "level_loop": dict(loops, sources=4),
           "autotuned": tuned,
           "roofline": roof, "kernels": table,
           "cpu_baseline": {"value": round(sum(edges[s] for s in cpu_src) / tc / 1e9, 5), "unit": "GTEPS",
                            "cores": 1, "kind": "oracle",
                            "sample": "FIFO-queue BFS from 2 of the 16 sources (%.1f s)" % tc}}
    log("lattice:", json.dumps({k: v for k, v in res.items() if k != "kernels"}))
    dobfs.graph_destroy(gl)
    return res


# The paper's own RMAT scale-22 graph has edge factor 64 (483M directed edges): its DOBFS runs it
# in 4.781 ms, 101.0 GTEPS counted as nnz / time, on one Tesla K40c (Fig. 7 table, Table 3).
PAPER_RMAT22_EF64 = {"gpu": "Tesla K40c", "dataset": "rmat_s22_e64, 483M directed edges",
                     "ms_per_bfs": 4.781, "gteps_paper_convention": 101.038,
                     "where": "Fig. 7 table (This Work), Table 3"}


def measure_paper_scale(args, heur, alpha, beta):
    """Context beside the paper's figure for its scale-22 RMAT graph: the same generator at edge
    factor 64 (graph seed 1, 16 sources with seed 2), every source checked against the oracle,
    then timed in the benchmarked mode and rule and under the paper's ratio rule
    (alpha = beta = 0.01). Other hardware, so a context figure, not a target."""
    import torch
    import gen
    import oracle
    from paper_1804_03327_amd import dobfs
    from paper_1804_03327_amd.helpers import BfsRunner, upload

    t0 = time.time()
    hp = gen.rmat(args.scale, 64, seed=1)
    log("generated rmat%d ef64: V=%d nnz=%d in %.1fs" % (args.scale, hp.V, hp.nnz, time.time() - t0))
    srcs = [int(x) for x in gen.sample_sources(hp, 16, seed=2)]
    gp = upload(hp, device=0, hubs_first=not args.stored_order)
    r = BfsRunner(gp, with_parent=True)
    stream = torch.cuda.current_stream()
    opt = dobfs.make_options("full", heur, alpha, beta)
    opt_ratio = dobfs.make_options("full", dobfs.HEUR_RATIO, 0.01, 0.01)

    def run_one(s):
        r.run(s, opt=opt, stream=stream)
        return r.result()

    want = validate_sources(hp, srcs, run_one)
    edges = sum(oracle.teps_edges(hp, want[s])["graph500"] for s in srcs)
    levels = float(np.mean([int(want[s].max()) + 1 for s in srcs]))
    reps = 5
    res = {}
    for name, o in (("benchmarked_rule", opt), ("ratio_rule", opt_ratio)):
        for s in srcs[:4]:
            dobfs.bfs(gp, s, r.depth, r.parent, o, r.ws, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            for s in srcs:
                dobfs.bfs(gp, s, r.depth, r.parent, o, r.ws, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        res[name] = {"ms_per_bfs": round(1e3 * dt / (reps * len(srcs)), 4),
                     "gteps": round(edges * reps / dt / 1e9, 3),
                     "gteps_paper_convention": round(hp.nnz * reps * len(srcs) / dt / 1e9, 3)}
    out = {"workload": "rmat%d_ef64 (same a/b/c/d, graph seed 1), 16 sources (seed 2)" % args.scale,
           "vertices": hp.V, "directed_edges": hp.nnz, "levels_mean": round(levels, 2),
           "validated_sources": len(want),
           "heuristic": "%s alpha=%.4g beta=%.4g" % (args.heuristic, alpha, beta),
           "benchmarked_rule": res["benchmarked_rule"],
           "ratio_rule_alpha_beta_0.01": res["ratio_rule"],
           "paper": PAPER_RMAT22_EF64,
           "x_paper_ms_per_bfs": round(PAPER_RMAT22_EF64["ms_per_bfs"] / res["benchmarked_rule"]["ms_per_bfs"], 1)}
    log("paper scale:", json.dumps(out))
    dobfs.graph_destroy(gp)
    del r
    return out


def batched_roofline(gb, hb, srcs, rows, opt, ws, depth, stream, heur, alpha, beta, reps=5):
    """Roofline of the multi-source step kernel (k_mb_step) over the steps that push or pull
    (the bulk of a launch): algorithmic bytes of every level over its step's own execution time,
    from `reps` launches whose kernels are timed with start/end events. Bytes per level (int32
    indices, uint64 source words, each random word access counted at its size):
      push: 20 nf (list entry, offset pair, F[u]) + 12 m_f (column index, Vis[w]) + 12 n_new (claim, list)
      pull: 24 V (Vis read, Vis' and F' written) + 24 n_cand (slab, offset pair) + 12 checks
    where n_cand (rows with a source still expanding that has not reached them, in-degree > 0)
    comes from the 64 oracle-checked depth rows. The scan steps of push levels (merge, clears,
    degree scan) are reported beside it; `traffic` is the PMC-counted bytes per push or pull step
    of the same launch (load_mb_traffic)."""
    from paper_1804_03327_amd import dobfs
    import torch
    ot = dobfs.make_options("full", heur, alpha, beta, time_kernels=True)
    indeg_nz = hb.in_degree() > 0
    ecc = rows.max(axis=1)
    cand_cache = {}

    def n_cand(L):
        if L not in cand_cache:
            active = ecc >= L
            unreached = (rows[active] < 0) | (rows[active] > L)
            cand_cache[L] = int((unreached.any(axis=0) & indeg_nz).sum())
        return cand_cache[L]

    tot_bytes, tot_ms, tot_scan, n_main, n_scan, levels = 0, 0.0, 0.0, 0, 0, []
    for _ in range(reps):
        st = dobfs.make_stats(256)
        dobfs.bfs_batch(gb, srcs, depth, opt=ot, workspace=ws, stream=stream, stats=st)
        torch.cuda.synchronize()
        lv = dobfs.stats_levels(st)
        for L, x in enumerate(lv):
            if x["dir"] == dobfs.DIR_PUSH:
                b = 20 * x["nf"] + 12 * x["m_f"] + 12 * x["n_new"]
            else:
                b = 24 * hb.V + 24 * n_cand(L) + 12 * x["edges"]
            tot_bytes += b
            tot_ms += x["ms_main"]
            if x["dir"] == dobfs.DIR_PUSH:
                tot_scan += x["ms_aux"]
                n_scan += 1
            n_main += 1
        levels = [("push", "pull")[x["dir"]] for x in lv]
    gbps = tot_bytes / (tot_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "k_mb_step (push and pull steps)", "achieved": round(gbps, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4), "traffic": load_mb_traffic(levels),
            "algorithmic_bytes_per_launch": int(tot_bytes / n_main), "avg_launch_us": round(1e3 * tot_ms / n_main, 3),
            "launches": n_main, "levels": levels,
            "scan_step_avg_us": round(1e3 * tot_scan / max(1, n_scan), 3),
            "steps_per_launch": st.launches_main,
            "timing": "each kernel's own start/end events (hipExtLaunchKernel), %d launches of 64 sources" % reps}


def measure_batched(args, heur, alpha, beta):
    """Multi-source BFS: 64 sources per launch on RMAT-20 (edge factor 16), against the same 64
    queries run one after another through the single-source call on the same GPU. A query's
    latency is its launch's duration (all 64 are admitted together and finish together)."""
    import torch
    import gen
    import oracle
    from paper_1804_03327_amd import dobfs
    from paper_1804_03327_amd.helpers import BfsRunner, upload

    hb = gen.rmat(args.batched_scale, args.edgefactor, seed=1)
    srcs = [int(x) for x in gen.sample_sources(hb, 64, seed=5)]
    gb = upload(hb, device=0, hubs_first=not args.stored_order)
    stream = torch.cuda.current_stream()
    opt = dobfs.make_options("full", heur, alpha, beta)
    ws = torch.empty(dobfs.bfs_batch_workspace_bytes(gb, 64), dtype=torch.uint8, device="cuda")
    depth = torch.empty(64 * gb.V, dtype=torch.int32, device="cuda")
    for _ in range(2):
        dobfs.bfs_batch(gb, srcs, depth, opt=opt, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    lat = []
    t_all = time.perf_counter()
    for _ in range(args.batched_launches):
        t1 = time.perf_counter()
        dobfs.bfs_batch(gb, srcs, depth, opt=opt, workspace=ws, stream=stream)  # blocks until final
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t_all
    qps = 64 * args.batched_launches / t_all
    d = depth.cpu().numpy().reshape(64, gb.V)
    rows = iter(d)
    validate_sources(hb, srcs, lambda s: (next(rows), None))  # every row, depths only
    # the same queries one at a time through the single-source path: depths only (the output
    # the batched call gives), and with parents as well for reference
    qps_seq = {}
    for with_parent in (False, True):
        r = BfsRunner(gb, with_parent=with_parent)
        for s in srcs[:8]:
            r.run(s, opt=opt, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(2):
            for s in srcs:
                dobfs.bfs(gb, s, r.depth, r.parent, opt, r.ws, stream=stream)
        torch.cuda.synchronize()
        qps_seq[with_parent] = 2 * 64 / (time.perf_counter() - t1)
        del r
    lat_ms = np.array(lat) * 1e3
    # the same launches with the level loop as one persistent kernel per 64 steps
    op = dobfs.make_options("full", heur, alpha, beta, persistent=True)
    dobfs.bfs_batch(gb, srcs, depth, opt=op, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.batched_launches):
        dobfs.bfs_batch(gb, srcs, depth, opt=op, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    loop = {"step_launches_ms_per_launch": round(1e3 * t_all / args.batched_launches, 4),
            "persistent_ms_per_launch": round(1e3 * (time.perf_counter() - t1) / args.batched_launches, 4)}
    rows_p = depth.cpu().numpy().reshape(64, gb.V)
    assert np.array_equal(rows_p, d), "persistent multi-source rows differ from the step loop's"
    roof = batched_roofline(gb, hb, srcs, d, opt, ws, depth, stream, heur, alpha, beta)
    tuned = None
    if not args.no_autotune:
        from paper_1804_03327_amd import autotune
        pool = [int(x) for x in gen.sample_sources(hb, 160, seed=8)]
        tsrc = [x for x in pool if x not in set(srcs)][:64]
        rt = autotune.tune_batch(gb, tsrc, reps=3)
        ot = dobfs.make_options("full", rt["heuristic"], rt["alpha"], rt["beta"])
        dobfs.bfs_batch(gb, srcs, depth, opt=ot, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.batched_launches):
            dobfs.bfs_batch(gb, srcs, depth, opt=ot, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        tuned = {"rule": autotune.describe(rt),
                 "queries_per_s": round(64 * args.batched_launches / (time.perf_counter() - t1), 1)}
    res = {"workload": "rmat%d_ef%d, 64 sources per launch (seed 5)" % (args.batched_scale, args.edgefactor),
           "queries_per_s": round(qps, 1),
           "sequential_single_source_queries_per_s": round(qps_seq[False], 1),
           "speedup_vs_sequential": round(qps / qps_seq[False], 2),
           "sequential_with_parents_queries_per_s": round(qps_seq[True], 1),
           "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
           "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3),
           "launches": args.batched_launches, "rows_checked_against_oracle": 64,
           "level_loop": loop,
           "roofline": roof,
           "autotuned_direction_rule": tuned}
    log("batched:", json.dumps(res))
    del ws, depth
    return res


def measure_serving(args, hg22, g22, heur, alpha, beta):
    """The query server on four device-resident graphs (RMAT-16, RMAT-20, RMAT-22, a 2048x2048
    grid): single-source queries with a uniformly drawn graph and a source drawn from 64
    seeded degree > 0 vertices of it (seed 6) arrive as a Poisson stream at 0.5x .. 16x the
    sequential capacity. A point offers up to --serve-queries queries, fewer when they would
    take more than --serve-seconds of arrivals. Compared with the same arrival sequence served
    first-in first-out by plain single-source DOBFS, one query at a time, using each query's
    own measured service time (host gaps between queries ignored, which favours the baseline).
    Latency = arrival to depth final in device memory. Depth buffers are recycled once a query
    is answered; a submission that finds none free waits (counted as buffer stalls)."""
    import queue
    import threading
    import torch
    import gen
    from paper_1804_03327_amd import dobfs
    from paper_1804_03327_amd.helpers import BfsRunner, upload

    specs = [("rmat16", gen.rmat(16, args.edgefactor, seed=1)), ("rmat20", gen.rmat(20, args.edgefactor, seed=1)),
             ("rmat22", hg22), ("grid2048", gen.grid2d(2048, 2048))]
    gs = [g22 if h is hg22 else upload(h, device=0, hubs_first=not args.stored_order) for _, h in specs]
    opt = dobfs.make_options("full", heur, alpha, beta)
    rng = np.random.default_rng(6)
    npool = 64
    pools = [np.asarray(gen.sample_sources(h, npool, seed=7 + i)) for i, (_, h) in enumerate(specs)]
    # standalone service time of every (graph, source) a query can ask for (plain single-source
    # DOBFS, depths only: the output the server gives), the median of two runs
    svc_tab = np.zeros((len(specs), npool))
    for gi, g in enumerate(gs):
        r = BfsRunner(g, with_parent=False)
        r.run(int(pools[gi][0]), opt=opt)
        torch.cuda.synchronize()
        for j in range(npool):
            ts = []
            for _ in range(2):
                t1 = time.perf_counter()
                dobfs.bfs(g, int(pools[gi][j]), r.depth, r.parent, opt, r.ws)  # blocks until final
                ts.append(time.perf_counter() - t1)
            svc_tab[gi, j] = min(ts)
        del r
    cap = 1.0 / float(svc_tab.mean())  # uniform graph and source
    grid_loops = loop_costs(gs[3], [int(x) for x in pools[3][:2]], heur, alpha, beta, 1, torch.cuda.current_stream())
    log("grid level loops:", json.dumps(grid_loops))
    # device-side overlap: two grid traversals from two host threads on two streams, against the
    # same two one after the other (best of three each)
    ov_runners = [BfsRunner(gs[3], with_parent=False) for _ in range(2)]
    ov_streams = [torch.cuda.Stream() for _ in range(2)]
    ov_src = [int(pools[3][0]), int(pools[3][1])]

    def ov_one(i):
        ov_runners[i].run(ov_src[i], opt=opt, stream=ov_streams[i])

    ov_seq, ov_par = [], []
    for _ in range(3):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ov_one(0)
        ov_one(1)
        torch.cuda.synchronize()
        ov_seq.append(time.perf_counter() - t1)
        ths = [threading.Thread(target=ov_one, args=(i,)) for i in range(2)]
        t1 = time.perf_counter()
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        torch.cuda.synchronize()
        ov_par.append(time.perf_counter() - t1)
    overlap = {"two_grid_traversals_sequential_ms": round(1e3 * min(ov_seq), 2),
               "two_grid_traversals_two_streams_ms": round(1e3 * min(ov_par), 2)}
    log("two-stream overlap:", json.dumps(overlap))
    del ov_runners
    log("serving: sequential capacity %.1f q/s (mean service %s ms)" % (
        cap, ", ".join("%s %.3f" % (n, 1e3 * svc_tab[i].mean()) for i, (n, _) in enumerate(specs))))
    nbuf = [512, 512, 384, 384]
    bufs = [[torch.empty(g.V, dtype=torch.int32, device="cuda") for _ in range(nbuf[gi])] for gi, g in enumerate(gs)]
    free = [queue.SimpleQueue() for _ in gs]
    for gi in range(len(gs)):
        for b in range(nbuf[gi]):
            free[gi].put(b)
    points = []
    for mult in [float(x) for x in args.serve_points.split(",")]:
        lam = mult * cap
        N = int(min(args.serve_queries, max(64, round(lam * args.serve_seconds))))
        qg = rng.integers(0, len(specs), N)
        qj = rng.integers(0, npool, N)
        svc = svc_tab[qg, qj]
        arrivals = np.cumsum(rng.exponential(1.0 / lam, N))
        # FIFO, one query at a time (Lindley recursion on the measured service times)
        done, fifo_lat = 0.0, np.zeros(N)
        for i in range(N):
            start = max(arrivals[i], done)
            done = start + svc[i]
            fifo_lat[i] = done - arrivals[i]
        fifo_qps = N / (done - arrivals[0])
        srv = dobfs.Server(gs, slots=args.serve_slots, max_batch=64, opt=opt)
        ids = [None] * N
        bid = [None] * N
        infos = [None] * N
        todo = queue.SimpleQueue()
        stalls = [0]

        def waiter():
            while True:
                i = todo.get()
                if i is None:
                    return
                infos[i] = srv.wait(ids[i])
                free[int(qg[i])].put(bid[i])

        nw = 8
        ths = [threading.Thread(target=waiter) for _ in range(nw)]
        for th in ths:
            th.start()
        t_base = time.perf_counter()
        for i in range(N):
            delay = t_base + arrivals[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            gi = int(qg[i])
            try:
                b = free[gi].get_nowait()
            except queue.Empty:
                stalls[0] += 1
                b = free[gi].get()
            bid[i] = b
            ids[i] = srv.submit(gi, int(pools[gi][qj[i]]), bufs[gi][b])
            todo.put(i)
        for _ in ths:
            todo.put(None)
        for th in ths:
            th.join()
        srv.close()
        lat = np.array([x["t_done_ms"] - x["t_submit_ms"] for x in infos])
        t_first = min(x["t_submit_ms"] for x in infos)
        span = (max(x["t_done_ms"] for x in infos) - t_first) / 1e3
        sizes = np.array([x["batch_size"] for x in infos])
        points.append({"rate_x_sequential": mult, "queries": N, "offered_qps": round(lam, 1),
                       "served_qps": round(N / span, 1),
                       "p50_ms": round(float(np.percentile(lat, 50)), 2),
                       "p99_ms": round(float(np.percentile(lat, 99)), 2),
                       "p99_ms_by_graph": {name: round(float(np.percentile(lat[qg == gi], 99)), 2)
                                           for gi, (name, _) in enumerate(specs) if (qg == gi).any()},
                       "mean_batch": round(float(sizes.mean()), 2), "buffer_stalls": stalls[0],
                       "fifo_plain_dobfs": {"served_qps": round(fifo_qps, 1),
                                            "p50_ms": round(float(np.percentile(fifo_lat, 50)) * 1e3, 2),
                                            "p99_ms": round(float(np.percentile(fifo_lat, 99)) * 1e3, 2)}})
        log("serving %.1fx:" % mult, json.dumps(points[-1]))
    del bufs
    for g in gs:
        if g is not g22:
            dobfs.graph_destroy(g)
    peak = max(p["served_qps"] for p in points)
    return {"workload": "4 graphs (rmat16, rmat20, rmat22 ef%d; grid 2048x2048), uniform graph and "
                        "source (64 seeded sources per graph), Poisson arrivals (seed 6)" % args.edgefactor,
            "queries_per_point": "min(%d, %.0f s of arrivals)" % (args.serve_queries, args.serve_seconds),
            "slots": args.serve_slots, "max_batch": 64,
            "sequential_capacity_qps": round(cap, 1),
            "peak_served_qps": peak, "peak_served_x_sequential": round(peak / cap, 2),
            "mean_service_ms": {name: round(1e3 * float(svc_tab[gi].mean()), 3) for gi, (name, _) in enumerate(specs)},
            "grid2048_level_loop": dict(grid_loops, sources=2),
            "device_overlap": overlap,
            "points": points}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--cpu-sources", type=int, default=8, help="oracle sample size (0: skip)")
    ap.add_argument("--heuristic", choices=("ratio", "edges"), default="edges",
                    help="direction rule: Section 6.3 ratio form or the edge-count form")
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--stored-order", action="store_true",
                    help="upload the graph without reordering in-neighbours (DOBFS_UPLOAD_HUBS_FIRST off)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the multi-source (64 sources per launch) RMAT-20 measurement")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (rule and schedule settings tuned on 16 other sources, then timed on these)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the query-server measurement (4 graphs, Poisson arrivals)")
    ap.add_argument("--serve-queries", type=int, default=10000)
    ap.add_argument("--serve-seconds", type=float, default=6.0,
                    help="a serving point offers at most this many seconds of arrivals")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-lattice", action="store_true",
                    help="skip the 256^3 lattice (5%% of edges deleted, 16 sources) measurement")
    ap.add_argument("--lattice-n", type=int, default=256)
    ap.add_argument("--no-paper-scale", action="store_true",
                    help="skip the edge-factor-64 RMAT graph timed beside the paper's own figure for it")
    ap.add_argument("--batched-scale", type=int, default=20)
    ap.add_argument("--batched-launches", type=int, default=20)
    ap.add_argument("--no-validate", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many BFS steps (for rocprofv3), print nothing else")
    ap.add_argument("--profile-batched", type=int, default=0,
                    help="only run this many multi-source launches on the batched workload "
                         "(for rocprofv3), print nothing else")
    ap.add_argument("--profile-overlap", type=int, default=0,
                    help="only run N rounds of two 2048x2048 grid traversals from two host threads on two "
                         "streams (for a rocprofv3 kernel trace of their overlap on the device)")
    ap.add_argument("--profile-lattice", type=int, default=0,
                    help="only run the lattice's timed configuration from this many of its 16 sources "
                         "(for rocprofv3), print nothing else")
    ap.add_argument("--profile-serving", action="store_true",
                    help="only run the serving workload at --serve-points (for a rocprofv3 kernel trace)")
    ap.add_argument("--serve-points", default="0.5,1,2,4,8,16",
                    help="offered loads of the serving sweep, in multiples of the sequential capacity")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="with --profile-steps: also copy this many MiB device-to-device once, "
                         "the known-size reference for scaling PMC byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    from paper_1804_03327_amd import dobfs
    from paper_1804_03327_amd.helpers import BfsRunner, upload

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.profile_lattice:  # the configuration of the lattice's roofline pass
        hl = gen.lattice3d(args.lattice_n, 0.05, seed=3)
        srcs = [int(x) for x in gen.sample_sources(hl, 16, seed=4)][: args.profile_lattice]
        gl = upload(hl, device=0, hubs_first=not args.stored_order)
        r = BfsRunner(gl, with_parent=True)
        heur_l = dobfs.HEUR_EDGES if args.heuristic == "edges" else dobfs.HEUR_RATIO
        ol = dobfs.make_options("full", heur_l, args.alpha if args.alpha is not None else (
            1 / 14 if heur_l == dobfs.HEUR_EDGES else 0.01), args.beta if args.beta is not None else (
            1 / 24 if heur_l == dobfs.HEUR_EDGES else 0.01), time_kernels=True)
        for s in srcs:
            dobfs.bfs(gl, s, r.depth, r.parent, ol, r.ws, stats=dobfs.make_stats(4096))
            torch.cuda.synchronize()
            log("profile lattice source %d done" % s)
        return

    if args.profile_batched:
        hb = gen.rmat(args.batched_scale, args.edgefactor, seed=1)
        srcs = [int(x) for x in gen.sample_sources(hb, 64, seed=5)]
        gb = upload(hb, device=0, hubs_first=not args.stored_order)
        ws = torch.empty(dobfs.bfs_batch_workspace_bytes(gb, 64), dtype=torch.uint8, device="cuda")
        depth = torch.empty(64 * gb.V, dtype=torch.int32, device="cuda")
        heur_b = dobfs.HEUR_EDGES if args.heuristic == "edges" else dobfs.HEUR_RATIO
        ob = dobfs.make_options("full", heur_b, args.alpha if args.alpha is not None else (
            1 / 14 if heur_b == dobfs.HEUR_EDGES else 0.01), args.beta if args.beta is not None else (
            1 / 24 if heur_b == dobfs.HEUR_EDGES else 0.01))
        for k in range(args.profile_batched):
            dobfs.bfs_batch(gb, srcs, depth, opt=ob, workspace=ws)
            log("profile batched launch %d done" % k)
        return

    t0 = time.time()
    hg = gen.rmat(args.scale, args.edgefactor, seed=1)
    log("generated rmat%d ef%d: V=%d nnz=%d in %.1fs" % (args.scale, args.edgefactor, hg.V, hg.nnz,
                                                          time.time() - t0))
    sources = [int(s) for s in gen.sample_sources(hg, args.sources, seed=2)]
    # in-neighbours by decreasing out-degree (DOBFS_UPLOAD_HUBS_FIRST), arranged once at upload
    # like the CSR/CSC themselves and outside the timed region; --stored-order keeps the input order
    g = upload(hg, device=0, hubs_first=not args.stored_order)
    outdeg = hg.out_degree()
    indeg_nz = hg.in_degree() > 0
    runner = BfsRunner(g, with_parent=True)
    stream = torch.cuda.current_stream()
    heur = dobfs.HEUR_EDGES if args.heuristic == "edges" else dobfs.HEUR_RATIO
    alpha = args.alpha if args.alpha is not None else (1 / 14 if heur == dobfs.HEUR_EDGES else 0.01)
    beta = args.beta if args.beta is not None else (1 / 24 if heur == dobfs.HEUR_EDGES else 0.01)

    def options(mode, time_kernels=False):
        return dobfs.make_options(mode, heur, alpha, beta, time_kernels=time_kernels)

    if args.profile_overlap:
        import threading
        hgr = gen.grid2d(2048, 2048)
        gr = upload(hgr, device=0)
        pool = [int(x) for x in gen.sample_sources(hgr, 2, seed=7)]
        runners = [BfsRunner(gr, with_parent=False) for _ in range(2)]
        streams = [torch.cuda.Stream() for _ in range(2)]
        for i in range(2):
            runners[i].run(pool[i], opt=options("full"), stream=streams[i])
        torch.cuda.synchronize()
        for k in range(args.profile_overlap):
            ths = [threading.Thread(target=runners[i].run, args=(pool[i],),
                                    kwargs=dict(opt=options("full"), stream=streams[i])) for i in range(2)]
            for th in ths:
                th.start()
            for th in ths:
                th.join()
            torch.cuda.synchronize()
            log("profile overlap round %d done" % k)
        return

    if args.profile_serving:
        res = measure_serving(args, hg, g, heur, alpha, beta)
        log("profile serving:", json.dumps(res["points"]))
        return

    opt_plain = options("full")
    opt_timed = options("full", time_kernels=True)

    if args.profile_steps:
        if args.copy_mb:
            # counter calibration, each stream larger than the 256 MB Infinity Cache: a write-only
            # fill, a read-only reduction (its output is a few bytes), and a copy
            n = args.copy_mb << 20
            src_t = torch.empty(n // 4, dtype=torch.int32, device="cuda")
            src_t.fill_(1)
            torch.cuda.synchronize()
            log("calibration fill (write only) of %d bytes done" % n)
            tot = int(src_t.sum())
            torch.cuda.synchronize()
            log("calibration sum (read only) of %d bytes done (%d)" % (n, tot))
            dst_t = torch.empty_like(src_t)
            dst_t.copy_(src_t)
            torch.cuda.synchronize()
            log("calibration copy of %d bytes done" % n)
            del src_t, dst_t
        for k in range(args.profile_steps):  # the configuration of the roofline pass
            for s in sources:
                runner.run(s, opt=opt_timed, stream=stream)
            torch.cuda.synchronize()
            log("profile step %d done" % k)
        return

    # warm-up; the first pass checks every source's result against the oracle (depths exact,
    # parents valid) and takes the per-source edge counts and pull candidate tables from the
    # oracle's depths
    import oracle
    edges_g500, cand_tables, validated = {}, {}, None
    for w in range(max(1, args.warmup)):
        if w == 0 and not args.no_validate:
            def run_one(s):
                runner.run(s, opt=opt_plain, stream=stream)
                return runner.result()

            res = validate_sources(hg, sources, run_one)
            for s, want in res.items():
                edges_g500[s] = oracle.teps_edges(hg, want)["graph500"]
                cand_tables[s] = candidates_per_level(want, indeg_nz)
            validated = {"sources": len(res), "depth_exact_and_parents_valid": True,
                         "edge_counts": "oracle (Graph500 count)"}
            log("validated %d sources against the oracle" % len(res))
            continue
        for s in sources:
            runner.run(s, opt=opt_plain, stream=stream)
    if not edges_g500:  # --no-validate: counts from the GPU's depths (reported as such)
        for s in sources:
            runner.run(s, opt=opt_plain, stream=stream)
            d = runner.depth.cpu().numpy()
            edges_g500[s] = int(outdeg[d >= 0].sum()) // 2
            cand_tables[s] = candidates_per_level(d, indeg_nz)
    torch.cuda.synchronize()
    log("warm-up done")

    # timed region: K steps x 64 sources, nothing but the BFS calls
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        for s in sources:
            dobfs.bfs(g, s, runner.depth, runner.parent, opt_plain, runner.ws, stream=stream)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    total_edges = sum(edges_g500[s] for s in sources) * args.steps
    gteps = total_edges / t_total / 1e9
    gteps_paper = hg.nnz * len(sources) * args.steps / t_total / 1e9
    log("timed: %.3f ms/step, %.2f GTEPS (graph500 count), %.2f GTEPS (nnz/time)" % (
        ms_per_step, gteps, gteps_paper))

    # roofline pass: the same K steps again, every kernel launched with start
    # and end events of its own execution (by the library, on this stream);
    # per-kernel durations and algorithmic bytes come from here
    caps = 64
    pool = [[dobfs.make_stats(caps) for _ in sources] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_ev = time.perf_counter()
    for k in range(args.steps):
        row = pool[k]
        for i, s in enumerate(sources):
            dobfs.bfs(g, s, runner.depth, runner.parent, opt_timed, runner.ws, stream=stream,
                      stats=row[i])
    torch.cuda.synchronize()
    t_ev = time.perf_counter() - t_ev

    runs = [(s, pool[k][i]) for k in range(args.steps) for i, s in enumerate(sources)]
    roofline, kernel_table, bfs_ms = step_roofline(hg.V, heur, runs, cand_tables,
                                                   load_traffic("step"))
    roofline["timing"] = ("each kernel's own start/end events (hipExtLaunchKernel) on the BFS stream, "
                          "over a repeat of the timed steps (%.1f ms/step with events)" % (1e3 * t_ev / args.steps))
    log("kernels:", json.dumps(kernel_table))

    # the two forms of the level loop on the same graph (NEXT-2 A/B)
    level_loop = dict(loop_costs(g, sources[:16], heur, alpha, beta, 2, stream), sources=16)
    log("level loops:", json.dumps(level_loop))

    # the library's own Graph500 edge counts (stats) against the oracle's
    if validated is not None:
        bad = [s for i, s in enumerate(sources) if pool[0][i].edges_g500 != edges_g500[s]]
        if bad:
            raise SystemExit("bench: library edge count differs from the oracle's on sources %s" % bad[:4])
        validated["library_edge_counts_match"] = True

    # CPU baseline: the oracle as it stands, single thread, on a bounded sample of sources
    cpu = None
    if args.cpu_sources > 0:
        sample = sources[: args.cpu_sources]
        tc, ec = 0.0, 0
        for s in sample:
            t1 = time.perf_counter()
            oracle.bfs(hg, s)
            tc += time.perf_counter() - t1
            ec += edges_g500[s]
        cpu = {"value": round(ec / tc / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "FIFO-queue BFS from the first %d of the 64 sources on the same RMAT-22 "
                         "graph (%.1f s), Graph500 edge count; host %s, %d cpus visible" % (
                             len(sample), tc, platform.processor() or platform.machine(),
                             os.cpu_count() or 0)}
        log("cpu oracle: %.4f GTEPS over %d sources (%.1fs)" % (cpu["value"], len(sample), tc))

    # Table 2 factoring: each mode once over all sources
    ablation = None
    if not args.no_ablation:
        ablation = {}
        # Table 2's rows in order: the sort-based push (Baseline: key-value sort), the
        # structure-only push (key-only sort, no parents), then the atomic push, direction
        # change, masking, early exit and operand reuse added one at a time
        for mode in ("push_sort", "push_sort_keys", "push_only", "pull_unmasked", "pull_masked",
                     "pull_masked_ee", "full"):
            o = options(mode)
            sort = mode.startswith("push_sort")
            ws_m = None if sort else runner.ws  # the sort needs its larger workspace
            par = None if mode == "push_sort_keys" else runner.parent

            def one(s):
                dobfs.bfs(g, s, runner.depth, par, o, ws_m, stream=stream)

            for s in sources[:4]:
                one(s)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for s in sources:
                one(s)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            ablation[mode] = round(sum(edges_g500[s] for s in sources) / dt / 1e9, 3)
        log("ablation GTEPS:", json.dumps(ablation))

    # the same traversals on the graph in its stored in-neighbour order, for comparison
    stored = None
    if not args.stored_order and not args.no_ablation:
        g_st = upload(hg, device=0)
        for s in sources[:4]:
            dobfs.bfs(g_st, s, runner.depth, runner.parent, opt_plain, runner.ws, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(3):
            for s in sources:
                dobfs.bfs(g_st, s, runner.depth, runner.parent, opt_plain, runner.ws, stream=stream)
        torch.cuda.synchronize()
        stored = round(sum(edges_g500[s] for s in sources) / ((time.perf_counter() - t1) / 3) / 1e9, 3)
        dobfs.graph_destroy(g_st)
        log("stored in-neighbour order: %.2f GTEPS" % stored)

    # the other direction rule on the same workload, for comparison
    other = None
    if not args.no_ablation:
        oh = dobfs.HEUR_RATIO if heur == dobfs.HEUR_EDGES else dobfs.HEUR_EDGES
        oo = dobfs.make_options("full", oh, 0.01 if oh == dobfs.HEUR_RATIO else 1 / 14,
                                0.01 if oh == dobfs.HEUR_RATIO else 1 / 24)
        for s in sources[:4]:
            runner.run(s, opt=oo, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for s in sources:
            runner.run(s, opt=oo, stream=stream)
        torch.cuda.synchronize()
        other = {"heuristic": "ratio alpha=beta=0.01" if oh == dobfs.HEUR_RATIO else
                 "edges alpha=1/14 beta=1/24",
                 "gteps": round(sum(edges_g500[s] for s in sources) / (time.perf_counter() - t1) / 1e9, 3)}
        log("other rule:", json.dumps(other))

    # the autotuner picks the rule and the schedule settings on 16 sources not among the 64;
    # then the 64 are timed with the tuned and the fixed settings in alternation (5 passes
    # each), so the gain can be set against the spread of the passes
    autotuned = None
    if not args.no_autotune:
        from paper_1804_03327_amd import autotune
        pool = [int(x) for x in gen.sample_sources(hg, 96, seed=3)]
        tune_src = [x for x in pool if x not in set(sources)][:16]
        res = autotune.tune_schedule(g, tune_src, reps=3)
        ot = dobfs.make_options("full", res["heuristic"], res["alpha"], res["beta"], sched=res["sched"])
        for s in sources[:4]:
            runner.run(s, opt=ot, stream=stream)
        torch.cuda.synchronize()
        passes = {"tuned": [], "fixed": []}
        for k in range(5):
            for name, o in (("fixed", opt_plain), ("tuned", ot)):
                t1 = time.perf_counter()
                for s in sources:
                    dobfs.bfs(g, s, runner.depth, runner.parent, o, runner.ws, stream=stream)
                torch.cuda.synchronize()
                passes[name].append(time.perf_counter() - t1)
        e64 = sum(edges_g500[s] for s in sources)
        gt = {k: [e64 / x / 1e9 for x in v] for k, v in passes.items()}

        def ms(xs):
            return round(1e3 * float(np.mean(xs)) / len(sources), 4)

        def sem(xs):
            return float(np.std(xs, ddof=1) / np.sqrt(len(xs)))

        gain = float(np.mean(gt["tuned"]) - np.mean(gt["fixed"]))
        band = 2.0 * float(np.hypot(sem(gt["tuned"]), sem(gt["fixed"])))
        autotuned = {"settings": autotune.describe(res),
                     "gteps": round(float(np.mean(gt["tuned"])), 3),
                     "gteps_fixed_same_passes": round(float(np.mean(gt["fixed"])), 3),
                     "ms_per_bfs": ms(passes["tuned"]), "ms_per_bfs_fixed": ms(passes["fixed"]),
                     "gain_gteps": round(gain, 3), "noise_band_gteps": round(band, 3),
                     "gain_beyond_noise": bool(gain > band),
                     "passes": 5, "tuning_sources": len(tune_src), "tuning_reps": 3,
                     "tuning_ms_per_bfs": round(res["ms"], 4),
                     "tuning_ms_per_bfs_default_schedule": round(res["default_ms"], 4),
                     "schedule_steps": res["steps"]}
        log("autotuned:", json.dumps(autotuned))

    lattice = None
    if not args.no_lattice:
        lattice = measure_lattice(args, heur, alpha, beta)

    paper_scale = None
    if not args.no_paper_scale:
        paper_scale = measure_paper_scale(args, heur, alpha, beta)

    batched = None
    if not args.no_batched:
        batched = measure_batched(args, heur, alpha, beta)

    serving = None
    if not args.no_serving:
        serving = measure_serving(args, hg, g, heur, alpha, beta)

    out = {
        "metric": METRIC, "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "rmat%d_ef%d" % (args.scale, args.edgefactor), "vertices": hg.V,
                   "directed_edges": hg.nnz, "sources_per_step": len(sources), "mode": "full",
                   "heuristic": "%s alpha=%.4g beta=%.4g" % (args.heuristic, alpha, beta),
                   "teps_edges": "graph500",
                   "csc_order": "stored" if args.stored_order else "hubs_first",
                   "rmat_abcd": [0.57, 0.19, 0.19, 0.05], "graph_seed": 1, "source_seed": 2},
        "gteps_paper_convention": round(gteps_paper, 3),
        # whole-call device time from the roofline pass, whose every kernel carries start/end
        # events (slower than the timed steps; ms_per_step / sources_per_step is the BFS time)
        "bfs_ms_median_with_kernel_events": round(float(np.median(bfs_ms)), 4),
        "roofline": roofline,
        "kernels": kernel_table,
        "cpu_baseline": cpu,
        "level_loop": level_loop,
        "ablation_gteps": ablation,
        "stored_order_gteps": stored,
        "other_direction_rule": other,
        "autotuned": autotuned,
        "validated": validated,
        "lattice": lattice,
        "paper_scale": paper_scale,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
