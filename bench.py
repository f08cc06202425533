"""Benchmark: single-source direction-optimized BFS on RMAT scale 22 (edge factor 16) on one
MI355X, through the C ABI.

A step is one BFS from each of the 64 seeded sources (vertices with degree > 0). The metric
is GTEPS with the Graph500 edge count (undirected edges with a reached endpoint); the
paper-convention figure (nnz(A) / time) is reported beside it. Prints one JSON line.

Also reported: the HBM roofline of the dominant kernel (algorithmic bytes per launch over its
HIP-event-timed duration inside the timed region), the CPU oracle on a bounded sample of the
same workload, and the Table 2 ablation modes.
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
METRIC = "GTEPS DOBFS RMAT-22 (1 GPU)"
KERNEL_SRC = os.path.join(ROOT, "paper_1804_03327_amd", "csrc", "kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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


def bytes_init(V):
    return 8 * V + V / 8


def candidates_per_level(depth, indeg_nz):
    """Rows a level-L pull lists: in-degree > 0 and not visited at level start (depth <= L)."""
    d = depth[indeg_nz]
    reached = d[d >= 0]
    cnt = np.bincount(reached) if reached.size else np.zeros(1, dtype=np.int64)
    total = int(indeg_nz.sum())
    return total - np.cumsum(cnt)  # index L -> candidates at level L


def load_traffic(kernel: str):
    """HBM traffic per launch from committed rocprofv3 PMC summaries, or None when absent or
    taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_rmat22.json" % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--cpu-sources", type=int, default=8, help="oracle sample size (0: skip)")
    ap.add_argument("--heuristic", choices=("ratio", "edges"), default="ratio",
                    help="direction rule: Section 6.3 ratio form or the edge-count form")
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--beta", type=float, default=None)
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-validate", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many BFS steps (for rocprofv3), print nothing else")
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

    t0 = time.time()
    hg = gen.rmat(args.scale, args.edgefactor, seed=1)
    log("generated rmat%d ef%d: V=%d nnz=%d in %.1fs" % (args.scale, args.edgefactor, hg.V, hg.nnz,
                                                          time.time() - t0))
    sources = [int(s) for s in gen.sample_sources(hg, args.sources, seed=2)]
    g = upload(hg, device=0)
    outdeg = hg.out_degree()
    indeg_nz = hg.in_degree() > 0
    runner = BfsRunner(g, with_parent=True)
    stream = torch.cuda.current_stream()
    heur = dobfs.HEUR_EDGES if args.heuristic == "edges" else dobfs.HEUR_RATIO
    alpha = args.alpha if args.alpha is not None else (1 / 14 if heur == dobfs.HEUR_EDGES else 0.01)
    beta = args.beta if args.beta is not None else (1 / 24 if heur == dobfs.HEUR_EDGES else 0.01)

    def options(mode, time_kernels=False):
        return dobfs.make_options(mode, heur, alpha, beta, time_kernels=time_kernels)

    opt_plain = options("full")
    opt_timed = options("full", time_kernels=True)

    if args.profile_steps:
        if args.copy_mb:
            n = args.copy_mb << 20
            src_t = torch.ones(n, dtype=torch.uint8, device="cuda")
            dst_t = torch.empty_like(src_t)
            torch.cuda.synchronize()
            dst_t.copy_(src_t)
            torch.cuda.synchronize()
            log("reference copy of %d bytes done" % n)
            del src_t, dst_t
        for k in range(args.profile_steps):
            for s in sources:
                runner.run(s, opt=opt_plain, stream=stream)
            torch.cuda.synchronize()
            log("profile step %d done" % k)
        return

    # warm-up, and per-source edge counts / candidate tables from the GPU's own depths
    edges_g500, cand_tables = {}, {}
    for w in range(max(1, args.warmup)):
        for s in sources:
            runner.run(s, opt=opt_plain, stream=stream)
            if w == 0:
                d = runner.depth.cpu().numpy()
                edges_g500[s] = int(outdeg[d >= 0].sum()) // 2
                cand_tables[s] = candidates_per_level(d, indeg_nz)
    torch.cuda.synchronize()
    log("warm-up done")

    # timed region: K steps x 64 sources, per-kernel HIP events recorded by the library
    caps = 64
    pool = [[dobfs.make_stats(caps) for _ in sources] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        row = pool[k]
        for i, s in enumerate(sources):
            dobfs.bfs(g, s, runner.depth, runner.parent, opt_timed, runner.ws, stream=stream,
                      stats=row[i])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    total_edges = sum(edges_g500[s] for s in sources) * args.steps
    gteps = total_edges / t_total / 1e9
    gteps_paper = hg.nnz * len(sources) * args.steps / t_total / 1e9
    log("timed: %.3f ms/step, %.2f GTEPS (graph500 count), %.2f GTEPS (nnz/time)" % (
        ms_per_step, gteps, gteps_paper))

    # per-kernel times and algorithmic bytes over the timed region
    kinds = {k: {"ms": 0.0, "launches": 0, "bytes": 0.0} for k in
             ("push_scan", "push_expand", "pull", "init")}
    bfs_ms = []
    for k in range(args.steps):
        for i, s in enumerate(sources):
            st = pool[k][i]
            if st.levels > st.cap:
                raise RuntimeError("level stats truncated: %d levels > cap %d" % (st.levels, st.cap))
            bfs_ms.append(st.ms_total)
            kinds["init"]["ms"] += st.ms_init
            kinds["init"]["launches"] += 1
            kinds["init"]["bytes"] += bytes_init(hg.V)
            prev = dobfs.DIR_PUSH
            for L, lv in enumerate(dobfs.stats_levels(st)):
                if lv["dir"] == dobfs.DIR_PUSH:
                    kinds["push_expand"]["ms"] += lv["ms_main"]
                    kinds["push_expand"]["launches"] += 1
                    kinds["push_expand"]["bytes"] += bytes_push_expand(lv["nf"], lv["m_f"], lv["n_new"])
                    kinds["push_scan"]["ms"] += lv["ms_aux"]  # includes a pull->push conversion
                    kinds["push_scan"]["launches"] += 1
                    kinds["push_scan"]["bytes"] += bytes_push_scan(lv["nf"]) + (
                        bytes_d2s(hg.V, lv["nf"]) if (prev == dobfs.DIR_PULL) else 0)
                else:
                    nc = cand_tables[s][L] if L < len(cand_tables[s]) else cand_tables[s][-1]
                    kinds["pull"]["ms"] += lv["ms_main"]
                    kinds["pull"]["launches"] += 1
                    kinds["pull"]["bytes"] += bytes_pull(hg.V, int(nc), lv["edges"], lv["n_new"])
                prev = lv["dir"]
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    kd = kinds[dom]
    avg_ms = kd["ms"] / max(1, kd["launches"])
    per_launch = kd["bytes"] / max(1, kd["launches"])
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = load_traffic(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": round(per_launch), "avg_launch_us": round(avg_ms * 1e3, 3),
                "launches": kd["launches"]}
    kernel_table = {k: {"total_ms": round(v["ms"], 3), "launches": v["launches"],
                        "avg_us": round(1e3 * v["ms"] / max(1, v["launches"]), 3),
                        "GBps": round(v["bytes"] / max(1e-12, v["ms"] * 1e-3) / 1e9, 1)}
                    for k, v in kinds.items()}
    log("kernels:", json.dumps(kernel_table))

    # parity spot-check of the benchmarked configuration against the oracle
    import oracle
    validated = None
    if not args.no_validate:
        s = sources[0]
        runner.run(s, opt=opt_plain, stream=stream)
        d, p = runner.result()
        want, _ = oracle.bfs(hg, s)
        ok = bool(np.array_equal(d, want)) and oracle.validate(hg, s, d, p)[0] == 0
        validated = {"source": s, "depth_exact_and_parents_valid": ok}
        if not ok:
            raise SystemExit("bench: GPU result differs from the oracle on source %d" % s)
        log("validated source %d against the oracle" % s)

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
        for mode in ("push_only", "pull_unmasked", "pull_masked", "pull_masked_ee", "full"):
            o = options(mode)
            for s in sources[:4]:
                runner.run(s, opt=o, stream=stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for s in sources:
                runner.run(s, opt=o, stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            ablation[mode] = round(sum(edges_g500[s] for s in sources) / dt / 1e9, 3)
        log("ablation GTEPS:", json.dumps(ablation))

    out = {
        "metric": METRIC, "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "rmat%d_ef%d" % (args.scale, args.edgefactor), "vertices": hg.V,
                   "directed_edges": hg.nnz, "sources_per_step": len(sources), "mode": "full",
                   "heuristic": "%s alpha=%.4g beta=%.4g" % (args.heuristic, alpha, beta),
                   "teps_edges": "graph500",
                   "rmat_abcd": [0.57, 0.19, 0.19, 0.05], "graph_seed": 1, "source_seed": 2},
        "gteps_paper_convention": round(gteps_paper, 3),
        "bfs_ms_median": round(float(np.median(bfs_ms)), 4),
        "roofline": roofline,
        "kernels": kernel_table,
        "cpu_baseline": cpu,
        "ablation_gteps": ablation,
        "validated": validated,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
