"""GPU parity at the full sizes of the benchmarked and configured workloads, in the launch
configuration the benchmark times (in-neighbours uploaded hubs-first, edge-count rule with
alpha = 1/14, beta = 1/24, caller-owned workspace, current stream).

Every depth vector is compared with the oracle's over all vertices and every parent vector
passes the validator; under the edge-count rule the direction sequence is the oracle's. The
benchmark's 64 RMAT-22 sources are all checked in the benchmarked mode, every Table 2 mode the
benchmark times is checked on two of them, two sources of the edge-factor-64 RMAT-22 graph run
under both rules, one source of RMAT-24 with edge factor 64 (just under 2^31 entries), four of
the lattice's 16 sources run in three modes, and every row of the 64-source RMAT-20 launch is
checked."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1804_03327_amd import dobfs  # noqa: E402
from paper_1804_03327_amd.helpers import BfsRunner, upload  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


BENCH_OPT = dict(mode="full", heuristic=dobfs.HEUR_EDGES, alpha=1 / 14, beta=1 / 24)
# the Table 2 rows the benchmark times, each with the benchmark's direction rule
ABLATION_MODES = ("push_sort", "push_sort_keys", "push_only", "pull_unmasked", "pull_masked", "pull_masked_ee",
                  "full")


def _oracle_many(hg, sources):
    """Oracle depths of many sources at once (the C oracle runs outside the GIL)."""
    with ThreadPoolExecutor(8) as ex:
        return dict(zip(sources, ex.map(lambda s: oracle.bfs(hg, s)[0], sources)))


def _check(hg, s, want, d, p, tag, opt=None, levels=None):
    bad = int((d != want).sum())
    assert bad == 0, "%s: %d depths differ" % (tag, bad)
    code, at = oracle.validate(hg, s, d, p)
    assert code == 0, "%s: parent check %d failed at %d" % (tag, code, at)
    if opt is not None and opt.get("heuristic") == dobfs.HEUR_EDGES and levels is not None:
        dirs = [x["dir"] for x in levels]
        assert dirs == oracle.schedule_edges(hg, want, opt["alpha"], opt["beta"]), tag


@pytest.fixture(scope="module")
def rmat22():
    hg = gen.rmat(22, 16, seed=1)
    srcs = [int(x) for x in gen.sample_sources(hg, 64, seed=2)]
    _say("rmat22 generated: V=%d nnz=%d" % (hg.V, hg.nnz))
    return hg, srcs


def test_rmat22_all_bench_sources(rmat22):
    """The 64 benchmark sources in the benchmarked configuration, and the library's Graph500
    edge count of each against the oracle's."""
    hg, srcs = rmat22
    g = upload(hg, hubs_first=True)
    r = BfsRunner(g)
    want = _oracle_many(hg, srcs)
    for k, s in enumerate(srcs):
        st = r.run(s, **BENCH_OPT)
        d, p = r.result()
        tag = "rmat22 bench source #%d (%d)" % (k, s)
        if k % 8 == 0:
            _say(tag)
        _check(hg, s, want[s], d, p, tag, BENCH_OPT, r.levels())
        assert st.edges_g500 == oracle.teps_edges(hg, want[s])["graph500"], tag
    dobfs.graph_destroy(g)


def test_rmat22_ablation_modes(rmat22):
    """Every Table 2 mode the benchmark times, on two of its sources, with its upload and rule."""
    hg, srcs = rmat22
    g = upload(hg, hubs_first=True)
    r = BfsRunner(g)
    pick = [srcs[0], srcs[37]]
    want = _oracle_many(hg, pick)
    for s in pick:
        for mode in ABLATION_MODES:
            tag = "rmat22 source %d mode %s" % (s, mode)
            _say(tag)
            opt = dobfs.make_options(mode, BENCH_OPT["heuristic"], BENCH_OPT["alpha"], BENCH_OPT["beta"])
            # the sort-based push needs its larger workspace: the library's own, as the bench runs it
            ws = None if mode.startswith("push_sort") else r.ws
            if mode == "push_sort_keys":  # depths only
                dobfs.bfs(g, s, r.depth, None, opt, ws, stats=r.stats)
                d = r.depth.cpu().numpy()
                assert np.array_equal(d, want[s]), tag
                continue
            dobfs.bfs(g, s, r.depth, r.parent, opt, ws, stats=r.stats)
            d, p = r.result()
            _check(hg, s, want[s], d, p, tag)
    # the paper's ratio rule in the stored order as well
    g2 = upload(hg)
    r2 = BfsRunner(g2)
    r2.run(pick[1], mode="full")
    d, p = r2.result()
    _check(hg, pick[1], want[pick[1]], d, p, "rmat22 stored order, ratio rule")
    dobfs.graph_destroy(g)
    dobfs.graph_destroy(g2)


def test_rmat22_ef64_paper_scale():
    """The paper's own scale-22 RMAT graph (edge factor 64; 483M directed edges in its Table 3),
    which the benchmark times beside the paper's figure: two of its 16 sources in the
    benchmarked configuration and under the ratio rule (alpha = beta = 0.01), with the
    library's Graph500 edge counts."""
    hg = gen.rmat(22, 64, seed=1)
    _say("rmat22 ef64 generated: V=%d nnz=%d" % (hg.V, hg.nnz))
    assert abs(hg.nnz - 483e6) < 0.01 * 483e6
    srcs = [int(x) for x in gen.sample_sources(hg, 16, seed=2)]
    pick = [srcs[0], srcs[9]]
    want = _oracle_many(hg, pick)
    g = upload(hg, hubs_first=True)
    r = BfsRunner(g)
    for s in pick:
        for o in (BENCH_OPT, dict(mode="full")):
            tag = "rmat22 ef64 source %d %s" % (s, o)
            _say(tag)
            st = r.run(s, **o)
            d, p = r.result()
            _check(hg, s, want[s], d, p, tag, o, r.levels())
            assert st.edges_g500 == oracle.teps_edges(hg, want[s])["graph500"], tag
    dobfs.graph_destroy(g)


def test_rmat24_ef64_near_the_int32_edge_limit():
    """The largest graph the int32 CSR/CSC boundary admits in practice: RMAT scale 24 with edge
    factor 64, just under 2^31 directed entries. One source in the benchmarked configuration:
    depths exact, parents valid, the library's Graph500 edge count equal to the oracle's."""
    hg = gen.rmat(24, 64, seed=1)
    _say("rmat24 ef64 generated: V=%d nnz=%d" % (hg.V, hg.nnz))
    assert 0.9 * 2**31 < hg.nnz < 2**31
    s = int(gen.sample_sources(hg, 1, seed=2)[0])
    g = upload(hg, hubs_first=True)
    r = BfsRunner(g)
    st = r.run(s, **BENCH_OPT)
    d, p = r.result()
    dobfs.graph_destroy(g)
    del r
    want, _ = oracle.bfs(hg, s)
    _check(hg, s, want, d, p, "rmat24 ef64 source %d" % s)
    assert st.edges_g500 == oracle.teps_edges(hg, want)["graph500"]


def test_lattice256_sources():
    """Four of the 16 lattice sources in the full, push-only and benchmarked configurations."""
    hg = gen.lattice3d(256, 0.05, seed=3)
    assert hg.nnz == 95_256_576
    srcs = [int(x) for x in gen.sample_sources(hg, 16, seed=4)]
    pick = [srcs[0], srcs[5], srcs[10], srcs[15]]
    want = _oracle_many(hg, pick)
    g = upload(hg, hubs_first=True)
    r = BfsRunner(g)
    for s in pick:
        for o in (dict(mode="full"), dict(mode="push_only"), BENCH_OPT):
            tag = "lattice256 source %d %s" % (s, o)
            _say(tag)
            r.run(s, **o)
            d, p = r.result()
            _check(hg, s, want[s], d, p, tag, o, r.levels())
    dobfs.graph_destroy(g)


def test_grid2048_single_source():
    hg = gen.grid2d(2048, 2048)
    assert hg.nnz == 16_769_024
    g = upload(hg)
    r = BfsRunner(g)
    want, _ = oracle.bfs(hg, 0)
    r.run(0, mode="full")
    d, p = r.result()
    _check(hg, 0, want, d, p, "grid2048 source 0")
    dobfs.graph_destroy(g)


def test_rmat20_multi_source_all_rows():
    """Every row of the benchmark's 64-source RMAT-20 launch, in its configuration."""
    hg = gen.rmat(20, 16, seed=1)
    srcs = [int(x) for x in gen.sample_sources(hg, 64, seed=5)]
    g = upload(hg, hubs_first=True)
    depth = torch.full((64 * g.V,), -7, dtype=torch.int32, device="cuda")
    dobfs.bfs_batch(g, srcs, depth, opt=dobfs.make_options(**BENCH_OPT))
    rows = depth.cpu().numpy().reshape(64, g.V)
    want = _oracle_many(hg, srcs)
    for b in range(64):
        assert np.array_equal(rows[b], want[srcs[b]]), "row %d (source %d) differs" % (b, srcs[b])
    _say("rmat20: 64 rows match")
    dobfs.graph_destroy(g)


def test_multi_source_large_graphs(rmat22):
    """Multi-source launches on graphs with more pull tiles than the step launch has blocks
    (8192): 64 RMAT-22 bench sources, every row; and 8 sources on the 2048^2 grid, whose 4095
    push levels run over many batches, the later ones on the smaller grid the host sizes from
    the pushes before (twice: the second call starts from the first call's step count)."""
    hg, srcs = rmat22
    g = upload(hg, hubs_first=True)
    depth = torch.full((64 * g.V,), -7, dtype=torch.int32, device="cuda")
    dobfs.bfs_batch(g, srcs, depth, opt=dobfs.make_options(**BENCH_OPT))
    rows = depth.cpu().numpy().reshape(64, g.V)
    want = _oracle_many(hg, srcs)
    for b in range(64):
        assert np.array_equal(rows[b], want[srcs[b]]), "rmat22 row %d (source %d) differs" % (b, srcs[b])
    _say("rmat22: 64 rows match")
    dobfs.graph_destroy(g)
    del depth
    hgr = gen.grid2d(2048, 2048)
    g = upload(hgr, hubs_first=True)
    gs = [0, hgr.V - 1] + [int(x) for x in gen.sample_sources(hgr, 6, seed=9)]
    want = _oracle_many(hgr, gs)
    for call in range(2):
        depth = torch.full((8 * g.V,), -7, dtype=torch.int32, device="cuda")
        st = dobfs.make_stats(8192)
        dobfs.bfs_batch(g, gs, depth, opt=dobfs.make_options(**BENCH_OPT), stats=st)
        rows = depth.cpu().numpy().reshape(8, g.V)
        for b in range(8):
            assert np.array_equal(rows[b], want[gs[b]]), "grid2048 call %d row %d differs" % (call, b)
        assert st.levels == max(int(w.max()) for w in want.values()) + 1
        _say("grid2048 call %d: 8 rows match over %d levels" % (call, st.levels))
    dobfs.graph_destroy(g)


def test_full_size_persistent_loop(rmat22):
    """The persistent level loop at full size: four RMAT-22 bench sources and two lattice
    sources in the benchmarked configuration, against the oracle and the step-launch loop's
    per-level sizes and directions."""
    hg, srcs = rmat22
    g = upload(hg, hubs_first=True)
    r = BfsRunner(g)
    pick = [srcs[0], srcs[13], srcs[29], srcs[51]]
    want = _oracle_many(hg, pick)
    for s in pick:
        tag = "rmat22 persistent source %d" % s
        _say(tag)
        r.run(s, **BENCH_OPT)
        ref = [(x["dir"], x["nf"], x["n_new"]) for x in r.levels()]
        r.run(s, persistent=True, **BENCH_OPT)
        d, p = r.result()
        _check(hg, s, want[s], d, p, tag, BENCH_OPT, r.levels())
        assert [(x["dir"], x["nf"], x["n_new"]) for x in r.levels()] == ref, tag
    dobfs.graph_destroy(g)
    hl = gen.lattice3d(256, 0.05, seed=3)
    lsrc = [int(x) for x in gen.sample_sources(hl, 16, seed=4)]
    pick = [lsrc[3], lsrc[12]]
    want = _oracle_many(hl, pick)
    g = upload(hl, hubs_first=True)
    r = BfsRunner(g)
    for s in pick:
        tag = "lattice256 persistent source %d" % s
        _say(tag)
        r.run(s, persistent=True, **BENCH_OPT)
        d, p = r.result()
        _check(hl, s, want[s], d, p, tag, BENCH_OPT, r.levels())
    dobfs.graph_destroy(g)
