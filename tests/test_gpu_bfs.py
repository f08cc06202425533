"""GPU parity of dobfs_bfs against the CPU oracle, through the C ABI.

Depths must equal the oracle's bit for bit (they are unique); parents must pass the
Graph500-style validator, and on pull levels equal the first in-neighbour one level up in
stored CSC order (the early-exit parent). Per-level statistics are checked against the
oracle's level sizes, the Section 6.3 schedule and the exact work counts (Table 1)."""
import sys

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

PUSH, PULL = dobfs.DIR_PUSH, dobfs.DIR_PULL
MODES = ["full", "push_only", "pull_unmasked", "pull_masked", "pull_masked_ee", "pull_only"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _graphs():
    rng = np.random.default_rng(5)
    V = 100_003  # not a multiple of 32: ragged last bitmap word and tile
    m = 8 * V
    src = rng.integers(0, V, m)
    dst = (src + rng.zipf(1.6, m)) % V  # directed, skewed in-degrees, some long rows
    directed = gen.from_edges(V, src, dst, directed=True, name="directed100003")
    return {
        "rmat10": gen.rmat(10, 16, seed=1),
        "rmat14": gen.rmat(14, 16, seed=1),
        "directed100003": directed,
        "lattice37": gen.lattice3d(37, 0.05, seed=3),
        "grid61x53": gen.grid2d(61, 53),
    }


@pytest.fixture(scope="module")
def graphs():
    out = {}
    for name, hg in _graphs().items():
        _say("upload", name, hg.V, hg.nnz)
        out[name] = (hg, upload(hg, validate=True))
    return out


def _check(hg, runner, s, mode, want_depth, first_par, tag):
    d, p = runner.result()
    assert np.array_equal(d, want_depth), "%s: depth mismatch (%d differ)" % (tag, int((d != want_depth).sum()))
    code, bad = oracle.validate(hg, s, d, p)
    assert code == 0, "%s: parent check %d failed at %d (%s)" % (tag, code, bad, oracle.VALIDATE_MESSAGES[code])
    lv = runner.levels()
    assert len(lv) == runner.stats.levels
    pulled = np.zeros(hg.V, dtype=bool)
    for L, row in enumerate(lv):
        if row["dir"] == PULL:
            pulled |= want_depth == L + 1
    assert np.array_equal(p[pulled], first_par[pulled]), tag + ": pull parent is not the first in CSC order"


def _sources(hg, k, seed):
    s = [gen.max_degree_vertex(hg)]
    s += [int(x) for x in gen.sample_sources(hg, k, seed) if int(x) != s[0]][: k - 1]
    return s


@pytest.mark.parametrize("name", ["rmat10", "rmat14", "directed100003", "lattice37", "grid61x53"])
def test_all_modes_match_oracle(graphs, name):
    hg, g = graphs[name]
    runner = BfsRunner(g)
    for s in _sources(hg, 3, seed=2):
        want, _ = oracle.bfs(hg, s)
        fp = oracle.first_parent(hg, want, s)
        sizes = oracle.level_sizes(want)
        for mode in MODES:
            tag = "%s src=%d mode=%s" % (name, s, mode)
            _say(tag)
            runner.run(s, mode=mode)
            _check(hg, runner, s, mode, want, fp, tag)
            lv = runner.levels()
            assert [r["nf"] for r in lv] == sizes, tag
            assert [r["n_new"] for r in lv] == sizes[1:] + [0], tag
            assert runner.stats.reached == int((want >= 0).sum())
            dirs = [r["dir"] for r in lv]
            if mode == "full":
                assert dirs == oracle.schedule(sizes, hg.V), tag
            if mode == "push_only":
                assert set(dirs) == {PUSH}
            if mode == "pull_only":
                assert set(dirs) == {PULL}


@pytest.mark.parametrize("name", ["rmat10", "rmat14", "directed100003", "lattice37", "grid61x53"])
def test_push_sort_matches_oracle(graphs, name):
    """Table 2's baseline row: gather, key-value radix sort, first of each key, mask filter
    (Algorithm 3 as printed). Depths exact, parents valid, push at every level, the per-level
    sizes of the oracle, and the gathered pairs of a level are exactly nnz(m_f^+)."""
    hg, g = graphs[name]
    outdeg = hg.out_degree()
    opt = dobfs.make_options("push_sort")
    need = dobfs.bfs_workspace_bytes(g, opt)
    assert need > dobfs.bfs_workspace_bytes(g)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    depth = torch.empty(g.V, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.V, dtype=torch.int32, device="cuda")
    st = dobfs.make_stats(4096)
    for s in _sources(hg, 3, seed=2):
        tag = "%s src=%d push_sort" % (name, s)
        _say(tag)
        want, _ = oracle.bfs(hg, s)
        dobfs.bfs(g, s, depth, parent, opt, ws, stats=st)
        d, p = depth.cpu().numpy(), parent.cpu().numpy()
        assert np.array_equal(d, want), tag + ": depth mismatch"
        code, bad = oracle.validate(hg, s, d, p)
        assert code == 0, "%s: parent check %d failed at %d" % (tag, code, bad)
        lv = dobfs.stats_levels(st)
        sizes = oracle.level_sizes(want)
        assert [r["nf"] for r in lv] == sizes, tag
        assert set(r["dir"] for r in lv) == {PUSH}, tag
        for L, r in enumerate(lv):
            m_f = int(outdeg[want == L].sum())
            assert r["m_f"] == m_f and r["edges"] == m_f, "%s level %d" % (tag, L)
    # too small a workspace for this mode is refused
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs(g, 0, depth, parent, opt, ws, ws_bytes=need - 256)
    assert e.value.status == dobfs.ERR_WORKSPACE_TOO_SMALL


@pytest.mark.parametrize("name", ["rmat10", "rmat14", "directed100003", "lattice37", "grid61x53"])
def test_push_sort_keys_matches_oracle(graphs, name):
    """Table 2's structure-only row as the paper measures it: the sort push with the values
    dropped (key-only radix sort, unique keys, mask filter). Depths exact, push at every level,
    the oracle's level sizes and nnz(m_f^+) gathered per level; parents are not computed, so a
    parent buffer is refused, and the larger sort workspace is needed."""
    hg, g = graphs[name]
    outdeg = hg.out_degree()
    opt = dobfs.make_options("push_sort_keys")
    need = dobfs.bfs_workspace_bytes(g, opt)
    assert need == dobfs.bfs_workspace_bytes(g, dobfs.make_options("push_sort"))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    depth = torch.full((g.V,), -7, dtype=torch.int32, device="cuda")
    st = dobfs.make_stats(4096)
    for s in _sources(hg, 3, seed=2):
        tag = "%s src=%d push_sort_keys" % (name, s)
        _say(tag)
        want, _ = oracle.bfs(hg, s)
        dobfs.bfs(g, s, depth, None, opt, ws, stats=st)
        assert np.array_equal(depth.cpu().numpy(), want), tag + ": depth mismatch"
        lv = dobfs.stats_levels(st)
        assert [r["nf"] for r in lv] == oracle.level_sizes(want), tag
        assert set(r["dir"] for r in lv) == {PUSH}, tag
        for L, r in enumerate(lv):
            m_f = int(outdeg[want == L].sum())
            assert r["m_f"] == m_f and r["edges"] == m_f, "%s level %d" % (tag, L)
        assert st.edges_g500 == oracle.teps_edges(hg, want)["graph500"], tag
    parent = torch.empty(g.V, dtype=torch.int32, device="cuda")
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs(g, 0, depth, parent, opt, ws)
    assert e.value.status == dobfs.ERR_INVALID_ARG


@pytest.mark.parametrize("name", ["rmat14", "lattice37"])
def test_launch_totals(graphs, name):
    """The whole-call launch totals count what a kernel profiler counts: every launch of the
    step kernel (one or two per level, the step that finds the end, any enqueued past it);
    their time covers the per-level times. A run in push_sort mode leaves them at 0."""
    hg, g = graphs[name]
    opt = dobfs.make_options("full", time_kernels=True)
    ws = torch.empty(dobfs.bfs_workspace_bytes(g), dtype=torch.uint8, device="cuda")
    depth = torch.empty(g.V, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.V, dtype=torch.int32, device="cuda")
    st = dobfs.make_stats(4096)
    for s in _sources(hg, 4, seed=8):
        _say(name, "src", s)
        dobfs.bfs(g, s, depth, parent, opt, ws, stats=st)
        lv = dobfs.stats_levels(st)
        scanned = sum(1 for r in lv if r["dir"] == PUSH and r["variant"] == 0)
        assert st.launches_main >= st.levels + scanned + 1 and st.levels == len(lv)
        assert st.launches_aux == 0 and st.ms_aux_all == 0
        assert all(r["ms_main"] > 0 for r in lv)
        assert all((r["ms_aux"] > 0) == (r["dir"] == PUSH and r["variant"] == 0) for r in lv)
        assert st.ms_main_all >= sum(r["ms_main"] + r["ms_aux"] for r in lv) * (1 - 1e-5) > 0
        assert st.ms_main_all + st.ms_init <= st.ms_total * (1 + 1e-5)
    opt = dobfs.make_options("push_sort", time_kernels=True)
    ws = torch.empty(dobfs.bfs_workspace_bytes(g, opt), dtype=torch.uint8, device="cuda")
    dobfs.bfs(g, 0, depth, parent, opt, ws, stats=st)
    assert (st.launches_main, st.launches_aux, st.ms_main_all, st.ms_aux_all) == (0, 0, 0.0, 0.0)


def _hubs_first_order(hg):
    """Host copy of hg with every CSC column in the order DOBFS_UPLOAD_HUBS_FIRST gives it on the
    device: decreasing out-degree of the in-neighbour, ties in stored order."""
    import copy
    deg = np.diff(hg.rowptr).astype(np.int64)
    col = np.repeat(np.arange(hg.V, dtype=np.int64), np.diff(hg.csc_colptr))
    order = np.lexsort((np.arange(hg.nnz), -deg[hg.csc_rowind], col))
    out = copy.copy(hg)
    out.csc_rowind = np.ascontiguousarray(hg.csc_rowind[order])
    return out


@pytest.mark.parametrize("name", ["rmat14", "directed100003", "lattice37"])
def test_hubs_first_upload(name):
    """In-neighbours reordered on the device by decreasing out-degree: depths unchanged, parents
    valid, and a pull reports the first hit in the new order with the exact check count."""
    hg = _graphs()[name]
    g = upload(hg, hubs_first=True)
    h2 = _hubs_first_order(hg)
    r = BfsRunner(g)
    for s in _sources(hg, 2, seed=4):
        want, _ = oracle.bfs(hg, s)
        fp2 = oracle.first_parent(h2, want, s)
        for mode in ("full", "pull_only", "pull_masked_ee"):
            tag = "%s hubs-first src=%d %s" % (name, s, mode)
            r.run(s, mode=mode)
            d, p = r.result()
            assert np.array_equal(d, want), tag
            assert oracle.validate(hg, s, d, p)[0] == 0, tag
            for L, row in enumerate(r.levels()):
                if row["dir"] != PULL:
                    continue
                lvl = want == L + 1
                assert np.array_equal(p[lvl], fp2[lvl]), tag + ": level %d parents" % L
                assert row["edges"] == oracle.pull_checks(h2, want, L), tag + ": level %d checks" % L
    dobfs.graph_destroy(g)


@pytest.mark.parametrize("name", ["rmat14", "directed100003", "lattice37"])
def test_work_counts_match_table1(graphs, name):
    """Edges touched per level: push reads nnz(m_f^+); pull with early exit checks exactly the
    sequential first-hit count; pull without early exit reads every in-edge of the rows it
    computes (all rows when unmasked)."""
    hg, g = graphs[name]
    runner = BfsRunner(g)
    s = gen.max_degree_vertex(hg)
    want, _ = oracle.bfs(hg, s)
    outdeg, indeg = hg.out_degree(), hg.in_degree()
    for mode in MODES:
        runner.run(s, mode=mode)
        for L, row in enumerate(runner.levels()):
            tag = "%s mode=%s level=%d" % (name, mode, L)
            unvisited = ~((want >= 0) & (want <= L))
            if row["dir"] == PUSH:
                m_f = int(outdeg[want == L].sum())
                assert row["m_f"] == m_f and row["edges"] == m_f, tag
            elif mode in ("full", "pull_only", "pull_masked_ee"):
                assert row["edges"] == oracle.pull_checks(hg, want, L), tag
            elif mode == "pull_masked":
                assert row["edges"] == int(indeg[unvisited].sum()), tag
            elif mode == "pull_unmasked":
                assert row["edges"] == hg.nnz, tag


def test_forced_schedules(graphs):
    hg, g = graphs["rmat14"]
    runner = BfsRunner(g)
    s = gen.max_degree_vertex(hg)
    want, _ = oracle.bfs(hg, s)
    fp = oracle.first_parent(hg, want, s)
    nlev = len(oracle.level_sizes(want))
    rng = np.random.default_rng(9)
    schedules = [[PUSH] * nlev, [PULL] * nlev, [k % 2 for k in range(nlev)],
                 [1 - k % 2 for k in range(nlev)]] + [list(rng.integers(0, 2, nlev)) for _ in range(6)]
    for mode in MODES:
        for sched in schedules:
            tag = "forced %s %s" % (mode, sched)
            runner.run(s, mode=mode, forced_dirs=sched)
            _check(hg, runner, s, mode, want, fp, tag)
            assert [r["dir"] for r in runner.levels()] == [int(x) for x in sched][: runner.stats.levels]


def test_push_variants(graphs):
    """Push levels run one of three ways (stats variant): with the global degree scan (0),
    block-local over the frontier list a push left (1), or block-local over the bits a pull
    found (2, when no pull tile found more than 512 rows and none of out-degree above 32).
    All give the oracle's depths, valid parents and exact per-level counts; each kind occurs."""
    seen = set()
    for name in ("rmat14", "directed100003", "lattice37", "grid61x53"):
        hg, g = graphs[name]
        runner = BfsRunner(g)
        outdeg = hg.out_degree()
        for s in _sources(hg, 3, seed=11):
            want, _ = oracle.bfs(hg, s)
            fp = oracle.first_parent(hg, want, s)
            for heur, a, b in ((dobfs.HEUR_EDGES, 1 / 14, 1 / 24), (dobfs.HEUR_RATIO, 0.01, 0.01)):
                tag = "%s src=%d heur=%d" % (name, s, heur)
                runner.run(s, heuristic=heur, alpha=a, beta=b)
                _check(hg, runner, s, "full", want, fp, tag)
                lv = runner.levels()
                for L, r in enumerate(lv):
                    if r["dir"] == PULL:
                        assert r["variant"] == 0, tag
                        continue
                    m_f = int(outdeg[want == L].sum())
                    assert r["m_f"] == m_f and r["edges"] == m_f, "%s level %d" % (tag, L)
                    after_pull = L > 0 and lv[L - 1]["dir"] == PULL
                    assert r["variant"] in ((0, 2) if after_pull else (0, 1)), "%s level %d" % (tag, L)
                    if after_pull and r["variant"] == 2:
                        found = want == L  # what the pull before found: no heavy row
                        assert outdeg[found].max(initial=0) <= 32, tag
                    seen.add(r["variant"])
    assert {1, 2} <= seen, seen  # the global scan (0) is forced below
    # a push right after a pull that found high-degree rows must take the global scan
    hg, g = graphs["rmat14"]
    s = gen.max_degree_vertex(hg)
    want, _ = oracle.bfs(hg, s)
    runner = BfsRunner(g)
    runner.run(s, forced_dirs=[PULL, PUSH, PUSH])
    lv = runner.levels()
    assert outdeg_max_at(hg, want, 1) > 32
    assert [r["variant"] for r in lv[:2]] == [0, 0]
    _check(hg, runner, s, "full", want, oracle.first_parent(hg, want, s), "forced pull-push")


def test_local_culling_wide_frontiers():
    """Push levels whose frontier has 8192 vertices or more drop repeated targets in LDS before
    the claim. A layered graph where every level-1 vertex shares most of its targets with
    others, with duplicate edges and self-loops kept, pushed from frontiers of 10 000 and
    ~20 000 vertices: depths, parents and every level's counts still match the oracle, in the
    step loop and the persistent loop, block-local over the list and over the pull's bits."""
    rng = np.random.default_rng(31)
    n1, n2, n3 = 10_000, 20_000, 3_000
    V = 1 + n1 + 10 * n2 + n3
    l1 = np.arange(1, 1 + n1)
    # level 2 every tenth id (isolated vertices between): a pull finds at most ~410 of them per
    # 4096-row tile, so the push after it can run over the pull's bits
    l2 = 1 + n1 + 10 * np.arange(n2)
    l3 = 1 + n1 + 10 * n2 + np.arange(n3)
    src = [np.zeros(n1, np.int64), np.repeat(l1, 8), np.repeat(l2, 3), l1[:500], l2[:700]]
    dst = [l1, rng.choice(l2, 8 * n1), rng.choice(l3, 3 * n2), l1[:500], l2[:700]]
    src.append(np.repeat(l1[:2000], 2))  # duplicate edges
    dst.append(np.repeat(rng.choice(l2, 2000), 2))
    hg = gen.from_edges(V, np.concatenate(src), np.concatenate(dst), directed=True,
                        keep_self_loops=True, keep_duplicates=True, name="layers_culling")
    g = upload(hg, hubs_first=True)
    want, _ = oracle.bfs(hg, 0)
    fp = oracle.first_parent(hg, want, 0)
    assert int((want == 1).sum()) == n1 and int((want == 2).sum()) > 8192
    runner = BfsRunner(g)
    outdeg = hg.out_degree()
    cases = [dict(mode="push_only"), dict(mode="push_only", persistent=True),
             dict(forced_dirs=[PUSH, PUSH, PUSH, PUSH]), dict(forced_dirs=[PUSH, PULL, PUSH, PUSH]),
             dict(forced_dirs=[PUSH, PULL, PUSH, PUSH], persistent=True)]
    variants = set()
    for c in cases:
        tag = "layers %s" % c
        runner.run(0, **c)
        _check(hg, runner, 0, "full", want, fp, tag)
        lv = runner.levels()
        variants.update(r["variant"] for r in lv[2:3] if r["dir"] == PUSH)
        for L, r in enumerate(lv):
            assert r["nf"] == int((want == L).sum()), "%s level %d" % (tag, L)
            assert r["n_new"] == int((want == L + 1).sum()), "%s level %d" % (tag, L)
            if r["dir"] == PUSH:
                assert r["edges"] == int(outdeg[want == L].sum()), "%s level %d" % (tag, L)
    assert variants == {1, 2}, variants  # the level-2 push over the list and over the pull's bits
    dobfs.graph_destroy(g)


def outdeg_max_at(hg, depth, L):
    return int(hg.out_degree()[depth == L].max(initial=0))


def test_repeat_determinism(graphs):
    hg, g = graphs["rmat14"]
    runner = BfsRunner(g)
    s = gen.max_degree_vertex(hg)
    want, _ = oracle.bfs(hg, s)
    for _ in range(30):
        runner.run(s)
        d, p = runner.result()
        assert np.array_equal(d, want)
        assert oracle.validate(hg, s, d, p)[0] == 0


def test_edges_heuristic(graphs):
    """Beamer's edge-count rule: exact depths, valid parents, and the direction sequence the
    oracle derives from m_f and m_u of its own depths (the device tracks m_u incrementally)."""
    for name in ("rmat14", "directed100003", "lattice37"):
        hg, g = graphs[name]
        runner = BfsRunner(g)
        for s in _sources(hg, 3, seed=4):
            want, _ = oracle.bfs(hg, s)
            fp = oracle.first_parent(hg, want, s)
            for a, b in ((1 / 14, 1 / 24), (1 / 40, 1 / 96), (1 / 3, 1 / 12)):
                tag = "%s src=%d edges-rule %.4g %.4g" % (name, s, a, b)
                _say(tag)
                runner.run(s, heuristic=dobfs.HEUR_EDGES, alpha=a, beta=b)
                _check(hg, runner, s, "edges", want, fp, tag)
                dirs = [r["dir"] for r in runner.levels()]
                assert dirs == oracle.schedule_edges(hg, want, a, b), tag


def test_directed_orientation(tmp_path):
    hg = gen.from_edges(3, [0, 1], [1, 2], directed=True)
    g = upload(hg)
    r = BfsRunner(g)
    for mode in MODES:
        r.run(0, mode=mode)
        assert r.result()[0].tolist() == [0, 1, 2]
        assert r.result()[1].tolist() == [0, 0, 1]
        r.run(2, mode=mode)
        assert r.result()[0].tolist() == [-1, -1, 0]
        assert r.result()[1].tolist() == [-1, -1, 2]


def test_small_edge_cases():
    cases = {
        "single": gen.from_edges(1, [], []),
        "edgeless": gen.from_edges(70, [], []),
        "path": gen.from_edges(3000, np.arange(2999), np.arange(1, 3000)),
        "star": gen.from_edges(5000, np.zeros(4999, int), np.arange(1, 5000)),
        "loops_dups": gen.from_edges(6, [0, 0, 0, 1, 1, 2, 4], [0, 1, 1, 2, 2, 3, 5], directed=True,
                                     keep_self_loops=True, keep_duplicates=True),
        "two_components": gen.from_edges(40, [0, 1, 2, 20, 21], [1, 2, 3, 21, 22]),
    }
    for name, hg in cases.items():
        g = upload(hg, validate=True)
        r = BfsRunner(g)
        for s in sorted({0, hg.V - 1, hg.V // 2}):
            want, _ = oracle.bfs(hg, s)
            fp = oracle.first_parent(hg, want, s)
            for mode in MODES:
                r.run(s, mode=mode)
                _check(hg, r, s, mode, want, fp, "%s src=%d %s" % (name, s, mode))


def test_errors_and_workspace(graphs):
    hg, g = graphs["rmat10"]
    r = BfsRunner(g)
    r.depth.fill_(7)
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs(g, hg.V, r.depth, r.parent, None, r.ws)
    assert e.value.status == dobfs.ERR_INVALID_ARG
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs(g, -1, r.depth, r.parent, None, r.ws)
    assert e.value.status == dobfs.ERR_INVALID_ARG
    assert int((r.depth != 7).sum()) == 0, "nothing may be written on a rejected call"
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs(g, 0, r.depth, r.parent, None, r.ws, ws_bytes=r.ws.numel() - 256)
    assert e.value.status == dobfs.ERR_WORKSPACE_TOO_SMALL
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs(g, 0, r.depth, r.parent, dobfs.make_options(mode=17), r.ws)
    assert e.value.status == dobfs.ERR_INVALID_ARG
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs(g, 0, r.depth, r.parent, dobfs.make_options(forced_dirs=[0, 3]), r.ws)
    assert e.value.status == dobfs.ERR_INVALID_ARG
    # library-owned workspace, no parent output, and a side stream give the same depths
    s = gen.max_degree_vertex(hg)
    want, _ = oracle.bfs(hg, s)
    depth = torch.empty(hg.V, dtype=torch.int32, device="cuda")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        dobfs.bfs(g, s, depth, None, None, None, stream=side)
    side.synchronize()
    assert np.array_equal(depth.cpu().numpy(), want)


def test_upload_checks():
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.graph_upload(3, 2, [0, 2, 1, 2], [1, 2], [0, 2, 1, 2], [1, 2])
    assert e.value.status == dobfs.ERR_INVALID_ARG
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.graph_upload(3, 2, [0, 1, 2, 2], [1, 5], [0, 0, 1, 2], [0, 1], flags=dobfs.UPLOAD_VALIDATE)
    assert e.value.status == dobfs.ERR_INVALID_ARG


def test_wrap_device_matches_upload(graphs):
    hg, _ = graphs["directed100003"]
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in
         (hg.rowptr, hg.colind, hg.csc_colptr, hg.csc_rowind)]
    g = dobfs.graph_wrap_device(hg.V, hg.nnz, *t, flags=dobfs.UPLOAD_VALIDATE)
    r = BfsRunner(g)
    s = gen.max_degree_vertex(hg)
    want, _ = oracle.bfs(hg, s)
    r.run(s)
    assert np.array_equal(r.result()[0], want)
    bad = t[0].clone()
    bad[5] = bad[6] + 1
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.graph_wrap_device(hg.V, hg.nnz, bad, t[1], t[2], t[3])
    assert e.value.status == dobfs.ERR_INVALID_ARG


def test_permutation_invariance(graphs):
    """Relabelling the vertices relabels the depths."""
    hg, g = graphs["rmat14"]
    rng = np.random.default_rng(3)
    perm = rng.permutation(hg.V)
    rows = np.repeat(np.arange(hg.V), np.diff(hg.rowptr.astype(np.int64)))
    pg = gen.from_edges(hg.V, perm[rows], perm[hg.colind], directed=True)
    r1, r2 = BfsRunner(g), BfsRunner(upload(pg))
    s = gen.max_degree_vertex(hg)
    r1.run(s)
    r2.run(int(perm[s]))
    d1, d2 = r1.result()[0], r2.result()[0]
    assert np.array_equal(d2[perm], d1)
