"""GPU parity of the multi-source BFS (dobfs_bfs_batch) against the CPU oracle, through the C
ABI.

Every depth row must equal the oracle's single-source depths from that row's source, bit for
bit, in every supported mode and under forced push/pull schedules. Per-level statistics are
checked against what the oracle's depth rows fix: the vertices carrying any frontier bit at
each level, the (vertex, source) pairs reached, and the level count."""
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _graphs():
    rng = np.random.default_rng(7)
    V = 100_003  # ragged last bitmap word and tile
    m = 8 * V
    src = rng.integers(0, V, m)
    dst = (src + rng.zipf(1.6, m)) % V
    return {
        "rmat10": gen.rmat(10, 16, seed=1),
        "rmat14": gen.rmat(14, 16, seed=1),
        "directed100003": gen.from_edges(V, src, dst, directed=True, name="directed100003"),
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


_ref_cache = {}


def _ref(hg, s):
    key = (hg.name, hg.V, int(s))
    if key not in _ref_cache:
        _ref_cache[key] = oracle.bfs(hg, int(s))[0]
    return _ref_cache[key]


def _sources(hg, k, seed):
    return [int(x) for x in gen.sample_sources(hg, k, seed)]


def _run(g, sources, opt=None, cap=256):
    k = len(sources)
    depth = torch.full((k * g.V,), -7, dtype=torch.int32, device="cuda")
    st = dobfs.make_stats(cap)
    dobfs.bfs_batch(g, sources, depth, opt=opt, stats=st)
    return depth.cpu().numpy().reshape(k, g.V), st


def _check(hg, sources, d, st, tag):
    refs = [_ref(hg, s) for s in sources]
    for b, s in enumerate(sources):
        bad = int((d[b] != refs[b]).sum())
        assert bad == 0, "%s: row %d (source %d): %d depths differ" % (tag, b, s, bad)
    R = np.stack(refs)
    ecc = int(R.max())
    assert st.levels == ecc + 1, "%s: %d levels, oracle says %d" % (tag, st.levels, ecc + 1)
    assert st.reached == int((R >= 0).sum()), tag + ": reached pairs"
    lv = dobfs.stats_levels(st)
    # one step per pull level, two per push level (scan, expansion), one that finds the end
    pushes = sum(1 for x in lv if x["dir"] == PUSH)
    assert st.launches_main >= st.levels + pushes + 1 and st.launches_aux == 0, tag + ": launch totals"
    for L, row in enumerate(lv):
        nf = int((R == L).any(axis=0).sum())
        n_new = int((R == L + 1).any(axis=0).sum())
        assert (row["nf"], row["n_new"]) == (nf, n_new), "%s: level %d sizes %s vs (%d, %d)" % (
            tag, L, (row["nf"], row["n_new"]), nf, n_new)


@pytest.mark.parametrize("name", ["rmat10", "rmat14", "directed100003", "lattice37", "grid61x53"])
def test_batch_modes_match_oracle(graphs, name):
    hg, g = graphs[name]
    srcs = _sources(hg, 64, 11)
    for mode in ["full", "push_only", "pull_only"]:
        for heur, a, b in [(dobfs.HEUR_RATIO, 0.01, 0.01), (dobfs.HEUR_EDGES, 1 / 14, 1 / 24)]:
            tag = "%s k=64 %s heur=%d" % (name, mode, heur)
            _say(tag)
            d, st = _run(g, srcs, dobfs.make_options(mode, heur, a, b))
            _check(hg, srcs, d, st, tag)
            dirs = [x["dir"] for x in dobfs.stats_levels(st)]
            if mode == "push_only":
                assert set(dirs) == {PUSH}
            if mode == "pull_only":
                assert set(dirs) == {PULL}


@pytest.mark.parametrize("k", [1, 2, 31, 33, 63, 64])
def test_batch_widths(graphs, k):
    hg, g = graphs["rmat14"]
    srcs = _sources(hg, k, 100 + k)
    d, st = _run(g, srcs)
    _check(hg, srcs, d, st, "rmat14 k=%d" % k)


def test_batch_forced_schedules(graphs):
    hg, g = graphs["rmat14"]
    srcs = _sources(hg, 40, 21)
    rng = np.random.default_rng(3)
    scheds = [[PUSH, PULL] * 8, [PULL, PUSH] * 8, [PUSH, PUSH, PULL, PULL] * 4]
    scheds += [list(rng.integers(0, 2, 16)) for _ in range(5)]
    for sc in scheds:
        tag = "forced %s" % "".join(str(int(x)) for x in sc)
        _say(tag)
        d, st = _run(g, srcs, dobfs.make_options("full", forced_dirs=[int(x) for x in sc]))
        _check(hg, srcs, d, st, tag)
        dirs = [x["dir"] for x in dobfs.stats_levels(st)]
        assert dirs == [int(x) for x in sc[: len(dirs)]], tag


def test_batch_duplicates_and_isolated(graphs):
    hg, g = graphs["rmat14"]
    deg = np.diff(hg.rowptr)
    iso = [int(x) for x in np.nonzero(deg == 0)[0][:3]]
    assert len(iso) == 3
    s = _sources(hg, 10, 5)
    srcs = s + s[:4] + iso + [s[0]] * 5  # repeats and degree-0 sources
    d, st = _run(g, srcs)
    _check(hg, srcs, d, st, "duplicates+isolated")


def test_batch_repeated_calls_reuse_workspace(graphs):
    """Back-to-back calls with different sources and widths on one workspace: nothing of a
    previous call may leak into the next (frontier words, level table, counters)."""
    hg, g = graphs["directed100003"]
    k_max = 64
    ws = torch.empty(dobfs.bfs_batch_workspace_bytes(g, k_max), dtype=torch.uint8, device="cuda")
    for it, k in enumerate([64, 5, 64, 17, 1, 64]):
        srcs = _sources(hg, k, 300 + it)
        depth = torch.full((k * g.V,), -7, dtype=torch.int32, device="cuda")
        st = dobfs.make_stats(256)
        mode = ["full", "pull_only", "push_only"][it % 3]
        dobfs.bfs_batch(g, srcs, depth, opt=dobfs.make_options(mode), workspace=ws, stats=st)
        _check(hg, srcs, depth.cpu().numpy().reshape(k, g.V), st, "repeat %d k=%d %s" % (it, k, mode))


def test_batch_small_graphs():
    cases = {
        "one_vertex": gen.from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64), directed=False),
        "path9": gen.from_edges(9, np.arange(8), np.arange(1, 9), directed=False),
        "directed_path": gen.from_edges(3, np.array([0, 1]), np.array([1, 2]), directed=True),
        "two_parts": gen.from_edges(70, np.array([0, 1, 2, 40, 41]), np.array([1, 2, 3, 41, 42]),
                                    directed=False),
        "self_loops_dups": gen.from_edges(5, np.array([0, 0, 1, 1, 2, 3]), np.array([0, 1, 1, 2, 2, 4]),
                                          directed=True, keep_self_loops=True, keep_duplicates=True),
    }
    for name, hg in cases.items():
        g = upload(hg)
        for srcs in ([0], list(range(min(hg.V, 64))), [hg.V - 1] * 3):
            for mode in ["full", "push_only", "pull_only"]:
                d, st = _run(g, srcs, dobfs.make_options(mode))
                _check(hg, srcs, d, st, "%s %s k=%d" % (name, mode, len(srcs)))


@pytest.mark.parametrize("V", [15, 16, 17, 18, 19, 40])
def test_batch_kept_level_boundary(V):
    """Paths whose eccentricities straddle the number of levels whose frontier words are kept
    (16): depths below it come from those words, deeper ones from the level table, and the
    two alternating frontier buffers past it start out holding a previous call's words."""
    hg = gen.from_edges(V, np.arange(V - 1), np.arange(1, V), directed=False, name="path%d" % V)
    g = upload(hg)
    rng = np.random.default_rng(V)
    for k in (33, 64):
        srcs = [0, V - 1, V // 2, 1] + [int(x) for x in rng.integers(0, V, k - 4)]
        for mode in ["full", "push_only", "pull_only"]:
            d, st = _run(g, srcs, dobfs.make_options(mode))
            _check(hg, srcs, d, st, "path%d %s k=%d" % (V, mode, k))


def test_batch_forced_schedules_deep(graphs):
    """Push and pull alternating over a traversal far deeper than the kept frontier levels: a
    push after a pull must clear a recycled frontier buffer densely, a push after a push
    through the earlier push's list."""
    hg, g = graphs["grid61x53"]
    srcs = [0] + _sources(hg, 32, 41)
    for sc in ([PUSH, PULL] * 70, [PULL, PULL, PUSH] * 50, [PUSH, PUSH, PULL] * 50):
        tag = "grid forced %s..." % "".join(str(int(x)) for x in sc[:6])
        _say(tag)
        d, st = _run(g, srcs, dobfs.make_options("full", forced_dirs=[int(x) for x in sc]))
        _check(hg, srcs, d, st, tag)
        dirs = [x["dir"] for x in dobfs.stats_levels(st)]
        assert dirs == [int(x) for x in sc[: len(dirs)]], tag


def test_batch_step_times(graphs):
    """Timed steps: every level's pull or expansion step has a time, every push level's scan
    step too (and only those), and the per-launch totals cover them; no second kernel kind."""
    for name in ("rmat14", "lattice37"):
        hg, g = graphs[name]
        srcs = _sources(hg, 64, 17)
        st = dobfs.make_stats(1024)
        depth = torch.empty(64 * g.V, dtype=torch.int32, device="cuda")
        dobfs.bfs_batch(g, srcs, depth, opt=dobfs.make_options("full", time_kernels=True), stats=st)
        _check(hg, srcs, depth.cpu().numpy().reshape(64, g.V), st, name + " timed")
        lv = dobfs.stats_levels(st)
        assert all(x["ms_main"] > 0 for x in lv), name
        assert all((x["ms_aux"] > 0) == (x["dir"] == PUSH) for x in lv), name
        assert st.launches_aux == 0 and st.ms_aux_all == 0, name
        assert st.ms_main_all >= sum(x["ms_main"] + x["ms_aux"] for x in lv) * (1 - 1e-5), name


def test_batch_deep_path_past_the_state_ring():
    """A 2600-vertex path: push levels take two steps each, so the step count passes the
    device's ring of 1024 states several times; forced directions cover the first 1024 levels
    only, later levels follow the rule."""
    V = 2600
    hg = gen.from_edges(V, np.arange(V - 1), np.arange(1, V), directed=False, name="path%d" % V)
    g = upload(hg)
    srcs = [0, V - 1, V // 2, 7]
    for mode in ["push_only", "full"]:
        _say("path%d %s" % (V, mode))
        d, st = _run(g, srcs, dobfs.make_options(mode), cap=4096)
        _check(hg, srcs, d, st, "path%d %s" % (V, mode))
    sc = [PUSH, PULL, PULL] * 400  # 1200 levels asked for
    d, st = _run(g, srcs, dobfs.make_options("push_only", forced_dirs=sc), cap=4096)
    _check(hg, srcs, d, st, "path forced")
    dirs = [x["dir"] for x in dobfs.stats_levels(st)]
    assert dirs[:1024] == sc[:1024] and set(dirs[1024:]) == {PUSH}


def test_batch_pull_after_push_only_batches():
    """A 400 x 400 grid (625 pull tiles) forced to push for 300 levels, then to alternate: the
    batches of pushes shrink the step launches below the tile count, and the pulls after them
    run on that smaller grid, a block taking several tiles."""
    hg = gen.grid2d(400, 400)
    g = upload(hg)
    srcs = [0, hg.V - 1] + _sources(hg, 6, 77)
    sc = [PUSH] * 300 + [PULL, PUSH] * 300
    for mode in ["full", "push_only"]:
        tag = "grid400 %s forced" % mode
        _say(tag)
        d, st = _run(g, srcs, dobfs.make_options(mode, forced_dirs=sc), cap=2048)
        _check(hg, srcs, d, st, tag)
        dirs = [x["dir"] for x in dobfs.stats_levels(st)]
        assert dirs == sc[: len(dirs)], tag
    d, st = _run(g, srcs, dobfs.make_options("push_only"), cap=2048)
    _check(hg, srcs, d, st, "grid400 push_only rule")


def test_batch_wide_pushes_deep():
    """Consecutive layers of 200 vertices joined completely, 24 layers: every push level reads
    more than 64 Ki edges, so its winners are marked in the non-zero bitmap rather than listed,
    the next push lists them from that bitmap, and past the kept frontier levels the recycled
    buffers are cleared through those lists."""
    W, D = 200, 24
    src, dst = [], []
    for l in range(D - 1):
        a = np.arange(l * W, (l + 1) * W)
        b = np.arange((l + 1) * W, (l + 2) * W)
        src.append(np.repeat(a, W))
        dst.append(np.tile(b, W))
    hg = gen.from_edges(W * D, np.concatenate(src), np.concatenate(dst), directed=False, name="layers")
    g = upload(hg)
    rng = np.random.default_rng(5)
    srcs = [0, 1, W * D - 1] + [int(x) for x in rng.integers(0, W * D, 61)]
    for mode in ["push_only", "full"]:
        for sc in (None, [PUSH, PUSH, PULL] * 10):
            tag = "layers %s %s" % (mode, "forced" if sc else "rule")
            _say(tag)
            opt = dobfs.make_options(mode, forced_dirs=sc) if sc else dobfs.make_options(mode)
            d, st = _run(g, srcs, opt)
            _check(hg, srcs, d, st, tag)
            if mode == "push_only" or sc:  # the rule itself may pull the wide levels
                lv = dobfs.stats_levels(st)
                assert max(x["edges"] for x in lv if x["dir"] == PUSH) > 64 * 1024, tag


def test_batch_errors(graphs):
    hg, g = graphs["rmat10"]
    depth = torch.zeros(64 * g.V, dtype=torch.int32, device="cuda")
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_batch(g, [], depth)
    assert e.value.status == dobfs.ERR_INVALID_ARG
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_batch(g, list(range(65)), torch.zeros(65 * g.V, dtype=torch.int32, device="cuda"))
    assert e.value.status == dobfs.ERR_INVALID_ARG
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_batch(g, [0, g.V], depth)
    assert e.value.status == dobfs.ERR_INVALID_ARG
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_batch(g, [0, 1], depth, opt=dobfs.make_options("pull_masked"))
    assert e.value.status == dobfs.ERR_UNSUPPORTED
    need = dobfs.bfs_batch_workspace_bytes(g, 2)
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_batch(g, [0, 1], depth, workspace=ws)
    assert e.value.status == dobfs.ERR_WORKSPACE_TOO_SMALL
    assert dobfs.bfs_batch_workspace_bytes(g, 64) > dobfs.bfs_batch_workspace_bytes(g, 1)


def test_interleaved_with_single_source_reports():
    """Single-source and multi-source traversals share the thread's pinned report buffer: many
    calls of each, interleaved on one thread, each answer checked (a report sequence number left
    by one loop must never satisfy the other's wait)."""
    hg = gen.rmat(10, 16, seed=1)
    g = upload(hg)
    runner = BfsRunner(g, with_parent=False)
    srcs = _sources(hg, 8, seed=12)
    refs = {s: _ref(hg, s) for s in srcs}
    for rnd in range(3):
        for i in range(250):
            s = srcs[i % len(srcs)]
            runner.run(s)
            if i % 25 == 0:
                assert np.array_equal(runner.result()[0], refs[s]), "single source %d, round %d" % (s, rnd)
        for i in range(250):
            b = srcs[i % 4: i % 4 + 4]
            d, _ = _run(g, b)
            if i % 25 == 0:
                for row, s in zip(d, b):
                    assert np.array_equal(row, refs[s]), "batch row of source %d, round %d" % (s, rnd)
        _say("interleaved round", rnd, "ok")



@pytest.mark.parametrize("name", ["rmat14", "lattice37"])
def test_batch_last_level_pull_after_push(graphs, name):
    """Schedules whose last level is a pull right after a push: that pull merges the push's
    winners into the visited words itself, and the depth rows must read its output."""
    hg, g = graphs[name]
    srcs = _sources(hg, 64, 11)
    n = int(np.stack([_ref(hg, s) for s in srcs]).max()) + 1  # levels of the batch
    alternating = [PUSH if (n - 1 - i) % 2 == 1 else PULL for i in range(n)]
    for sc in ([PUSH] * (n - 1) + [PULL], [PULL] * (n - 2) + [PUSH, PULL], alternating):
        tag = "%s last-pull schedule %s" % (name, "".join(str(int(x)) for x in sc))
        _say(tag)
        d, st = _run(g, srcs, dobfs.make_options("full", forced_dirs=sc))
        _check(hg, srcs, d, st, tag)
        assert [x["dir"] for x in dobfs.stats_levels(st)] == sc, tag
