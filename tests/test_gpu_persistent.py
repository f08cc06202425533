"""The persistent level loop (DOBFS_OPT_PERSISTENT) against the oracle and against the
one-launch-per-step loop: depths exact, parents valid and first-hit on pull levels, the same
per-level sizes, directions and work counts; forced direction schedules; traversals deeper
than one launch's 64 steps; per-level times from the device clock; the bounded barrier wait
forced to give up from the host (a spin limit of 0 polls), after which the next call is
correct again; and the allocation-free call in the persistent form. The multi-source
traversal's persistent form gets the same checks: every depth row against the oracle and the
level sequence against its step loop."""
import os
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
    V = 100_003
    m = 8 * V
    src = rng.integers(0, V, m)
    dst = (src + rng.zipf(1.6, m)) % V
    return {
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
        out[name] = (hg, upload(hg))
    return out


def _levels_key(lv):
    return [(r["dir"], r["nf"], r["n_new"], r["edges"], r["m_f"], r["variant"]) for r in lv]


def _check(hg, s, d, p, want, lv, tag):
    assert np.array_equal(d, want), "%s: %d depths differ" % (tag, int((d != want).sum()))
    code, at = oracle.validate(hg, s, d, p)
    assert code == 0, "%s: parent check %d failed at %d" % (tag, code, at)
    fp = oracle.first_parent(hg, want, s)
    pulled = np.zeros(hg.V, dtype=bool)
    for L, row in enumerate(lv):
        if row["dir"] == PULL:
            pulled |= want == L + 1
    assert np.array_equal(p[pulled], fp[pulled]), tag + ": pull parent is not the first in CSC order"


@pytest.mark.parametrize("name", ["rmat14", "directed100003", "lattice37", "grid61x53"])
def test_modes_match_step_loop_and_oracle(graphs, name):
    hg, g = graphs[name]
    r = BfsRunner(g)
    srcs = [gen.max_degree_vertex(hg)] + [int(x) for x in gen.sample_sources(hg, 2, seed=2)]
    for s in srcs:
        want, _ = oracle.bfs(hg, s)
        for mode in MODES:
            for heur, a, b in ((dobfs.HEUR_RATIO, 0.01, 0.01), (dobfs.HEUR_EDGES, 1 / 14, 1 / 24)):
                tag = "%s src=%d %s heur=%d" % (name, s, mode, heur)
                _say(tag)
                r.run(s, mode=mode, heuristic=heur, alpha=a, beta=b)
                ref = _levels_key(r.levels())
                r.run(s, mode=mode, heuristic=heur, alpha=a, beta=b, persistent=True)
                d, p = r.result()
                lv = r.levels()
                _check(hg, s, d, p, want, lv, tag)
                assert r.stats.levels == len(lv)
                key = _levels_key(lv)
                if mode in ("full", "push_only", "pull_only"):
                    assert key == ref, tag  # push levels' counts do not depend on the winners
                else:
                    assert [k[:3] for k in key] == [k[:3] for k in ref], tag


@pytest.mark.parametrize("name", ["rmat14", "directed100003"])
def test_forced_schedules(graphs, name):
    hg, g = graphs[name]
    r = BfsRunner(g)
    s = gen.max_degree_vertex(hg)
    want, _ = oracle.bfs(hg, s)
    n = len(oracle.level_sizes(want))
    for pattern in ([PUSH, PULL], [PULL, PUSH], [PULL, PULL, PUSH], [PUSH, PUSH, PULL]):
        dirs = [pattern[k % len(pattern)] for k in range(n)]
        tag = "%s forced %s" % (name, pattern)
        _say(tag)
        r.run(s, mode="full", forced_dirs=dirs, persistent=True)
        d, p = r.result()
        lv = r.levels()
        _check(hg, s, d, p, want, lv, tag)
        assert [x["dir"] for x in lv] == dirs[: len(lv)], tag


def test_deep_traversal_spans_launches():
    """A 3000-vertex path and a 400 x 7 grid: more than 64 steps, so several launches."""
    V = 3000
    path = gen.from_edges(V, np.arange(V - 1), np.arange(1, V), directed=False, name="path3000")
    grid = gen.grid2d(400, 7)
    for hg in (path, grid):
        g = upload(hg)
        r = BfsRunner(g, stats_cap=8192)
        for s in (0, hg.V // 2):
            want, _ = oracle.bfs(hg, s)
            for mode in ("full", "push_only"):
                tag = "%s src=%d %s" % (hg.name, s, mode)
                _say(tag)
                st = r.run(s, mode=mode, persistent=True, time_kernels=True)
                d, p = r.result()
                lv = r.levels()
                _check(hg, s, d, p, want, lv, tag)
                assert len(lv) == len(oracle.level_sizes(want)), tag
                # one launch per 64 steps (levels here take one step each), the per-level times
                # from the device clock inside the launches' times
                assert st.launches_main == (len(lv) + 1 + 63) // 64, tag
                assert all(x["ms_main"] > 0 for x in lv), tag
                assert st.ms_main_all >= sum(x["ms_main"] for x in lv) * 0.9, tag
        dobfs.graph_destroy(g)


def test_barrier_wait_gives_up_and_recovers(graphs):
    hg, g = graphs["rmat14"]
    r = BfsRunner(g)
    s = gen.max_degree_vertex(hg)
    os.environ["DOBFS_SPIN_LIMIT"] = "0"
    try:
        with pytest.raises(dobfs.DobfsError) as e:
            r.run(s, mode="full", persistent=True)
        assert e.value.status == dobfs.ERR_INTERNAL and "barrier" in str(e.value)
    finally:
        del os.environ["DOBFS_SPIN_LIMIT"]
    want, _ = oracle.bfs(hg, s)
    r.run(s, mode="full", persistent=True)
    d, p = r.result()
    _check(hg, s, d, p, want, r.levels(), "after a given-up wait")


def test_static_call_persistent(graphs):
    hg, g = graphs["lattice37"]
    s = int(gen.sample_sources(hg, 1, seed=9)[0])
    want, _ = oracle.bfs(hg, s)
    depth = torch.full((g.V,), -7, dtype=torch.int32, device="cuda")
    parent = torch.full((g.V,), -7, dtype=torch.int32, device="cuda")
    st = dobfs.make_stats(1024)
    dobfs.bfs_static(g, s, depth, parent, dobfs.make_options("full", persistent=True), stats=st)
    torch.cuda.synchronize()
    _check(hg, s, depth.cpu().numpy(), parent.cpu().numpy(), want, dobfs.stats_levels(st), "static persistent")


# ------------------------------------------------------------------ multi-source
_rows_cache = {}


def _rows(hg, sources):
    out = []
    for v in sources:
        key = (hg.name, hg.V, int(v))
        if key not in _rows_cache:
            _rows_cache[key] = oracle.bfs(hg, int(v))[0]
        out.append(_rows_cache[key])
    return np.stack(out)


def _batch(g, sources, opt, cap=4096):
    k = len(sources)
    depth = torch.full((k * g.V,), -7, dtype=torch.int32, device="cuda")
    st = dobfs.make_stats(cap)
    dobfs.bfs_batch(g, sources, depth, opt=opt, stats=st)
    return depth.cpu().numpy().reshape(k, g.V), st


def _batch_key(st):
    return [(x["dir"], x["nf"], x["n_new"], x["edges"], x["m_f"]) for x in dobfs.stats_levels(st)]


@pytest.mark.parametrize("name", ["rmat14", "directed100003", "lattice37", "grid61x53"])
def test_batch_modes_match_step_loop_and_oracle(graphs, name):
    hg, g = graphs[name]
    srcs = [int(x) for x in gen.sample_sources(hg, 64, seed=31)]
    want = _rows(hg, srcs)
    for mode in ("full", "push_only", "pull_only"):
        for heur, a, b in ((dobfs.HEUR_RATIO, 0.01, 0.01), (dobfs.HEUR_EDGES, 1 / 14, 1 / 24)):
            tag = "%s batch %s heur=%d" % (name, mode, heur)
            _say(tag)
            _, ref = _batch(g, srcs, dobfs.make_options(mode, heur, a, b))
            d, st = _batch(g, srcs, dobfs.make_options(mode, heur, a, b, persistent=True))
            bad = int((d != want).sum())
            assert bad == 0, "%s: %d depths differ" % (tag, bad)
            assert st.levels == int(want.max()) + 1 and st.reached == int((want >= 0).sum()), tag
            assert _batch_key(st) == _batch_key(ref), tag


def test_batch_forced_and_deep():
    """Forced schedules over a grid, and a 3000-vertex path (several launches of 64 steps)."""
    grid = gen.grid2d(61, 53)
    gg = upload(grid)
    srcs = [0] + [int(x) for x in gen.sample_sources(grid, 20, seed=41)]
    want = _rows(grid, srcs)
    for sc in ([PUSH, PULL] * 70, [PULL, PULL, PUSH] * 50, [PUSH, PUSH, PULL] * 50):
        tag = "grid forced %s" % "".join(str(x) for x in sc[:6])
        _say(tag)
        d, st = _batch(gg, srcs, dobfs.make_options("full", forced_dirs=sc, persistent=True))
        assert np.array_equal(d, want), tag
        dirs = [x["dir"] for x in dobfs.stats_levels(st)]
        assert dirs == sc[: len(dirs)], tag
    dobfs.graph_destroy(gg)
    V = 3000
    path = gen.from_edges(V, np.arange(V - 1), np.arange(1, V), directed=False, name="path3000")
    gp = upload(path)
    srcs = [0, V - 1, V // 2]
    want = _rows(path, srcs)
    for mode in ("full", "push_only"):
        _say("path3000 batch", mode)
        d, st = _batch(gp, srcs, dobfs.make_options(mode, time_kernels=True, persistent=True))
        assert np.array_equal(d, want), mode
        lv = dobfs.stats_levels(st)
        assert len(lv) == V, mode
        assert all(x["ms_main"] > 0 for x in lv), mode
    dobfs.graph_destroy(gp)


def test_batch_barrier_wait_gives_up_and_recovers(graphs):
    hg, g = graphs["rmat14"]
    srcs = [int(x) for x in gen.sample_sources(hg, 64, seed=43)]
    os.environ["DOBFS_SPIN_LIMIT"] = "0"
    try:
        with pytest.raises(dobfs.DobfsError) as e:
            _batch(g, srcs, dobfs.make_options("full", persistent=True))
        assert e.value.status == dobfs.ERR_INTERNAL and "barrier" in str(e.value)
    finally:
        del os.environ["DOBFS_SPIN_LIMIT"]
    d, st = _batch(g, srcs, dobfs.make_options("full", persistent=True))
    assert np.array_equal(d, _rows(hg, srcs)), "after a given-up wait"
