"""The direction-rule autotuner on the GPU: it times every candidate, returns the fastest, and
the tuned rule leaves depths unchanged."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1804_03327_amd import autotune, dobfs  # noqa: E402
from paper_1804_03327_amd.helpers import BfsRunner, upload  # noqa: E402


def test_tune_single_and_batch():
    hg = gen.rmat(14, 16, seed=1)
    g = upload(hg)
    srcs = [int(x) for x in gen.sample_sources(hg, 8, seed=3)]
    res = autotune.tune_single(g, srcs, reps=1)
    assert len(res["table"]) == len(autotune.candidates())
    assert res["ms"] == min(r[3] for r in res["table"]) and res["ms"] > 0
    r = BfsRunner(g)
    for s in srcs[:3]:
        r.run(s, heuristic=res["heuristic"], alpha=res["alpha"], beta=res["beta"])
        d, p = r.result()
        assert np.array_equal(d, oracle.bfs(hg, s)[0])
        assert oracle.validate(hg, s, d, p)[0] == 0
    rb = autotune.tune_batch(g, srcs, reps=1)
    assert rb["ms"] == min(r[3] for r in rb["table"])
    assert autotune.describe(rb).split()[0] in ("edges", "ratio")


@pytest.mark.parametrize("sched", [
    {"pull_mid": 4}, {"pull_mid": 1 << 20}, {"bitmap_rows": 0}, {"bitmap_rows": 4096},
    {"local_unit": 1}, {"local_unit": 256}, {"local_unit": 37}, {"local_chunks": 1}, {"local_chunks": 1 << 20},
    {"pull_mid": 8, "bitmap_rows": 128, "local_unit": 64, "local_chunks": 2},
])
def test_schedule_settings_keep_results(sched):
    """Every schedule setting, at the ends of its range and inside it: depths exact, parents
    valid and first-hit on pull levels, the oracle's level sizes; the pull's check count does
    not depend on where the wave takes over."""
    graphs = [gen.rmat(14, 16, seed=1), gen.lattice3d(37, 0.05, seed=3), gen.grid2d(61, 53)]
    for hg in graphs:
        g = upload(hg)
        r = BfsRunner(g)
        for s in [gen.max_degree_vertex(hg)] + [int(x) for x in gen.sample_sources(hg, 2, seed=6)]:
            want, _ = oracle.bfs(hg, s)
            fp = oracle.first_parent(hg, want, s)
            for mode in ("full", "push_only", "pull_only", "pull_masked"):
                tag = "%s src=%d %s %s" % (hg.name, s, mode, sched)
                r.run(s, mode=mode)
                ref = [(x["dir"], x["nf"], x["n_new"], x["edges"]) for x in r.levels()]
                r.run(s, opt=dobfs.make_options(mode, sched=sched))
                d, p = r.result()
                assert np.array_equal(d, want), tag
                assert oracle.validate(hg, s, d, p)[0] == 0, tag
                lv = r.levels()
                pulled = np.zeros(hg.V, dtype=bool)
                for L, row in enumerate(lv):
                    if row["dir"] == dobfs.DIR_PULL:
                        pulled |= want == L + 1
                assert np.array_equal(p[pulled], fp[pulled]), tag
                assert [x["nf"] for x in lv] == oracle.level_sizes(want), tag
                if mode == "pull_only":
                    assert [(x["dir"], x["nf"], x["n_new"], x["edges"]) for x in lv] == ref, tag
        dobfs.graph_destroy(g)


def test_schedule_settings_refused():
    hg = gen.rmat(10, 16, seed=1)
    g = upload(hg)
    r = BfsRunner(g)
    for bad in ({"pull_mid": 3}, {"pull_mid": (1 << 20) + 1}, {"bitmap_rows": -1}, {"bitmap_rows": 4097},
                {"local_unit": -1}, {"local_unit": 257}, {"local_chunks": -2}):
        with pytest.raises(dobfs.DobfsError) as e:
            r.run(0, opt=dobfs.make_options("full", sched=bad))
        assert e.value.status == dobfs.ERR_INVALID_ARG, bad
    dobfs.graph_destroy(g)


def test_tune_schedule():
    hg = gen.rmat(14, 16, seed=1)
    g = upload(hg)
    srcs = [int(x) for x in gen.sample_sources(hg, 6, seed=3)]
    res = autotune.tune_schedule(g, srcs, reps=2, rule=(dobfs.HEUR_EDGES, 1 / 14, 1 / 24))
    assert set(res["sched"]) == set(autotune.SCHED_GRID)
    assert all(res["sched"][k] in v for k, v in autotune.SCHED_GRID.items())
    assert set(res["steps"]) == set(autotune.SCHED_GRID)
    assert res["ms"] > 0 and res["default_ms"] > 0
    r = BfsRunner(g)
    opt = dobfs.make_options("full", res["heuristic"], res["alpha"], res["beta"], sched=res["sched"])
    for s in srcs[:3]:
        r.run(s, opt=opt)
        d, p = r.result()
        assert np.array_equal(d, oracle.bfs(hg, s)[0])
        assert oracle.validate(hg, s, d, p)[0] == 0
    assert "pull_mid=" in autotune.describe(res)
