"""GPU parity at the full sizes of the benchmarked and configured workloads, in the launch
configuration the benchmark times (in-neighbours uploaded hubs-first, mode full, edge-count
rule with alpha = 1/14, beta = 1/24, library-owned workspace, current stream).

Every depth vector is compared with the oracle's over all vertices and every parent vector
passes the validator; under the edge-count rule the direction sequence is the oracle's; the
multi-source launch is checked on sampled rows."""
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


BENCH_OPT = dict(mode="full", heuristic=dobfs.HEUR_EDGES, alpha=1 / 14, beta=1 / 24)


def _single(hg, sources, opts, hubs_first=False):
    g = upload(hg, hubs_first=hubs_first)
    r = BfsRunner(g)
    for s in sources:
        want, _ = oracle.bfs(hg, s)
        for o in opts:
            tag = "%s source %d %s" % (hg.name, s, o)
            _say(tag)
            r.run(s, **o)
            d, p = r.result()
            bad = int((d != want).sum())
            assert bad == 0, "%s: %d depths differ" % (tag, bad)
            code, at = oracle.validate(hg, s, d, p)
            assert code == 0, "%s: parent check %d failed at %d" % (tag, code, at)
            if o.get("heuristic") == dobfs.HEUR_EDGES:
                dirs = [x["dir"] for x in r.levels()]
                assert dirs == oracle.schedule_edges(hg, want, o["alpha"], o["beta"]), tag
    dobfs.graph_destroy(g)


def test_rmat22_single_source():
    hg = gen.rmat(22, 16, seed=1)
    srcs = [int(x) for x in gen.sample_sources(hg, 64, seed=2)]
    _single(hg, [srcs[0], srcs[63]], [BENCH_OPT, dict(mode="full")], hubs_first=True)
    _single(hg, [srcs[1]], [BENCH_OPT])


def test_lattice256_single_source():
    hg = gen.lattice3d(256, 0.05, seed=3)
    assert hg.nnz == 95_256_576
    srcs = [int(x) for x in gen.sample_sources(hg, 16, seed=4)]
    _single(hg, [srcs[0]], [dict(mode="full"), BENCH_OPT])


def test_grid2048_single_source():
    hg = gen.grid2d(2048, 2048)
    assert hg.nnz == 16_769_024
    _single(hg, [0], [dict(mode="full")])


def test_rmat20_multi_source_rows():
    hg = gen.rmat(20, 16, seed=1)
    srcs = [int(x) for x in gen.sample_sources(hg, 64, seed=5)]
    g = upload(hg)
    depth = torch.full((64 * g.V,), -7, dtype=torch.int32, device="cuda")
    dobfs.bfs_batch(g, srcs, depth, opt=dobfs.make_options(**BENCH_OPT))
    rows = depth.cpu().numpy().reshape(64, g.V)
    for b in (0, 21, 42, 63):
        _say("rmat20 row", b)
        want, _ = oracle.bfs(hg, srcs[b])
        assert np.array_equal(rows[b], want), "row %d (source %d) differs" % (b, srcs[b])
    dobfs.graph_destroy(g)
