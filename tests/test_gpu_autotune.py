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
