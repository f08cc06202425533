"""The allocation-free single-source call (dobfs_bfs_static) through the C ABI, against
dobfs_bfs on the same inputs: depths equal (and equal to the oracle's), parents valid, and in
the pull-only mode (deterministic first-hit parents) parents equal too. Two calls in a row,
the second on a smaller graph, share the device's static scratch; the call allocates no
device memory; graphs beyond the scratch and options it cannot serve are refused."""
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

MODES = ["full", "push_only", "pull_only", "pull_masked_ee"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _static(g, s, opt, stats=None):
    dev = torch.device("cuda", g.device)
    depth = torch.full((g.V,), -7, dtype=torch.int32, device=dev)
    parent = torch.full((g.V,), -7, dtype=torch.int32, device=dev)
    dobfs.bfs_static(g, s, depth, parent, opt, stats=stats)
    torch.cuda.synchronize()
    return depth.cpu().numpy(), parent.cpu().numpy()


def _compare(hg, g, s, mode, heur=dobfs.HEUR_RATIO, alpha=0.01, beta=0.01, tag=""):
    opt = dobfs.make_options(mode, heur, alpha, beta)
    r = BfsRunner(g)
    st_ref = r.run(s, opt=opt)
    d_ref, p_ref = r.result()
    ref_levels, ref_reached, ref_edges = st_ref.levels, st_ref.reached, st_ref.edges_g500
    st = dobfs.make_stats(256)
    d, p = _static(g, s, opt, stats=st)
    tag = "%s source %d mode %s" % (tag, s, mode)
    assert np.array_equal(d, d_ref), "%s: %d depths differ from dobfs_bfs" % (tag, int((d != d_ref).sum()))
    want, _ = oracle.bfs(hg, s)
    assert np.array_equal(d, want), tag
    code, at = oracle.validate(hg, s, d, p)
    assert code == 0, "%s: parent check %d failed at %d" % (tag, code, at)
    if mode == "pull_only":
        assert np.array_equal(p, p_ref), tag
    assert (st.levels, st.reached, st.edges_g500) == (ref_levels, ref_reached, ref_edges), tag
    assert st.ms_total == 0.0
    lv, lv_ref = dobfs.stats_levels(st), r.levels()
    assert [(x["dir"], x["nf"], x["n_new"]) for x in lv] == [(x["dir"], x["nf"], x["n_new"]) for x in lv_ref]


def test_two_calls_second_smaller():
    big = gen.rmat(16, 16, seed=1)
    small = gen.rmat(10, 16, seed=1)
    gb, gs = upload(big, hubs_first=True), upload(small)
    sb = gen.max_degree_vertex(big)
    ss = int(gen.sample_sources(small, 1, seed=3)[0])
    for mode in MODES:
        _say("static vs dobfs_bfs:", mode)
        _compare(big, gb, sb, mode, dobfs.HEUR_EDGES, 1 / 14, 1 / 24, "rmat16")
        _compare(small, gs, ss, mode, tag="rmat10")
    dobfs.graph_destroy(gb)
    dobfs.graph_destroy(gs)


def test_deep_and_ragged():
    """Many batches of levels (a long path of a grid) and a ragged last bitmap word."""
    hg = gen.grid2d(61, 53)
    g = upload(hg)
    _compare(hg, g, 0, "full", tag="grid61x53")
    _compare(hg, g, hg.V - 1, "push_only", tag="grid61x53")
    dobfs.graph_destroy(g)


def test_no_device_allocation():
    hg = gen.rmat(14, 16, seed=1)
    g = upload(hg)
    s = gen.max_degree_vertex(hg)
    dev = torch.device("cuda", g.device)
    depth = torch.empty(g.V, dtype=torch.int32, device=dev)
    parent = torch.empty(g.V, dtype=torch.int32, device=dev)
    opt = dobfs.make_options("full")
    dobfs.bfs_static(g, s, depth, parent, opt)  # first call on the device: resolves the scratch
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(g.device)
    for _ in range(3):
        dobfs.bfs_static(g, s, depth, parent, opt)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info(g.device)
    assert free1 == free0, "device memory in use changed by %d bytes" % (free0 - free1)
    assert np.array_equal(depth.cpu().numpy(), oracle.bfs(hg, s)[0])
    dobfs.graph_destroy(g)


def test_refusals():
    # 2^23 vertices need 16 * 2^23 bytes of lists: beyond the static scratch
    V = 1 << 23
    ptr = np.zeros(V + 1, dtype=np.int32)
    empty = np.zeros(0, dtype=np.int32)
    g = dobfs.graph_upload(V, 0, ptr, empty, ptr, empty)
    dev = torch.device("cuda", g.device)
    depth = torch.empty(V, dtype=torch.int32, device=dev)
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_static(g, 0, depth)
    assert e.value.status == dobfs.ERR_INVALID_ARG and "static scratch" in str(e.value)
    dobfs.graph_destroy(g)
    hg = gen.rmat(10, 16, seed=1)
    g = upload(hg)
    depth = torch.empty(g.V, dtype=torch.int32, device=dev)
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_static(g, 0, depth, opt=dobfs.make_options("push_sort"))
    assert e.value.status == dobfs.ERR_UNSUPPORTED
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_static(g, 0, depth, opt=dobfs.make_options("full", time_kernels=True))
    assert e.value.status == dobfs.ERR_UNSUPPORTED
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.bfs_static(g, g.V, depth)
    assert e.value.status == dobfs.ERR_INVALID_ARG
    dobfs.graph_destroy(g)
