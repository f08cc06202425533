"""GPU tests of the query server (dobfs_server_*), through the C ABI.

Each query's depths must be the same whether it runs alone (dobfs_bfs) or inside the
server's mix of batches, and equal the oracle's; batches must really form and overlap on
the device; the memory budget must bound the batches in flight and their width."""
import random
import sys
import time

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


@pytest.fixture(scope="module")
def graphs():
    rng = np.random.default_rng(9)
    V = 50_021
    src = rng.integers(0, V, 6 * V)
    dst = (src + rng.zipf(1.7, 6 * V)) % V
    hgs = [gen.rmat(10, 16, seed=1), gen.rmat(14, 16, seed=1), gen.grid2d(61, 53),
           gen.from_edges(V, src, dst, directed=True, name="directed50021")]
    out = []
    for hg in hgs:
        _say("upload", hg.name, hg.V, hg.nnz)
        out.append((hg, upload(hg)))
    return out


def _result_buffer(n, fill=-7):
    """A query's result buffer. torch fills it on its current stream; the server's slots run on
    streams of their own that are not ordered after that one, so the fill must be complete
    before the buffer is submitted, or it may land on top of the server's result."""
    t = torch.full((n,), fill, dtype=torch.int32, device="cuda")
    torch.cuda.current_stream().synchronize()
    return t


def _alone(g, source):
    r = BfsRunner(g, with_parent=False)
    r.run(source)
    return r.result()[0]


def _batches(infos):
    """Group query infos into batches: same graph, start and end time."""
    b = {}
    for i in infos:
        b.setdefault((i["graph"], i["t_start_ms"], i["t_done_ms"]), []).append(i)
    return b


def test_server_mix_equals_alone(graphs):
    rnd = random.Random(4)
    srv = dobfs.Server([g for _, g in graphs], slots=2, max_batch=64)
    queries = []
    for n in range(400):
        gi = rnd.randrange(len(graphs))
        hg, g = graphs[gi]
        s = int(gen.sample_sources(hg, 1, seed=1000 + n)[0])
        depth = _result_buffer(g.V)
        queries.append((gi, s, depth, srv.submit(gi, s, depth)))
        if rnd.random() < 0.3:
            time.sleep(rnd.expovariate(1 / 0.002))  # bursts with pauses of ~2 ms on average
    infos = [srv.wait(q[3]) for q in queries]
    srv.close()
    assert all(i["status"] == dobfs.OK for i in infos)
    for (gi, s, depth, _), info in zip(queries, infos):
        assert (info["graph"], info["source"]) == (gi, s)
        assert info["t_submit_ms"] <= info["t_start_ms"] <= info["t_done_ms"]
    # each result equals the same query run alone, and the oracle on a sample
    torch.cuda.synchronize()
    for k, (gi, s, depth, _) in enumerate(queries):
        hg, g = graphs[gi]
        d = depth.cpu().numpy()
        alone = _alone(g, s)
        if not np.array_equal(d, alone):
            want = oracle.bfs(hg, s)[0]
            raise AssertionError(
                "query %d (graph %s, source %d, batch of %d) differs from alone: the mix %s the oracle "
                "(%d depths differ), alone %s it (%d differ); first differing vertices %s" % (
                    k, hg.name, s, infos[k]["batch_size"],
                    "matches" if np.array_equal(d, want) else "differs from", int((d != want).sum()),
                    "matches" if np.array_equal(alone, want) else "differs from", int((alone != want).sum()),
                    [(int(v), int(d[v]), int(alone[v]), int(want[v])) for v in np.nonzero(d != alone)[0][:6]]))
        if k % 20 == 0:
            assert np.array_equal(d, oracle.bfs(hg, s)[0]), "query %d differs from the oracle" % k
    # batching happened, and batches ran side by side on the device
    b = _batches(infos)
    assert max(len(v) for v in b.values()) > 1, "no query shared a traversal"
    spans = sorted((k[1], k[2]) for k in b)
    overlap = any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    _say("batches", len(b), "largest", max(len(v) for v in b.values()), "overlap", overlap)
    assert overlap, "no two batches were in flight at once"


def test_one_buffer_across_graphs_and_kinds(graphs):
    """What the server's pool does to a workspace: one buffer serves single-source and
    multi-source traversals of different graphs and widths in turn, each starting on what the
    one before left there. Every result must equal the oracle's."""
    rnd = random.Random(12)
    nbytes = max(max(dobfs.bfs_workspace_bytes(g), dobfs.bfs_batch_workspace_bytes(g, 64)) for _, g in graphs)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    want = {}
    for it in range(48):
        gi = it % len(graphs) if it < 24 else rnd.randrange(len(graphs))
        hg, g = graphs[gi]
        k = [1, 2, 5, 17, 64, 1][it % 6]
        srcs = [int(x) for x in gen.sample_sources(hg, k, seed=3000 + it)]
        depth = torch.full((k * g.V,), -7, dtype=torch.int32, device="cuda")
        if k == 1:
            dobfs.bfs(g, srcs[0], depth, None, None, ws)
        else:
            dobfs.bfs_batch(g, srcs, depth, workspace=ws)
        d = depth.cpu().numpy().reshape(k, g.V)
        for b, s in enumerate(srcs):
            if (gi, s) not in want:
                want[(gi, s)] = oracle.bfs(hg, s)[0]
            bad = int((d[b] != want[(gi, s)]).sum())
            assert bad == 0, "call %d (graph %s, %d sources, row %d, source %d): %d depths differ" % (
                it, hg.name, k, b, s, bad)


def _run_bytes(g, k):
    """Workspace a server batch of k takes: a batch of one runs the single-source call."""
    return dobfs.bfs_workspace_bytes(g) if k == 1 else dobfs.bfs_batch_workspace_bytes(g, k)


def test_server_memory_budget(graphs):
    hg, g = graphs[1]
    need8 = dobfs.bfs_batch_workspace_bytes(g, 8)
    # room for one 8-source batch: batches are cut to 8, and the batches in flight at any time
    # never hold more workspace than the budget (a lone query's smaller one may run beside
    # another)
    # the device memory a server holds is its pool of the budget's size, whatever the slots and
    # batch widths would want (up to HIP's allocation granularity and its streams' own memory)
    slack = 16 << 20
    for budget in (need8, 256 << 20):
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        probe = dobfs.Server([g], slots=3, max_batch=64, mem_budget=budget)
        used = free0 - torch.cuda.mem_get_info()[0]
        probe.close()
        assert budget - slack <= used <= budget + slack, "server holds %d bytes for a budget of %d" % (used, budget)
    srv = dobfs.Server([g], slots=3, max_batch=64, mem_budget=need8)
    qs = []
    for n in range(120):
        s = int(gen.sample_sources(hg, 1, seed=2000 + n)[0])
        depth = _result_buffer(g.V)
        qs.append((s, depth, srv.submit(0, s, depth)))
    infos = [srv.wait(q[2]) for q in qs]
    srv.close()
    b = _batches(infos)
    assert max(len(v) for v in b.values()) <= 8
    spans = sorted((k[1], k[2], _run_bytes(g, len(v))) for k, v in b.items())
    for t0, _, _ in spans:  # the bytes in flight at every batch start
        held = sum(nb for s0, s1, nb in spans if s0 <= t0 < s1)
        assert held <= need8, "batches in flight hold %d bytes, budget %d" % (held, need8)
    for s, depth, _ in qs:
        assert np.array_equal(depth.cpu().numpy(), _alone(g, s))


def test_server_budget_below_one_source(graphs):
    hg, g = graphs[1]
    srv = dobfs.Server([g], slots=1, mem_budget=1024)
    depth = _result_buffer(g.V, 0)
    qid = srv.submit(0, 0, depth)
    with pytest.raises(dobfs.DobfsError) as e:
        srv.wait(qid)
    assert e.value.status == dobfs.ERR_OUT_OF_MEMORY
    srv.close()


def test_server_destroy_answers_queued(graphs):
    hg, g = graphs[0]
    srv = dobfs.Server([g], slots=1, max_batch=4)
    qs = []
    for s in range(0, 200, 7):
        depth = _result_buffer(g.V)
        qs.append((s, depth, srv.submit(0, s, depth)))
    srv.close()  # returns after every submitted query is answered
    for s, depth, _ in qs:
        assert np.array_equal(depth.cpu().numpy(), _alone(g, s))


def test_server_errors(graphs):
    hg, g = graphs[0]
    srv = dobfs.Server([g])
    depth = _result_buffer(g.V, 0)
    for gi, s in ((1, 0), (-1, 0), (0, g.V), (0, -1)):
        with pytest.raises(dobfs.DobfsError) as e:
            srv.submit(gi, s, depth)
        assert e.value.status == dobfs.ERR_INVALID_ARG
    with pytest.raises(dobfs.DobfsError) as e:
        srv.wait(12345)
    assert e.value.status == dobfs.ERR_INVALID_ARG
    srv.close()
    with pytest.raises(dobfs.DobfsError):
        dobfs.Server([g], slots=0)
    with pytest.raises(dobfs.DobfsError):
        dobfs.Server([g], max_batch=65)
    with pytest.raises(dobfs.DobfsError) as e:
        dobfs.Server([g], opt=dobfs.make_options("pull_masked"))
    assert e.value.status == dobfs.ERR_UNSUPPORTED


def test_long_graph_keeps_a_slot_free(graphs):
    """With two slots, batches of a graph whose traversals take more than 2 ms (a 400 x 400
    grid, about 800 levels) never hold both slots once that is known: the other graph's
    queries find a free slot."""
    hg_long = gen.grid2d(400, 400)
    g_long = upload(hg_long)
    hg, g = graphs[1]
    srv = dobfs.Server([g_long, g], slots=2, max_batch=1)
    d0 = _result_buffer(g_long.V)
    first = srv.wait(srv.submit(0, 0, d0))  # its service time is now known
    assert first["t_done_ms"] - first["t_start_ms"] > 2.0
    qs = []
    for n in range(8):
        s = int(gen.sample_sources(hg_long, 1, seed=3000 + n)[0])
        depth = _result_buffer(g_long.V)
        qs.append((0, s, depth, srv.submit(0, s, depth)))
        for m in range(5):
            s = int(gen.sample_sources(hg, 1, seed=4000 + 5 * n + m)[0])
            depth = _result_buffer(g.V)
            qs.append((1, s, depth, srv.submit(1, s, depth)))
    infos = [srv.wait(q[3]) for q in qs]
    srv.close()
    spans = sorted((i["t_start_ms"], i["t_done_ms"]) for i in infos if i["graph"] == 0)
    for a, b in zip(spans, spans[1:]):
        assert b[0] >= a[1], "two long batches ran at once: %s and %s" % (a, b)
    for (gi, s, depth, _), info in zip(qs, infos):
        assert info["status"] == dobfs.OK
        gg = g_long if gi == 0 else g
        assert np.array_equal(depth.cpu().numpy(), _alone(gg, s))
    dobfs.graph_destroy(g_long)


def test_long_graph_batches_only_from_eight_queued(graphs):
    """Queries of a graph known to be long (a 400 x 400 grid) run one per slot while fewer than 8
    are queued, and as one multi-source batch once 8 or more are: 5 queries submitted while a
    query of the graph occupies the only slot run alone, each; 12 run as batches of 8 or more
    (or the leftover singles). Every depth vector equals the query run alone."""
    hg = gen.grid2d(400, 400)
    g = upload(hg)
    srv = dobfs.Server([g], slots=1, max_batch=64)
    d0 = _result_buffer(g.V)
    first = srv.wait(srv.submit(0, 0, d0))  # its service time is now known
    assert first["t_done_ms"] - first["t_start_ms"] > 2.0
    for count, seed in ((5, 5000), (12, 6000)):
        blocker = _result_buffer(g.V)
        hb = srv.submit(0, hg.V - 1, blocker)  # holds the slot while the others queue up
        qs = []
        for n in range(count):
            s = int(gen.sample_sources(hg, 1, seed=seed + n)[0])
            depth = _result_buffer(g.V)
            qs.append((s, depth, srv.submit(0, s, depth)))
        srv.wait(hb)
        infos = [srv.wait(q[2]) for q in qs]
        sizes = [i["batch_size"] for i in infos]
        if count < 8:
            assert sizes == [1] * count, sizes
        else:
            assert max(sizes) >= 8 and all(k >= 8 or k == 1 for k in sizes), sizes
        for (s, depth, _), info in zip(qs, infos):
            assert info["status"] == dobfs.OK
            assert np.array_equal(depth.cpu().numpy(), _alone(g, s))
    srv.close()
    dobfs.graph_destroy(g)


def test_two_streams_overlap_on_device():
    """Two deep traversals (a 400 x 400 grid, about 800 levels of small kernels) from two host
    threads on two streams take much less than the two one after the other: their kernels run
    at the same time on the device. Depths stay exact."""
    import threading
    hg = gen.grid2d(400, 400)
    g = upload(hg)
    srcs = [0, hg.V - 1]
    runners = [BfsRunner(g, with_parent=False) for _ in srcs]
    streams = [torch.cuda.Stream() for _ in srcs]
    for r, s, st in zip(runners, srcs, streams):
        r.run(s, stream=st)
    torch.cuda.synchronize()

    def one(i):
        runners[i].run(srcs[i], stream=streams[i])

    best_seq, best_par = 1e9, 1e9
    for _ in range(3):
        t = time.perf_counter()
        one(0)
        one(1)
        torch.cuda.synchronize()
        best_seq = min(best_seq, time.perf_counter() - t)
        ths = [threading.Thread(target=one, args=(i,)) for i in range(2)]
        t = time.perf_counter()
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        torch.cuda.synchronize()
        best_par = min(best_par, time.perf_counter() - t)
    _say("two grid traversals: one after the other %.2f ms, at once %.2f ms" % (1e3 * best_seq, 1e3 * best_par))
    assert best_par < 0.8 * best_seq
    for r, s in zip(runners, srcs):
        assert np.array_equal(r.result()[0], oracle.bfs(hg, s)[0])
    dobfs.graph_destroy(g)
