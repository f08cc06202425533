"""Pins of the CPU oracle against things other than itself: brute force over tiny graphs
(Boolean matrix powers), a library shortest-path routine, closed forms, the paper's worked
example (Figure 3 text) and printed tables, and self-tests of the validator."""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.csgraph

import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _graph_from_dense(A, name="dense"):
    src, dst = np.nonzero(A)
    return gen.from_edges(A.shape[0], src, dst, directed=True, keep_self_loops=True, name=name)


def _depth_by_matrix_powers(A, s):
    """Hop distance as the first k with a length-k walk s->v: row s of A^k (Boolean)."""
    n = A.shape[0]
    depth = np.full(n, -1, dtype=np.int64)
    walk = np.zeros(n, dtype=bool)
    walk[s] = True  # row s of A^0
    for k in range(n):
        newly = walk & (depth < 0)
        depth[newly] = k
        walk = (walk.astype(np.int64) @ A.astype(np.int64)) > 0  # row s of A^(k+1)
    return depth


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_bfs_all_directed_graphs_bruteforce(n):
    """Every directed graph on n <= 4 vertices (self-loops included for n <= 3), every source."""
    pairs = [(i, j) for i in range(n) for j in range(n) if (n <= 3 or i != j)]
    for bits in range(1 << len(pairs)):
        A = np.zeros((n, n), dtype=bool)
        for k, (i, j) in enumerate(pairs):
            if bits >> k & 1:
                A[i, j] = True
        g = _graph_from_dense(A)
        for s in range(n):
            depth, parent = oracle.bfs(g, s)
            assert np.array_equal(depth, _depth_by_matrix_powers(A, s)), (A, s)
            assert oracle.validate(g, s, depth, parent) == (0, -1)


def test_bfs_all_undirected_graphs_n5():
    n = 5
    pairs = list(itertools.combinations(range(n), 2))
    for bits in range(1 << len(pairs)):
        A = np.zeros((n, n), dtype=bool)
        for k, (i, j) in enumerate(pairs):
            if bits >> k & 1:
                A[i, j] = A[j, i] = True
        g = _graph_from_dense(A)
        for s in range(n):
            depth, parent = oracle.bfs(g, s)
            assert np.array_equal(depth, _depth_by_matrix_powers(A, s))
            assert oracle.validate(g, s, depth, parent)[0] == 0


@pytest.mark.parametrize("seed", range(12))
def test_bfs_random_vs_library_shortest_path(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 65))
    A = rng.random((n, n)) < rng.uniform(0.01, 0.2)
    g = _graph_from_dense(A)
    dist = scipy.sparse.csgraph.shortest_path(scipy.sparse.csr_matrix(A.astype(np.float64)),
                                              directed=True, unweighted=True)
    for s in range(n):
        depth, parent = oracle.bfs(g, s)
        want = np.where(np.isinf(dist[s]), -1, dist[s]).astype(np.int64)
        assert np.array_equal(depth, want)
        assert oracle.validate(g, s, depth, parent)[0] == 0


def test_directed_orientation_pin():
    """Edges 0->1->2: from 0 depths [0,1,2]; from 2 nothing else is reachable."""
    g = gen.from_edges(3, [0, 1], [1, 2], directed=True)
    assert oracle.bfs(g, 0)[0].tolist() == [0, 1, 2]
    assert oracle.bfs(g, 2)[0].tolist() == [-1, -1, 0]
    assert oracle.bfs(g, 1)[0].tolist() == [-1, 0, 1]
    # A^T x with x = e_0 gives the out-neighbours of 0
    assert oracle.mxv(g, [1, 0, 0]).tolist() == [0, 1, 0]
    assert oracle.mxv(g, [0, 1, 0]).tolist() == [0, 0, 1]


# ---------------------------------------------------------------- closed forms
def _path(n):
    return gen.from_edges(n, np.arange(n - 1), np.arange(1, n))


@pytest.mark.parametrize("n,s", [(1, 0), (2, 1), (10, 0), (10, 4), (1000, 377)])
def test_path(n, s):
    d, p = oracle.bfs(_path(n), s)
    assert np.array_equal(d, np.abs(np.arange(n) - s))
    assert all(p[v] == v + (1 if v < s else -1) for v in range(n) if v != s)


@pytest.mark.parametrize("n,s", [(3, 0), (8, 3), (9, 8), (101, 50)])
def test_cycle(n, s):
    g = gen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    k = np.abs(np.arange(n) - s)
    assert np.array_equal(oracle.bfs(g, s)[0], np.minimum(k, n - k))


def test_directed_cycle():
    n = 9
    g = gen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n, directed=True)
    assert np.array_equal(oracle.bfs(g, 4)[0], (np.arange(n) - 4) % n)


def test_star_and_complete():
    n = 50
    star = gen.from_edges(n, np.zeros(n - 1, int), np.arange(1, n))
    assert np.array_equal(oracle.bfs(star, 0)[0], np.r_[0, np.ones(n - 1, int)])
    want = np.full(n, 2)
    want[0], want[7] = 1, 0
    assert np.array_equal(oracle.bfs(star, 7)[0], want)
    i, j = np.triu_indices(n, 1)
    K = gen.from_edges(n, i, j)
    d = oracle.bfs(K, 13)[0]
    assert d[13] == 0 and np.all(np.delete(d, 13) == 1)


def test_binary_tree():
    n = 2 ** 10 - 1
    v = np.arange(1, n)
    g = gen.from_edges(n, (v - 1) // 2, v)
    assert np.array_equal(oracle.bfs(g, 0)[0], np.floor(np.log2(np.arange(n) + 1)).astype(int))


def test_grid_and_lattice_l1():
    g = gen.grid2d(13, 7)
    s = 3 + 13 * 5
    x, y = np.arange(g.V) % 13, np.arange(g.V) // 13
    assert np.array_equal(oracle.bfs(g, s)[0], np.abs(x - 3) + np.abs(y - 5))
    n = 9
    L = gen.lattice3d(n, 0.0, seed=1)
    i = np.arange(L.V)
    c = [i % n, (i // n) % n, i // (n * n)]
    s = 2 + n * (7 + n * 4)
    assert np.array_equal(oracle.bfs(L, s)[0], np.abs(c[0] - 2) + np.abs(c[1] - 7) + np.abs(c[2] - 4))


def test_disconnected_components_and_isolated_source():
    g = gen.from_edges(7, [0, 1, 4], [1, 2, 5])
    assert oracle.bfs(g, 0)[0].tolist() == [0, 1, 2, -1, -1, -1, -1]
    assert oracle.bfs(g, 3)[0].tolist() == [-1, -1, -1, 0, -1, -1, -1]
    d, p = oracle.bfs(g, 6)
    assert p.tolist() == [-1] * 6 + [6]


def test_source_out_of_range():
    with pytest.raises(ValueError):
        oracle.bfs(_path(4), 4)
    with pytest.raises(ValueError):
        oracle.bfs(_path(4), -1)


def test_self_loops_and_duplicates_tolerated():
    g = gen.from_edges(4, [0, 0, 1, 1, 2], [0, 1, 2, 2, 3], directed=True, keep_self_loops=True,
                       keep_duplicates=True)
    d, p = oracle.bfs(g, 0)
    assert d.tolist() == [0, 1, 2, 3]
    assert oracle.validate(g, 0, d, p)[0] == 0


# ------------------------------------------------------------------ validator
def test_validator_rejects_corruptions():
    g = gen.rmat(8, 8, seed=3)
    s = gen.max_degree_vertex(g)
    d, p = oracle.bfs(g, s)
    assert oracle.validate(g, s, d, p)[0] == 0
    reached = np.nonzero((d > 0))[0]
    deep = reached[np.argmax(d[reached])]

    def code(dd, pp):
        return oracle.validate(g, s, dd, pp)[0]

    dd = d.copy(); dd[s] = 1
    assert code(dd, p) == 1
    pp = p.copy(); pp[s] = -1
    assert code(d, pp) == 1
    dd = d.copy(); dd[deep] = 0
    assert code(dd, p) == 2
    pp = p.copy(); pp[deep] = -1
    assert code(d, pp) == 3
    pp = p.copy(); pp[deep] = deep  # not an in-neighbour one level up
    assert code(d, pp) == 4
    # a vertex one level up but not adjacent
    cand = np.nonzero(d == d[deep] - 1)[0]
    nbrs = set(g.csc_rowind[g.csc_colptr[deep]:g.csc_colptr[deep + 1]].tolist())
    non_adj = [u for u in cand if u not in nbrs]
    if non_adj:
        pp = p.copy(); pp[deep] = non_adj[0]
        assert code(d, pp) == 4
    # too deep: shift one vertex's depth by +1 together with a fake parent chain
    dd = d.copy(); dd[deep] += 1
    assert code(dd, p) in (4, 5)
    # unreached but reachable
    dd, pp = d.copy(), p.copy()
    dd[deep], pp[deep] = -1, -1
    assert code(dd, pp) == 5


def test_validator_rejects_consistent_but_too_long_tree():
    """A parent chain that is valid edge by edge but not shortest: only the tightness
    check (every edge u->v has depth[v] <= depth[u] + 1) can reject it."""
    n = 6
    g = gen.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    depth = np.arange(n, dtype=np.int32)            # walk the cycle one way only
    parent = np.r_[0, np.arange(n - 1)].astype(np.int32)
    assert oracle.validate(g, 0, depth, parent) == (5, 5)
    d, p = oracle.bfs(g, 0)
    assert d.tolist() == [0, 1, 2, 3, 2, 1]
    # odd cycle: vertices 2 and 3 are adjacent and both at depth 2; a same-level parent
    # is an in-neighbour but not one level closer
    c5 = gen.from_edges(5, np.arange(5), (np.arange(5) + 1) % 5)
    d5, p5 = oracle.bfs(c5, 0)
    assert d5.tolist() == [0, 1, 2, 2, 1]
    p5[2] = 3
    assert oracle.validate(c5, 0, d5, p5) == (4, 2)


# -------------------------------------------------------------------- matvec
@pytest.mark.parametrize("seed", range(8))
def test_mxv_dense_definition(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 90))
    A = rng.random((n, n)) < 0.08
    g = _graph_from_dense(A)
    x = rng.random(n) < 0.3
    m = rng.random(n) < 0.5
    y0 = rng.random(n) < 0.5
    t = (A.T.astype(np.int64) @ x.astype(np.int64)) > 0
    assert np.array_equal(oracle.mxv(g, x).astype(bool), t)
    assert np.array_equal(oracle.mxv(g, x, m).astype(bool), t & m)
    assert np.array_equal(oracle.mxv(g, x, m, complement=True).astype(bool), t & ~m)
    assert np.array_equal(oracle.mxv(g, x, m, accum=True, y_old=y0).astype(bool), y0 | (t & m))
    assert np.array_equal(oracle.mxv(g, x, None, accum=True, y_old=y0).astype(bool), y0 | t)


def _fig3():
    with open(os.path.join(GOLDEN, "fig3_toy.json")) as f:
        fx = json.load(f)
    ids = {v: i for i, v in enumerate(fx["vertices"])}
    e = np.array([[ids[a], ids[b]] for a, b in fx["undirected_edges"]])
    g = gen.from_edges(len(ids), e[:, 0], e[:, 1])

    def vec(names):
        v = np.zeros(len(ids), dtype=np.uint8)
        v[[ids[x] for x in names]] = 1
        return v

    return fx, ids, g, vec


def test_fig3_worked_example():
    fx, ids, g, vec = _fig3()
    f, v = vec(fx["frontier"]), vec(fx["visited"])
    assert f[:4].tolist() == fx["frontier_values_of_first_four"]
    # push: children of the frontier combined by OR, then filtered by not(visited)
    assert np.array_equal(oracle.mxv(g, f), vec(fx["push_children_before_filter"]))
    assert np.array_equal(oracle.mxv(g, f, v, complement=True), vec(fx["next_after_filter"]))
    # pull starts from the unvisited vertices; with the visited vector as input (operand reuse)
    assert np.array_equal(1 - v, vec(fx["pull_start_unvisited"]))
    assert np.array_equal(oracle.mxv(g, v, v, complement=True), vec(fx["next_after_filter"]))
    # the BFS state of the figure is reached from A: frontier {B,C,D} after one level
    d, _ = oracle.bfs(g, ids["A"])
    assert np.array_equal((d == 1).astype(np.uint8), f)
    assert np.array_equal(((d >= 0) & (d <= 1)).astype(np.uint8), v)


# ----------------------------------------------------------- first-hit parents
def test_first_parent_is_first_in_stored_order():
    g = gen.rmat(9, 8, seed=5)
    s = gen.max_degree_vertex(g)
    d, _ = oracle.bfs(g, s)
    fp = oracle.first_parent(g, d, s)
    assert oracle.validate(g, s, d, fp)[0] == 0
    for v in np.nonzero(d > 0)[0][:200]:
        col = g.csc_rowind[g.csc_colptr[v]:g.csc_colptr[v + 1]]
        pos = np.nonzero(d[col] == d[v] - 1)[0]
        assert fp[v] == col[pos[0]]
        assert np.all(d[col[:pos[0]]] != d[v] - 1)


# ------------------------------------------------------- early-exit check counts
def test_pull_checks_complete_graph_closed_form():
    """K_n from s, level 0: column i (sorted) reaches s at position s (i > s) or s-1 (i < s)."""
    n = 40
    i, j = np.triu_indices(n, 1)
    K = gen.from_edges(n, i, j)
    for s in (0, 1, 17, n - 1):
        d, _ = oracle.bfs(K, s)
        assert oracle.pull_checks(K, d, 0) == s * s + (n - 1 - s) * (s + 1)


def test_pull_checks_bounds():
    """Between 'one check per row found' and the masked row-based work of Table 1."""
    g = gen.rmat(11, 16, seed=2)
    s = gen.max_degree_vertex(g)
    d, _ = oracle.bfs(g, s)
    indeg = g.in_degree()
    for L in range(int(d.max()) + 1):
        unvisited = ~((d >= 0) & (d <= L))
        k = oracle.pull_checks(g, d, L)
        found = int((d == L + 1).sum())
        assert found <= k <= int(indeg[unvisited].sum())
        assert oracle.table1_counts(g, mask=unvisited)["row_masked"] == int(indeg[unvisited].sum())
    # the path graph from one end: each unvisited row checks all its entries except
    # row L+1, which stops at its first entry (vertex L) and skips its second (L+2),
    # unless it is the last vertex and has no second entry
    p = _path(12)
    dp, _ = oracle.bfs(p, 0)
    for L in range(11):
        unvisited = np.arange(L + 1, 12)
        want = int(p.in_degree()[unvisited].sum()) - (1 if L + 1 < 11 else 0)
        assert oracle.pull_checks(p, dp, L) == want


# ---------------------------------------------------------------- work model
def test_table1_counts_small():
    # 0->1, 0->2, 1->2, 3->0
    g = gen.from_edges(4, [0, 0, 1, 3], [1, 2, 2, 0], directed=True)
    c = oracle.table1_counts(g, x=[1, 0, 0, 1], mask=[1, 0, 1, 0])
    assert c == {"row": 4, "row_masked": 1 + 2, "col": 2 + 1}
    c = oracle.table1_counts(g, mask=[1, 0, 1, 0], complement=True)
    assert c["row_masked"] == 1  # rows 1 and 3: in-degrees 1 and 0


def test_level_work_and_sizes():
    g = _path(6)
    d, _ = oracle.bfs(g, 0)
    assert oracle.level_sizes(d) == [1, 1, 1, 1, 1, 1]
    dirs = [oracle.PUSH] * 6
    rows = oracle.level_work(g, d, dirs)
    assert [r["edges"] for r in rows] == [1, 2, 2, 2, 2, 1]
    assert [r["n_new"] for r in rows] == [1, 1, 1, 1, 1, 0]


# ---------------------------------------------------------- direction schedule
def test_schedule_hand_example():
    """Section 6.3 rule on a scale-22-like level profile (alpha*M = 41943.04)."""
    V = 4194304
    sizes = [1, 10, 100000, 2000000, 50000, 100, 1]
    P, Q = oracle.PUSH, oracle.PULL
    assert oracle.schedule(sizes, V) == [P, P, Q, Q, Q, P, P]
    # frontier growing but still under 1% of M: stays in push
    assert oracle.schedule([1, 40000, 41943, 0], V) == [P, P, P, P]
    assert oracle.schedule([1, 40000, 41944, 0], V) == [P, P, Q, P]


def test_schedule_needs_trend():
    V = 1000
    P, Q = oracle.PUSH, oracle.PULL
    # big but shrinking frontier does not trigger push -> pull
    assert oracle.schedule([500, 400, 300, 0], V) == [P, P, P, P]
    # pull keeps pulling while the frontier is large or growing
    assert oracle.schedule([1, 50, 60, 5, 0], V) == [P, Q, Q, P, P]


def test_schedule_edges_hand_example():
    """Beamer's rule of Section 6.3 on a star 0-{1..8} with a tail 8-9 (undirected, 18
    entries), from vertex 0. Level 0 finds 1..8: m_f = 7*1 + 2 = 9 out-edges, and only vertex
    9 stays unvisited, m_u = 1. Level 1 finds 9 (nnz(f) = 1), level 2 nothing."""
    hg = gen.from_edges(10, [0] * 8 + [8], list(range(1, 9)) + [9])
    d, _ = oracle.bfs(hg, 0)
    assert d.tolist() == [0] + [1] * 8 + [2]
    P, Q = oracle.PUSH, oracle.PULL
    # 9 > alpha * 1 switches to pull; 1 < beta * 10 needs beta > 0.1, 0 < beta * 10 any beta > 0
    assert oracle.schedule_edges(hg, d, alpha=1 / 14, beta=1 / 24) == [P, Q, Q]
    assert oracle.schedule_edges(hg, d, alpha=1 / 14, beta=0.2) == [P, Q, P]
    # alpha = 10: 9 > 10 fails; after level 1, m_f = outdeg(9) = 1 > 10 * m_u = 0: pull
    assert oracle.schedule_edges(hg, d, alpha=10.0, beta=1 / 24) == [P, P, Q]
    # alpha = 9 exactly: 9 > 9 fails (strict)
    assert oracle.schedule_edges(hg, d, alpha=9.0, beta=1 / 24) == [P, P, Q]
    assert oracle.schedule_edges(hg, d, alpha=8.99, beta=1 / 24)[:2] == [P, Q]


def test_schedule_edges_directed_counts():
    """On a directed graph m_f counts out-edges and m_u in-edges: 0->1, 0->2, 1->3, 2->3,
    4->3, 4->1 (vertex 4 unreachable from 0). Level 0 finds {1, 2}: m_f = 2; unvisited
    {3, 4}, m_u = indeg 3 + indeg 0 = 3. Level 1 finds {3}: m_f = 0, m_u = 0."""
    hg = gen.from_edges(5, [0, 0, 1, 2, 4, 4], [1, 2, 3, 3, 3, 1], directed=True)
    d, _ = oracle.bfs(hg, 0)
    assert d.tolist() == [0, 1, 1, 2, -1]
    P, Q = oracle.PUSH, oracle.PULL
    assert oracle.schedule_edges(hg, d, alpha=0.66, beta=0.01) == [P, Q, Q]   # 2 > 1.98
    assert oracle.schedule_edges(hg, d, alpha=0.67, beta=0.01) == [P, P, P]   # 2 > 2.01 fails; 0 > 0 fails


# ------------------------------------------------------------------- TEPS
def test_teps_convention_matches_printed_figures():
    """The paper's MTEPS equal nnz(A) of the symmetrized graph divided by the runtime."""
    with open(os.path.join(GOLDEN, "fig7_this_work.json")) as f:
        rows = json.load(f)["rows"]
    for name, edges, ms, mteps in rows:
        assert abs(edges / (ms * 1e-3) / 1e6 - mteps) / mteps < 0.05, name


def test_table2_speedups_are_incremental():
    with open(os.path.join(GOLDEN, "table2_ablation.json")) as f:
        rows = json.load(f)["rows"]
    for (_, prev, _), (name, gteps, printed) in zip(rows, rows[1:]):
        assert abs(gteps / prev - printed) < 0.011, name


def test_teps_edges():
    g = _path(10)
    d, _ = oracle.bfs(g, 3)
    assert oracle.teps_edges(g, d) == {"graph500": 9, "paper": 18}
    g2 = gen.from_edges(6, [0, 1, 3], [1, 2, 4])
    d2, _ = oracle.bfs(g2, 0)
    assert oracle.teps_edges(g2, d2) == {"graph500": 2, "paper": 6}


# ------------------------------------------- first-hit parents: hand-worked pins
def _fig3_columns(fx, cols):
    """The Figure 3 graph with its CSC columns stored as `cols` lists them (CSR sorted)."""
    names = list(fx["vertices"])
    ids = {v: i for i, v in enumerate(names)}
    base = gen.from_edges(len(ids), *np.array([[ids[a], ids[b]] for a, b in fx["undirected_edges"]]).T)
    colptr = np.zeros(len(names) + 1, dtype=np.int32)
    rowind = []
    for i, v in enumerate(names):
        col = [ids[u] for u in cols[v]]
        # the hand-written columns hold exactly the graph's in-neighbours
        assert sorted(col) == base.csc_rowind[base.csc_colptr[i]:base.csc_colptr[i + 1]].tolist(), v
        rowind += col
        colptr[i + 1] = len(rowind)
    g = gen.HostGraph("fig3_cols", len(names), base.rowptr, base.colind, colptr,
                      np.asarray(rowind, dtype=np.int32), True, {})
    return g, ids, names


@pytest.mark.parametrize("order", ["sorted_columns", "reordered_columns"])
def test_first_parent_fig3_hand_worked(order):
    """Section 4.2 / Algorithm 2: a pull stops at the first in-neighbour, in the order the
    column is stored, that is one level up. On the Figure 3 graph from A, vertex E has two
    such in-neighbours (C and D): sorted it reports C (the last hit would be D); with the
    column stored as G, D, C it reports D, which is neither the smallest id nor the last hit."""
    with open(os.path.join(GOLDEN, "fig3_toy.json")) as f:
        fx = json.load(f)
    with open(os.path.join(GOLDEN, "fig3_first_parent.json")) as f:
        pin = json.load(f)
    g, ids, names = _fig3_columns(fx, pin[order]["columns"])
    s = ids[pin["source"]]
    d, _ = oracle.bfs(g, s)
    assert {v: int(d[ids[v]]) for v in names} == pin["depth"]
    fp = oracle.first_parent(g, d, s)
    assert {v: names[fp[ids[v]]] for v in names} == pin[order]["first_parent"]
    assert oracle.validate(g, s, d, fp)[0] == 0
    # the pull of level 1 (visited = {A, B, C, D}) checks this many in-neighbours
    assert oracle.pull_checks(g, d, 1) == pin[order]["pull_checks_level1"]
    if order == "sorted_columns":
        last = pin[order]["last_parent"]
        assert all(names[fp[ids[v]]] != p for v, p in last.items())


def _pull_traversal_parents(V, colptr, rowind, s):
    """Algorithm 1 run with the pull of Algorithm 2 at every level, written level by level:
    x = the visited set at the start of the level (operand reuse), every unvisited row scans
    its column in stored order and stops at the first entry with x set; that entry is the
    row's parent. A different route to first_parent's values: frontier membership level by
    level instead of the final depths."""
    visited = np.zeros(V, dtype=bool)
    visited[s] = True
    parent = np.full(V, -1, dtype=np.int64)
    parent[s] = s
    while True:
        found = {}
        for i in range(V):
            if visited[i]:
                continue
            for q in range(colptr[i], colptr[i + 1]):
                if visited[rowind[q]]:
                    found[i] = rowind[q]
                    break
        if not found:
            return parent
        for i, j in found.items():
            visited[i] = True
            parent[i] = j


@pytest.mark.parametrize("reverse", [False, True])
def test_first_parent_matches_level_by_level_pull(reverse):
    """All undirected graphs on 5 vertices, every source, columns stored sorted and reversed."""
    n = 5
    pairs = list(itertools.combinations(range(n), 2))
    for bits in range(0, 1 << len(pairs), 3):
        A = np.zeros((n, n), dtype=bool)
        for k, (i, j) in enumerate(pairs):
            if bits >> k & 1:
                A[i, j] = A[j, i] = True
        g = _graph_from_dense(A)
        if reverse:
            ri = np.concatenate([g.csc_rowind[g.csc_colptr[v]:g.csc_colptr[v + 1]][::-1] for v in range(n)])
            g = gen.HostGraph("rev", n, g.rowptr, g.colind, g.csc_colptr, ri.astype(np.int32), True, {})
        for s in range(n):
            d, _ = oracle.bfs(g, s)
            want = _pull_traversal_parents(n, g.csc_colptr, g.csc_rowind, s)
            assert np.array_equal(oracle.first_parent(g, d, s), want), (A, s, reverse)
