"""Generator checks: determinism, graph hygiene (Section 7.1: undirected, no self-loops, no
duplicate edges), exact sizes of the mesh-like graphs, and the R-MAT quadrant law."""
import numpy as np
import pytest

import gen


def _hygiene(g):
    V = g.V
    rp, ci = g.rowptr.astype(np.int64), g.colind.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == ci.size
    assert np.all(np.diff(rp) >= 0)
    assert ci.size == 0 or (ci.min() >= 0 and ci.max() < V)
    rows = np.repeat(np.arange(V), np.diff(rp))
    assert not np.any(rows == ci), "self-loop"
    key = rows * V + ci
    assert np.all(np.diff(key) > 0), "rows must be sorted and duplicate-free"
    # symmetric: the reversed edge set equals the edge set
    rkey = np.sort(ci * V + rows)
    assert np.array_equal(rkey, key)


@pytest.mark.parametrize("scale", [6, 10, 13])
def test_rmat_hygiene_and_determinism(scale):
    g1 = gen.rmat(scale, 16, seed=7)
    g2 = gen.rmat(scale, 16, seed=7)
    g3 = gen.rmat(scale, 16, seed=8)
    _hygiene(g1)
    assert g1.V == 1 << scale
    assert np.array_equal(g1.rowptr, g2.rowptr) and np.array_equal(g1.colind, g2.colind)
    assert not np.array_equal(g1.colind, g3.colind)
    # at most 2 * edgefactor * V directed entries; duplicates make it fewer
    assert g1.nnz <= 2 * 16 * g1.V


def test_rmat_quadrant_law():
    """P(source bit set) = c + d and P(destination bit set) = b + d at every level."""
    scale, n = 12, 400_000
    src, dst = gen.rmat_raw_edges(scale, n, seed=11)
    a, b, c = gen.RMAT_A, gen.RMAT_B, gen.RMAT_C
    d = 1 - a - b - c
    sd = 4 * np.sqrt(0.24 * 0.76 / n)
    for bit in range(scale):
        ps = ((src >> bit) & 1).mean()
        pd = ((dst >> bit) & 1).mean()
        assert abs(ps - (c + d)) < sd, (bit, ps)
        assert abs(pd - (b + d)) < sd, (bit, pd)
    # joint: both bits set with probability d
    both = (((src >> 3) & 1) & ((dst >> 3) & 1)).mean()
    assert abs(both - d) < 4 * np.sqrt(d * (1 - d) / n)


def test_rmat_raw_edges_are_counter_based():
    s1, d1 = gen.rmat_raw_edges(10, 1000, seed=3)
    s2, d2 = gen.rmat_raw_edges(10, 500, seed=3, start=500)
    assert np.array_equal(s1[500:], s2) and np.array_equal(d1[500:], d2)


def test_rmat_scale_free_shape():
    g = gen.rmat(16, 16, seed=1)
    deg = g.out_degree()
    # heavy tail: the largest degree is far above the mean
    assert deg.max() > 50 * deg[deg > 0].mean()
    # a sizeable fraction of R-MAT vertices is isolated
    assert 0.05 < (deg == 0).mean() < 0.6


@pytest.mark.parametrize("n", [1, 2, 5, 17])
def test_lattice_exact_counts(n):
    g = gen.lattice3d(n, 0.0, seed=1)
    _hygiene(g)
    assert g.V == n ** 3
    assert g.nnz == 2 * 3 * n * n * (n - 1)
    # every edge joins vertices at L1 distance 1
    rows = np.repeat(np.arange(g.V), np.diff(g.rowptr.astype(np.int64)))
    cols = g.colind.astype(np.int64)

    def xyz(i):
        return np.stack([i % n, (i // n) % n, i // (n * n)])

    assert np.all(np.abs(xyz(rows) - xyz(cols)).sum(axis=0) == 1)


def test_lattice_deletions_exact_and_seeded():
    n = 12
    M = 3 * n * n * (n - 1)
    g = gen.lattice3d(n, 0.05, seed=3)
    _hygiene(g)
    assert g.nnz == 2 * (M - int(0.05 * M))
    h = gen.lattice3d(n, 0.05, seed=4)
    assert h.nnz == g.nnz and not np.array_equal(h.colind, g.colind)


def test_lattice256_size():
    """The 256^3 lattice with 5% deletions: 47,628,288 undirected = 95,256,576 directed edges."""
    M = 3 * 256 * 256 * 255
    assert M - int(0.05 * M) == 47_628_288


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 7), (5, 4), (33, 29)])
def test_grid_exact_counts(nx, ny):
    g = gen.grid2d(nx, ny)
    _hygiene(g)
    assert g.nnz == 2 * ((nx - 1) * ny + nx * (ny - 1))


def test_from_edges_directed_csc_is_transpose():
    g = gen.from_edges(4, [0, 0, 1, 3, 3], [1, 2, 2, 0, 0], directed=True)
    assert g.rowptr.tolist() == [0, 2, 3, 3, 4]
    assert g.colind.tolist() == [1, 2, 2, 0]
    assert g.csc_colptr.tolist() == [0, 1, 2, 4, 4]
    assert g.csc_rowind.tolist() == [3, 0, 0, 1]


def test_transpose_matches_dense():
    rng = np.random.default_rng(0)
    A = rng.random((37, 37)) < 0.1
    src, dst = np.nonzero(A)
    g = gen.from_edges(37, src, dst, directed=True, keep_self_loops=True)
    D = np.zeros((37, 37), dtype=bool)
    for v in range(37):
        D[g.csc_rowind[g.csc_colptr[v]:g.csc_colptr[v + 1]], v] = True
    assert np.array_equal(D, A)


def test_sample_sources():
    g = gen.rmat(12, 16, seed=1)
    s = gen.sample_sources(g, 64, seed=2)
    assert s.size == 64 and np.unique(s).size == 64
    assert np.all(g.out_degree()[s] > 0)
    assert np.array_equal(s, gen.sample_sources(g, 64, seed=2))
    assert not np.array_equal(s, gen.sample_sources(g, 64, seed=5))


def test_max_degree_vertex_ties_smallest():
    g = gen.from_edges(5, [0, 1, 3, 3], [4, 4, 1, 2])
    # degrees: 0:1, 1:2, 2:1, 3:2, 4:2 -> smallest id among the maxima is 1
    assert gen.max_degree_vertex(g) == 1
