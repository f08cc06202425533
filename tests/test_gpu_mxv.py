"""GPU parity of the standalone dobfs_mxv against the oracle's Boolean masked matvec
(Equations 2-5, Section 3.2): the four variants of Section 6.3 / Table 1, with and without
early exit, structural complement and OR-accumulate, dense or sparse input."""
import itertools
import json
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1804_03327_amd import dobfs  # noqa: E402
from paper_1804_03327_amd.helpers import pack_bits, unpack_bits, upload  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _edge_set(hg):
    rows = np.repeat(np.arange(hg.V, dtype=np.int64), np.diff(hg.rowptr.astype(np.int64)))
    return np.unique(rows * hg.V + hg.colind.astype(np.int64))


def _run(g, hg, x, mask, complement, direction, flags, y_old, sparse_x):
    V = hg.V
    yb = _dev(pack_bits(y_old))
    y_idx = torch.full((V,), -7, dtype=torch.int32, device="cuda")
    wit = torch.full((V,), -7, dtype=torch.int32, device="cuda")
    kw = dict(mask_bits=_dev(pack_bits(mask)) if mask is not None else None, complement=complement,
              direction=direction, flags=flags, y_idx=y_idx, y_witness=wit)
    if sparse_x:
        idx = np.nonzero(x)[0].astype(np.int32)
        nnz = dobfs.mxv(g, yb, x_idx=_dev(idx) if idx.size else None, x_nnz=idx.size, **kw)
    else:
        nnz = dobfs.mxv(g, yb, x_bits=_dev(pack_bits(x)), **kw)
    y = unpack_bits(yb.cpu().numpy(), V)
    return y, nnz, y_idx.cpu().numpy(), wit.cpu().numpy()


@pytest.fixture(scope="module")
def cases():
    rng = np.random.default_rng(21)
    V = 70_001
    src = rng.integers(0, V, 6 * V)
    dst = (src * 7 + rng.zipf(1.5, src.size)) % V
    directed = gen.from_edges(V, src, dst, directed=True, name="directed70001")
    out = []
    for hg in (gen.rmat(13, 16, seed=4), directed):
        out.append((hg, upload(hg, validate=True), _edge_set(hg)))
    return out


def test_mxv_variants_match_oracle(cases):
    rng = np.random.default_rng(22)
    for hg, g, edges in cases:
        V = hg.V
        for dens in (0.0, 0.0005, 0.05, 0.6):
            x = rng.random(V) < dens
            m = rng.random(V) < 0.5
            y_old = rng.random(V) < 0.3
            for mask, comp, direction, ee, acc, sparse in itertools.product(
                    (None, m), (False, True), (dobfs.DIR_PUSH, dobfs.DIR_PULL), (False, True),
                    (False, True), (False, True)):
                if mask is None and comp:
                    continue
                flags = (dobfs.MXV_EARLY_EXIT if ee else 0) | (dobfs.MXV_ACCUM_OR if acc else 0)
                tag = "%s dens=%g mask=%s comp=%s dir=%d ee=%s acc=%s sparse=%s" % (
                    hg.name, dens, mask is not None, comp, direction, ee, acc, sparse)
                y, nnz, y_idx, wit = _run(g, hg, x, mask, comp, direction, flags, y_old, sparse)
                want = oracle.mxv(hg, x, mask, comp, acc, y_old).astype(bool)
                assert np.array_equal(y, want), tag
                assert nnz == int(want.sum()), tag
                assert np.array_equal(y_idx[:nnz], np.nonzero(want)[0]), tag
                # witnesses: exactly the result entries (not the accumulated ones) get one
                res = oracle.mxv(hg, x, mask, comp).astype(bool)
                assert np.all(wit[~res] == -7), tag
                r = np.nonzero(res)[0]
                w = wit[r].astype(np.int64)
                assert np.all((w >= 0) & (w < V)), tag
                assert np.all(x[w]), tag
                assert np.all(np.isin(w * V + r, edges)), tag
                if direction == dobfs.DIR_PULL and r.size:
                    # pull reports the first in-neighbour in CSC order with x set
                    for i in r[:: max(1, r.size // 300)]:
                        col = hg.csc_rowind[hg.csc_colptr[i]:hg.csc_colptr[i + 1]]
                        assert wit[i] == col[np.nonzero(x[col])[0][0]], tag


def test_mxv_fig3_toy():
    with open(os.path.join(GOLDEN, "fig3_toy.json")) as f:
        fx = json.load(f)
    ids = {v: i for i, v in enumerate(fx["vertices"])}
    e = np.array([[ids[a], ids[b]] for a, b in fx["undirected_edges"]])
    hg = gen.from_edges(len(ids), e[:, 0], e[:, 1])
    g = upload(hg)

    def vec(names):
        v = np.zeros(len(ids), dtype=bool)
        v[[ids[n] for n in names]] = True
        return v

    f, v = vec(fx["frontier"]), vec(fx["visited"])
    for direction in (dobfs.DIR_PUSH, dobfs.DIR_PULL):
        y, nnz, _, _ = _run(g, hg, f, None, False, direction, 0, np.zeros(8, bool), False)
        assert np.array_equal(y, vec(fx["push_children_before_filter"]))
        for x in (f, v):  # frontier, or the visited set (operand reuse)
            y, nnz, idx, _ = _run(g, hg, x, v, True, direction, dobfs.MXV_EARLY_EXIT,
                                  np.zeros(8, bool), False)
            assert np.array_equal(y, vec(fx["next_after_filter"]))
            assert sorted(idx[:nnz].tolist()) == sorted(ids[n] for n in fx["next_after_filter"])


def test_mxv_rejects_bad_args(cases):
    hg, g, _ = cases[0]
    yb = torch.zeros(g.nwords, dtype=torch.int32, device="cuda")
    with pytest.raises(dobfs.DobfsError):
        dobfs.mxv(g, yb, x_bits=yb, direction=5)
    with pytest.raises(dobfs.DobfsError):
        dobfs.mxv(g, yb, x_bits=yb, flags=8)
    with pytest.raises(dobfs.DobfsError):
        dobfs.mxv(g, yb, x_idx=None, x_nnz=3)


def test_mxv_in_place_operand_reuse(cases):
    """x = mask = y in one buffer: the in-place BFS form v = v OR A^T v .* not(v) (Section 5.4,
    complement and ACCUM_OR). The result must be the oracle's one-hop step from the vector
    as it was before the call, in both directions and with or without early exit, repeated
    from a few random starting sets (two hops never appear in one call)."""
    rng = np.random.default_rng(23)
    for hg, g, _ in cases:
        V = hg.V
        for dens in (0.0005, 0.02, 0.3):
            v0 = rng.random(V) < dens
            for direction, ee in itertools.product((dobfs.DIR_PUSH, dobfs.DIR_PULL), (False, True)):
                buf = _dev(pack_bits(v0))
                flags = dobfs.MXV_ACCUM_OR | (dobfs.MXV_EARLY_EXIT if ee else 0)
                nnz = dobfs.mxv(g, buf, x_bits=buf, mask_bits=buf, complement=True,
                                direction=direction, flags=flags)
                got = unpack_bits(buf.cpu().numpy(), V)
                want = oracle.mxv(hg, v0, v0, True, True, v0).astype(bool)
                tag = "%s dens=%g dir=%d ee=%s" % (hg.name, dens, direction, ee)
                assert np.array_equal(got, want), tag
                assert nnz == int(want.sum()), tag
