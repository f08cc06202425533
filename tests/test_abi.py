"""CPU checks of the C ABI: the library loads, exports every function include/dobfs.h
declares, and its host logic (direction rule, argument checks) behaves as specified. No
compute call is made here."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1804_03327_amd import dobfs
from paper_1804_03327_amd.helpers import pack_bits, unpack_bits


def test_library_exports_every_header_function():
    lib = dobfs.load()
    names = dobfs.header_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings_and_version():
    assert dobfs.status_string(0) == "DOBFS_OK"
    assert dobfs.status_string(4) == "DOBFS_ERR_WORKSPACE_TOO_SMALL"
    assert dobfs.version() >= 100


def test_default_options():
    o = dobfs.options_default()
    assert o.mode == dobfs.MODE_FULL and o.heuristic == dobfs.HEUR_RATIO
    assert o.alpha == pytest.approx(0.01) and o.beta == pytest.approx(0.01)
    assert o.n_forced == 0 and o.flags == 0


def _library_schedule(sizes, V, opt):
    """Replay the library's direction rule over a sequence of level sizes."""
    d, dirs = dobfs.DIR_PUSH, []
    for L in range(len(sizes)):
        dirs.append(d)
        nn = sizes[L + 1] if L + 1 < len(sizes) else 0
        d = dobfs.next_direction(opt, d, V, sizes[L], nn)
    return dirs


def test_direction_rule_matches_oracle_schedule():
    rng = np.random.default_rng(0)
    opt = dobfs.options_default()
    for _ in range(300):
        V = int(rng.integers(1, 1 << 23))
        n = int(rng.integers(1, 12))
        sizes = [1] + [int(x) for x in rng.integers(0, max(2, V // 10), n)]
        for alpha, beta in ((0.01, 0.01), (0.05, 0.002)):
            opt.alpha, opt.beta = alpha, beta
            assert _library_schedule(sizes, V, opt) == oracle.schedule(sizes, V, alpha, beta)


def test_direction_rule_boundaries():
    opt = dobfs.options_default()
    V = 4194304  # alpha * V = 41943.04
    P, Q = dobfs.DIR_PUSH, dobfs.DIR_PULL
    assert dobfs.next_direction(opt, P, V, 10, 41943) == P
    assert dobfs.next_direction(opt, P, V, 10, 41944) == Q
    assert dobfs.next_direction(opt, P, V, 50000, 45000) == P  # shrinking: stays push
    assert dobfs.next_direction(opt, Q, V, 50000, 41944) == Q  # shrinking but above beta
    assert dobfs.next_direction(opt, Q, V, 50000, 41943) == P
    assert dobfs.next_direction(opt, Q, V, 100, 200) == Q  # growing: stays pull
    e = dobfs.make_options(heuristic=dobfs.HEUR_EDGES, alpha=1 / 14, beta=1 / 24)
    assert dobfs.next_direction(e, P, V, 1, 5, m_f=1000, m_u=14001) == P
    assert dobfs.next_direction(e, P, V, 1, 5, m_f=1001, m_u=14001) == Q
    assert dobfs.next_direction(e, Q, V, 10, V // 24 - 1) == P
    assert dobfs.next_direction(e, Q, V, 10, V // 24 + 1) == Q


def test_host_side_argument_checks():
    lib = dobfs.load()
    h = ctypes.c_void_p()
    rp = np.array([0, 1, 2, 2], dtype=np.int32)
    ci = np.array([1, 2], dtype=np.int32)
    P = rp.ctypes.data, ci.ctypes.data
    assert lib.dobfs_graph_upload(0, 0, *P, *P, 0, 0, ctypes.byref(h)) == dobfs.ERR_INVALID_ARG
    assert lib.dobfs_graph_upload(3, 2, *P, *P, 0, 0, None) == dobfs.ERR_INVALID_ARG
    assert lib.dobfs_graph_upload(3, -1, *P, *P, 0, 0, ctypes.byref(h)) == dobfs.ERR_INVALID_ARG
    assert lib.dobfs_graph_upload(3, 3, *P, *P, 0, 0, ctypes.byref(h)) == dobfs.ERR_INVALID_ARG
    assert "expected nnz" in dobfs.last_error()
    bad = np.array([0, 2, 1, 2], dtype=np.int32)
    assert lib.dobfs_graph_upload(3, 2, bad.ctypes.data, ci.ctypes.data, *P, 0, 0,
                                  ctypes.byref(h)) == dobfs.ERR_INVALID_ARG
    assert "decreases" in dobfs.last_error()
    oob = np.array([1, 3], dtype=np.int32)
    assert lib.dobfs_graph_upload(3, 2, rp.ctypes.data, oob.ctypes.data, *P, 0, dobfs.UPLOAD_VALIDATE,
                                  ctypes.byref(h)) == dobfs.ERR_INVALID_ARG
    assert lib.dobfs_graph_upload(3, 2, *P, *P, 0, 0x80, ctypes.byref(h)) == dobfs.ERR_INVALID_ARG
    assert lib.dobfs_bfs(None, 0, None, None, None, None, 0, None, None) == dobfs.ERR_INVALID_ARG
    assert lib.dobfs_mxv(None, None, None, 0, None, 0, 0, 0, None, None, None, None, None, 0,
                         None) == dobfs.ERR_INVALID_ARG
    assert lib.dobfs_graph_destroy(None) == dobfs.OK


def test_bit_packing_layout():
    rng = np.random.default_rng(1)
    for V in (1, 31, 32, 33, 1000, 4097):
        m = rng.random(V) < 0.4
        w = pack_bits(m).view(np.uint32)
        assert w.size == (V + 31) // 32
        i = np.arange(V)
        assert np.array_equal(((w[i >> 5] >> (i & 31)) & 1).astype(bool), m)
        assert np.array_equal(unpack_bits(w, V), m)


def test_autotune_candidates_cover_both_rules():
    from paper_1804_03327_amd import autotune, dobfs
    c = autotune.candidates()
    assert len(c) == len(set(c))
    assert {h for h, _, _ in c} == {dobfs.HEUR_RATIO, dobfs.HEUR_EDGES}
    assert (dobfs.HEUR_RATIO, 0.01, 0.01) in c  # the paper's constants
    assert any(h == dobfs.HEUR_EDGES and abs(a - 1 / 14) < 1e-12 and abs(b - 1 / 24) < 1e-12 for h, a, b in c)
    assert autotune.describe(dict(heuristic=dobfs.HEUR_RATIO, alpha=0.01, beta=0.01)) == "ratio alpha=0.01 beta=0.01"
