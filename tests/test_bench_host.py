"""CPU checks of the benchmark's host-side bookkeeping: the pull candidate table against a
brute-force count, and the rule that a committed PMC traffic record is used only while the
kernel sources hash as when it was counted (and, for the multi-source record, while the
benchmarked launch runs the same level directions)."""
import json
import os
import shutil

import numpy as np

import bench


def test_candidates_per_level_brute_force():
    rng = np.random.default_rng(3)
    depth = rng.integers(-1, 6, 500)
    indeg_nz = rng.random(500) < 0.8
    got = bench.candidates_per_level(depth, indeg_nz)
    for L in range(int(depth.max()) + 1):
        # rows a level-L pull lists: in-degree > 0 and not yet visited when level L starts
        want = sum(1 for v in range(500) if indeg_nz[v] and (depth[v] < 0 or depth[v] > L))
        assert got[L] == want, L


def _fake_tree(tmp_path):
    """A copy of the kernel sources and an empty profiles folder, with bench pointed at them."""
    root = tmp_path / "repo"
    csrc = root / "paper_1804_03327_amd" / "csrc"
    inc = root / "include"
    csrc.mkdir(parents=True)
    inc.mkdir()
    (root / "profiles").mkdir()
    for name in ("kernels.hip", "batch.hip", "device_common.h", "dobfs_internal.h"):
        shutil.copy(os.path.join(bench.KERNEL_DIR, name), csrc / name)
    shutil.copy(os.path.join(bench.ROOT, "include", "dobfs.h"), inc / "dobfs.h")
    return root, csrc


def test_traffic_records_follow_the_sources(tmp_path, monkeypatch):
    root, csrc = _fake_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "KERNEL_DIR", str(csrc))
    levels = ["push", "push", "pull", "push"]
    h1 = bench.kernel_source_hash()
    h2 = bench.kernel_source_hash(bench.MULTI_SOURCE_KERNEL_FILES)
    assert h1 != h2
    with open(root / "profiles" / "traffic_step_rmat22.json", "w") as f:
        json.dump({"kernel_source_sha256_16": h1, "bytes_per_launch": 1234}, f)
    with open(root / "profiles" / "traffic_mb_step_rmat20.json", "w") as f:
        json.dump({"kernel_source_sha256_16": h2, "levels": levels, "bytes_per_push_or_pull_step": 99}, f)
    assert bench.load_traffic("step") == 1234
    assert bench.load_mb_traffic(levels) == 99
    assert bench.load_mb_traffic(levels[:-1]) is None  # another level sequence
    assert bench.load_traffic("init") is None  # no record
    # a change to the multi-source kernels voids only their record
    with open(csrc / "batch.hip", "a") as f:
        f.write("\n// edited\n")
    assert bench.load_mb_traffic(levels) is None
    assert bench.load_traffic("step") == 1234
    # a change to a shared header voids both
    with open(csrc / "device_common.h", "a") as f:
        f.write("\n// edited\n")
    assert bench.load_traffic("step") is None


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
