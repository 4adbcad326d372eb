"""Host-side logic of bench.py (no GPU): the byte accounting behind the
roofline fields, the digest that ties counter summaries to the kernels, and
the one-GPU guard."""
import json
import math
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_kernel_bytes_small_batch_by_hand():
    # frame 0: 100 points, 80 valid, 2 passes, 10 cells, keys stored (narrow)
    # frame 1: 50 points, none valid (no radix pass, no cells)
    # frame 2: 40 points, 40 valid, 3 passes, 5 cells, wide keys (recomputed in pass 0)
    kb = bench.kernel_bytes([100, 50, 40], [80, 0, 40], [2, 0, 3], [10, 0, 5],
                            [True, True, False])
    assert kb["bbox"] == 12 * 190
    assert kb["hist"] == 12 * 190 + 4 * 100          # stored keys of live narrow frames only
    assert kb["sort"] == (4 * 100 + 12 * 50 + 12 * 40) + 8 * (80 + 40) + 16 * (80 * 1 + 40 * 2)
    assert kb["reduce"] == 23 * (80 + 40) + 27 * (10 + 5)
    assert kb["fixup"] == 0 and kb["init"] == 0
    assert kb["pipeline"] == sum(v for k, v in kb.items() if k != "pipeline")
    # the point rows add 4 B per valid point to the reduce
    kb2 = bench.kernel_bytes([100], [80], [2], [10], [True], point_cell=True)
    assert kb2["reduce"] == 27 * 80 + 27 * 10


def test_frame_passes_matches_key_width():
    rng = np.random.default_rng(3)
    x, y, z = (rng.uniform(0.0, 1.0, 1000).astype(np.float32) for _ in range(3))
    x[5] = np.nan  # ignored
    p, bits = bench.frame_passes(x, y, z, 0.05, 8, with_bits=True)
    inv = np.float32(1.0) / np.float32(0.05)
    dims = []
    for a in (x, y, z):
        v = a[np.isfinite(x) & np.isfinite(y) & np.isfinite(z)]
        dims.append(int(np.floor((v.max() - v.min()) * inv)) + 1)
    top = dims[0] * dims[1] * dims[2] - 1
    assert bits == top.bit_length()
    assert p == max(1, math.ceil(bits / 8))
    nan = np.full(4, np.nan, np.float32)
    assert bench.frame_passes(nan, nan, nan, 0.05, 8, with_bits=True) == (0, 0)


def _copy_tree(dst):
    for rel in ("include", os.path.join("paper_2102_11084_amd", "csrc")):
        shutil.copytree(os.path.join(ROOT, rel), os.path.join(dst, rel))
    shutil.copy(os.path.join(ROOT, "paper_2102_11084_amd", "tuning_gfx950.json"),
                os.path.join(dst, "paper_2102_11084_amd", "tuning_gfx950.json"))


def test_source_digest_follows_tuning_choice_not_timings(tmp_path, monkeypatch):
    _copy_tree(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.source_digest()
    assert d0 == bench.source_digest()
    tpath = tmp_path / "paper_2102_11084_amd" / "tuning_gfx950.json"
    doc = json.loads(tpath.read_text())
    doc["median_ms"] = 123.0           # a new autotuner timing: same kernels
    tpath.write_text(json.dumps(doc))
    assert bench.source_digest() == d0
    doc["tuning"]["reduce_items"] = 4  # another tuning: other kernels
    tpath.write_text(json.dumps(doc))
    assert bench.source_digest() != d0
    doc["tuning"]["reduce_items"] = 8
    tpath.write_text(json.dumps(doc))
    src = tmp_path / "paper_2102_11084_amd" / "csrc" / "vg_pipeline.hpp"
    src.write_text(src.read_text() + "\n// edited\n")  # device code changed
    assert bench.source_digest() != d0


def test_read_traffic_rejects_other_kernels(tmp_path, monkeypatch):
    _copy_tree(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "hbm_traffic_x.txt").write_text(
        f"# header\nsource_digest: {bench.source_digest()}\nsort_bytes_per_launch: 1234\n")
    assert bench.read_traffic("sort", "x")[0] == 1234
    assert bench.read_traffic("reduce", "x")[0] is None
    (prof / "hbm_traffic_x.txt").write_text("source_digest: 0000\nsort_bytes_per_launch: 1234\n")
    v, why = bench.read_traffic("sort", "x")
    assert v is None and "other kernels" in why
    assert bench.read_traffic("sort", "missing")[0] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr


def test_step_bytes_by_kernel_by_hand():
    # the method's per-step bytes: 12 n (box) + 12 n + 4 n_v (keys, histograms)
    # + 16 P n_v (radix passes) + 23 n_v + 27 m (reduce), + 8 n_v pair write
    kb = bench.step_bytes_by_kernel([100, 50, 40], [80, 0, 40], [2, 0, 3], [10, 0, 5])
    assert kb["bbox"] == 12 * 190
    assert kb["hist"] == 12 * 190 + 4 * 120
    assert kb["sort"] == 16 * (2 * 80 + 3 * 40)
    assert kb["reduce"] == 23 * 120 + 27 * 15
    total = sum(bench.algorithmic_bytes(n, nv, p, m) for n, nv, p, m in
                [(100, 80, 2, 10), (50, 0, 0, 0), (40, 40, 3, 5)])
    assert kb["pipeline"] == total


def test_nbd_candidate_checks_by_brute_force():
    rng = np.random.default_rng(5)
    p = rng.uniform(0, 0.3, size=(300, 3)).astype(np.float32)
    p[7, 1] = np.nan
    x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
    v = np.isfinite(p).all(1)
    inv = np.float32(1.0) / np.float32(0.05)
    k = np.floor((p[v] - p[v].min(0)) * inv).astype(np.int64)
    exp = int((np.abs(k[:, None, :] - k[None, :, :]) <= 1).all(-1).sum())
    assert bench.nbd_candidate_checks(x, y, z, 0.05) == exp
