"""Seeded random cases against the oracle: batches of random composition
(empty and tiny frames, RGB-D frames of random size, large uniform clouds,
random leaves) under random built tunings, launch forms and key modes; the
decimation under random radius, umbral and round size; voxel-map sequences of
random marks, frustum clears and expiries with every operation's count."""
import numpy as np
import pytest
import torch

import oracle
import test_gpu_batched as tb
from gpu_util import to_dev
from paper_2102_11084_amd import datagen as dg
from paper_2102_11084_amd import vg

pytestmark = pytest.mark.gpu

SHAPES = [(512, 8, 8, 8), (512, 8, 8, 4), (256, 16, 8, 8), (256, 8, 8, 4), (256, 16, 6, 8)]


def built_tunings():
    out = []
    for blk, si, rb, ri in SHAPES:
        for mode in (vg.EXEC_PERSISTENT, vg.EXEC_PHASED):
            t = vg.default_tuning(sort_block=blk, sort_items=si, radix_bits=rb, reduce_block=blk,
                                  reduce_items=ri, exec_mode=mode, blocks_per_cu=0)
            if vg.tuning_supported(t):
                out.append(t)
    return out


@pytest.mark.parametrize("case", range(8))
def test_random_batches(case):
    rng = np.random.default_rng(7100 + case)
    B = int(rng.integers(1, 40))
    parts, leaves = [], []
    for _ in range(B):
        r = rng.random()
        if r < 0.1:
            n = int(rng.integers(0, 3))
            p = (rng.random((n, 3)) * 2).astype(np.float32)
            parts.append((p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(),
                          rng.integers(0, 256, (n, 3), dtype=np.uint8)))
        elif r < 0.2:
            parts.append(dg.uniform_cloud(int(rng.integers(100_000, 2_000_000)),
                                          seed=int(rng.integers(1 << 30)),
                                          side=float(rng.uniform(0.5, 5.0))))
        else:
            parts.append(dg.rgbd_frame(int(rng.integers(16, 400)), int(rng.integers(16, 300)),
                                       seed=int(rng.integers(1 << 30))))
        leaves.append(float(rng.choice([0.01, 0.02, 0.05, 0.1, 0.3])))
    offs = np.zeros(B + 1, np.int64)
    offs[1:] = np.cumsum([p[0].size for p in parts])
    x, y, z, rgb = (np.concatenate([p[a] for p in parts]) for a in range(4))
    lv = np.array(leaves, np.float32)
    tunings = built_tunings()
    t = tunings[int(rng.integers(len(tunings)))]
    km = vg.KEY_MORTON if rng.random() < 0.3 else vg.KEY_LINEAR
    print(f"case random batch {case}: B {B}, n {x.size}, tuning {t.as_dict()}, key mode {km}",
          flush=True)
    g = tb.run_batched(x, y, z, rgb, offs, lv, key_mode=km, tuning=t)
    tb.check_against_oracle(g, x, y, z, rgb, offs, lv, key_mode=km)


@pytest.mark.parametrize("case", range(12))
def test_random_decimation(case):
    rng = np.random.default_rng(7200 + case)
    W, H = int(rng.integers(20, 200)), int(rng.integers(20, 160))
    x, y, z, rgb = dg.rgbd_frame(W, H, seed=int(rng.integers(1 << 30)))
    leaf = float(rng.choice([0.02, 0.05, 0.1]))
    radius = leaf * float(rng.uniform(0.3, 1.0))
    umbral = int(rng.integers(0, 30))
    rs = int(rng.choice([1, 7, 50, 300, 1000]))
    seed = int(rng.integers(1 << 40))
    print(f"case random decimation {case}: {W}x{H} leaf {leaf} radius {radius:.4f} umbral {umbral} "
          f"round {rs}", flush=True)
    g = vg.nbd_decimate(*to_dev(x, y, z, rgb.reshape(-1)), leaf=leaf, radius=radius,
                        umbral=umbral, seed=seed, round_size=rs, with_count0=True)
    torch.cuda.synchronize()
    o = oracle.nbd_decimate(x, y, z, leaf, radius, umbral, seed, rs)
    assert g["rounds"] == o["rounds"]
    assert np.array_equal(g["marked"], o["marked"])
    assert np.array_equal(g["count0"].cpu().numpy().view(np.uint32), o["count0"])
    ki = g["keep_index"].cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(ki, np.flatnonzero(o["keep"]))


@pytest.mark.parametrize("case", range(4))
def test_random_map_sequences(case):
    rng = np.random.default_rng(7300 + case)
    res = float(rng.choice([0.05, 0.1, 0.2]))
    print(f"case random map sequence {case}: res {res}", flush=True)
    g, o = vg.VoxelMap(1 << 20, res), oracle.VoxelMap(res)
    for step in range(10):
        op = int(rng.integers(0, 3))
        if op == 0:
            n = int(rng.integers(0, 100_000))
            p = rng.uniform(-5, 5, (n, 3)).astype(np.float32)
            xx, yy, zz = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
            g.mark(*to_dev(xx, yy, zz), step + 1)
            kind, want = "skipped", o.mark(xx, yy, zz, step + 1)
        elif op == 1:
            R, t = dg.camera_pose(int(rng.integers(1 << 30)))
            args = (R, t, 525.0, 525.0, 319.5, 239.5, 640, 480, 0.3, 4.0)
            g.clear(vg.make_frustum(*args))
            kind, want = "cleared", o.clear(*args)
        else:
            g.expire(step)
            kind, want = "expired", o.expire(step)
        torch.cuda.synchronize()
        gk, gs = g.export()
        ok, os_ = o.export()
        assert np.array_equal(gk, ok) and np.array_equal(gs, os_), (case, step)
        info = g.stats()
        got = {"skipped": info.last_skipped, "cleared": info.last_cleared,
               "expired": info.last_expired}[kind]
        assert got == want, (case, step, kind, got, want)
    g.close()
    o.close()
