"""Neighbour-bucket decimation (the paper's Alg. 1) on the GPU against the
oracle: survivors, every point's initial neighbour count, the points marked in
every round and the number of rounds, all bit for bit (integer results; the
distance decisions are taken in binary32 on both sides by the same formula)."""
import numpy as np
import pytest
import torch

import nbd_pins
import oracle
from gpu_util import to_dev
from paper_2102_11084_amd import datagen as dg
from paper_2102_11084_amd import vg

pytestmark = pytest.mark.gpu


def run_both(x, y, z, rgb, leaf, radius, umbral, seed, rs):
    d = to_dev(x, y, z, None if rgb is None else rgb.reshape(-1))
    g = vg.nbd_decimate(*d, leaf=leaf, radius=radius, umbral=umbral, seed=seed, round_size=rs,
                        with_count0=True)
    torch.cuda.synchronize()
    o = oracle.nbd_decimate(x, y, z, leaf, radius, umbral, seed, rs)
    return g, o


def check(g, o, x, y, z, rgb, ctx):
    assert g["rounds"] == o["rounds"], (ctx, g["rounds"], o["rounds"])
    assert np.array_equal(g["marked"], o["marked"]), ctx
    assert np.array_equal(g["count0"].cpu().numpy().view(np.uint32), o["count0"]), ctx
    ki = g["keep_index"].cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(ki, np.flatnonzero(o["keep"])), ctx
    for a, arr in zip(("x", "y", "z"), (x, y, z)):
        assert np.array_equal(g[a].cpu().numpy().view(np.uint32), arr[ki].view(np.uint32)), (ctx, a)
    if rgb is not None:
        assert np.array_equal(g["rgb"].cpu().numpy(), rgb.reshape(-1, 3)[ki]), ctx


@pytest.mark.parametrize("case", [
    ((64, 48), 11, 0.05, 0.05, 8, 100),
    ((160, 120), 12, 0.05, 0.05, 16, 100),
    ((160, 120), 13, 0.02, 0.02, 4, 1000),
    ((200, 150), 14, 0.1, 0.06, 30, 7),
    ((320, 240), 15, 0.02, 0.02, 16, 1000),
    ((320, 240), 16, 0.05, 0.05, 0, 1000),
    ((97, 33), 17, 0.25, 0.25, 500, 1),
], ids=lambda c: f"{c[0][0]}x{c[0][1]}-l{c[2]}-r{c[3]}-u{c[4]}-k{c[5]}")
def test_frames_match_oracle(case):
    (W, H), seed, leaf, radius, umbral, rs = case
    print(f"case nbd {W}x{H} leaf {leaf} radius {radius} umbral {umbral} round {rs}", flush=True)
    x, y, z, rgb = dg.rgbd_frame(W, H, seed=seed)
    g, o = run_both(x, y, z, rgb, leaf, radius, umbral, seed, rs)
    check(g, o, x, y, z, rgb, case)


def test_random_clouds_with_duplicates_and_faces():
    rng = np.random.default_rng(3)
    for trial in range(6):
        n = int(rng.integers(1, 30000))
        leaf = float(rng.choice([0.05, 0.1]))
        p = rng.uniform(0.0, 1.0, size=(n, 3)).astype(np.float32)
        p[rng.integers(0, n, n // 10)] = p[rng.integers(0, n, n // 10)]
        p[rng.integers(0, n, n // 20), 1] = np.float32(leaf) * rng.integers(0, 10, n // 20)
        p[rng.integers(0, n, n // 50), rng.integers(0, 3)] = np.nan
        x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
        rs = int(rng.choice([1, 50, 1000]))
        umbral = int(rng.integers(0, 20))
        print(f"case nbd random cloud {trial}: n {n} leaf {leaf} umbral {umbral} round {rs}", flush=True)
        g, o = run_both(x, y, z, None, leaf, leaf, umbral, trial, rs)
        check(g, o, x, y, z, None, trial)


@pytest.mark.parametrize("rs", [1, 37, 1000])
def test_exact_select_gives_the_same_deletions(rs):
    """The exact select over every marked point (used when the priority window
    holds too few candidates) against the oracle and the windowed path."""
    print(f"case nbd exact select, round size {rs}", flush=True)
    x, y, z, rgb = dg.rgbd_frame(160, 120, seed=31)
    d = to_dev(x, y, z, rgb.reshape(-1))
    a = vg.nbd_decimate(*d, leaf=0.05, umbral=20, seed=9, round_size=rs, with_count0=True,
                        exact_select=True)
    b = vg.nbd_decimate(*d, leaf=0.05, umbral=20, seed=9, round_size=rs, with_count0=True)
    torch.cuda.synchronize()
    o = oracle.nbd_decimate(x, y, z, 0.05, 0.05, 20, 9, rs)
    check(a, o, x, y, z, rgb, ("exact", rs))
    check(b, o, x, y, z, rgb, ("window", rs))


def test_lattice_closed_form():
    s = 1.0 / 16
    x, y, z = nbd_pins.lattice(12, s)
    d = to_dev(x, y, z)
    g = vg.nbd_decimate(*d, leaf=s, radius=s, umbral=5, seed=1, round_size=1000, with_count0=True)
    k = np.stack([x, y, z], 1) / s
    interior = (((k == 0) | (k == 11)).sum(1)) == 0
    assert g["rounds"] == 1 and list(g["marked"]) == [1000]
    ki = g["keep_index"].cpu().numpy().view(np.uint32)
    assert np.array_equal(ki, np.flatnonzero(~interior))
    assert np.array_equal(g["count0"].cpu().numpy(), (6 - (((k == 0) | (k == 11)).sum(1))).astype(np.int32))


def test_coincident_cluster_many_rounds():
    far = np.array([[10.0, 10.0, 10.0], [20.0, 0.0, 0.0], [0.0, 20.0, 5.0]], np.float32)
    p = np.concatenate([np.full((2500, 3), 0.25, np.float32), far])
    x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
    g, o = run_both(x, y, z, None, 0.5, 0.5, 10, 5, 1000)
    assert list(g["marked"]) == [2500, 1500, 500] and g["rounds"] == 3
    check(g, o, x, y, z, None, "cluster")


def test_last_round_below_the_bound():
    """Two coincident clusters: the first round's deletions unmark the smaller
    cluster at once, so the second round holds fewer than round_size marked
    points although the bound carried over from the first round (its count
    less its deletions) is above round_size: that round deletes every marked
    point and is the last."""
    p = np.concatenate([np.full((1500, 3), 0.25, np.float32), np.full((600, 3), 5.25, np.float32)])
    x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
    print("case nbd two clusters 1500 + 600 umbral 550 round 1000", flush=True)
    g, o = run_both(x, y, z, None, 0.5, 0.5, 550, 5, 1000)
    assert list(o["marked"]) == [2100, 773] and o["rounds"] == 2
    check(g, o, x, y, z, None, "two clusters")


def test_edge_cases():
    e = np.zeros(0, np.float32)
    d = to_dev(e, e, e)
    g = vg.nbd_decimate(*d, leaf=0.1, umbral=1)
    assert g["n_keep"] == 0 and g["rounds"] == 1 and list(g["marked"]) == [0]
    nan = np.full(500, np.nan, np.float32)
    g, o = run_both(nan, nan.copy(), nan.copy(), None, 0.1, 0.1, 1, 1, 10)
    assert g["n_keep"] == 0 and g["rounds"] == o["rounds"] == 1
    one = np.array([0.5], np.float32)
    g, o = run_both(one, one.copy(), one.copy(), None, 0.1, 0.1, 0, 1, 10)
    check(g, o, one, one, one, None, "one")
    x = np.array([0.0, 1e4, 5.0], np.float32)
    zz = np.zeros(3, np.float32)
    with pytest.raises(vg.VGError) as err:
        vg.nbd_decimate(*to_dev(x, zz, zz.copy()), leaf=1e-3, radius=1e-3)
    assert err.value.status == vg.VG_ERR_GRID_OVERFLOW
    with pytest.raises(vg.VGError) as err:
        vg.nbd_decimate(*to_dev(x, zz, zz.copy()), leaf=0.1, radius=0.2)
    assert err.value.status == vg.VG_ERR_ARG


def test_deterministic():
    x, y, z, rgb = dg.rgbd_frame(320, 240, seed=21)
    d = to_dev(x, y, z, rgb.reshape(-1))
    a = vg.nbd_decimate(*d, leaf=0.02, umbral=12, seed=3, with_count0=True)
    b = vg.nbd_decimate(*d, leaf=0.02, umbral=12, seed=3, with_count0=True)
    for k in ("keep_index", "x", "y", "z", "rgb", "count0"):
        assert torch.equal(a[k], b[k]), k
    assert np.array_equal(a["marked"], b["marked"])


@pytest.mark.slow
def test_full_frame_matches_oracle():
    """The benchmarked workload: a 640x480 frame, leaf and radius 0.02 m,
    umbral 16, 1000 points per round (about 200 rounds)."""
    print("case nbd 640x480 leaf 0.02 umbral 16 round 1000", flush=True)
    x, y, z, rgb = dg.frame_640x480()
    g, o = run_both(x, y, z, rgb, 0.02, 0.02, 16, 7, 1000)
    check(g, o, x, y, z, rgb, "640x480")
