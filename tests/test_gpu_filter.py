"""The filtered form on the GPU (transform into the global frame, height
limit, minimum points per cell) against the oracle's filtered form, in the
plain and the batched calls; bit for bit except centroids (parity tolerance)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_matches_oracle, host, to_dev
from paper_2102_11084_amd import datagen as dg
from paper_2102_11084_amd import vg

pytestmark = pytest.mark.gpu


def rotation(rng):
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Q *= np.sign(np.linalg.det(Q))
    return Q.astype(np.float32)


def camera_pose(rng):
    return dg.camera_pose(int(rng.integers(0, 2 ** 31)))


def plain(x, y, z, rgb, leaf, kw):
    d = to_dev(x, y, z, rgb.reshape(-1))
    f = vg.make_filter(**kw)
    r = vg.voxel_downsample(*d, leaf=leaf, filter=f)
    torch.cuda.synchronize()
    return host(r)


CASES = [
    dict(),
    dict(rot=np.eye(3), trans=np.zeros(3)),
    dict(rot=[[0, -1, 0], [1, 0, 0], [0, 0, 1]], trans=[0.5, -1.25, 2.0]),
    dict(z_min=1.0, z_max=2.5),
    dict(min_points=2),
    dict(min_points=7),
    "pose",
    "pose+limit+min",
]


@pytest.mark.parametrize("ci", range(len(CASES)))
@pytest.mark.parametrize("leaf", [0.02, 0.05])
def test_plain_filtered_matches_oracle(ci, leaf):
    rng = np.random.default_rng(100 + ci)
    kw = CASES[ci]
    if kw == "pose":
        R, t = camera_pose(rng)
        kw = dict(rot=R, trans=t)
    elif kw == "pose+limit+min":
        R, t = camera_pose(rng)
        kw = dict(rot=R, trans=t, z_min=0.05, z_max=1.2, min_points=3)
    print(f"case filtered plain {ci} leaf {leaf}: {sorted(kw)}", flush=True)
    x, y, z, rgb = dg.rgbd_frame(320, 240, seed=40 + ci)
    g = plain(x, y, z, rgb, leaf, kw)
    o = oracle.downsample_filtered(x, y, z, rgb, leaf, **kw)
    assert_matches_oracle(g, o, leaf)


def test_plain_filtered_large_frame_general_rotation():
    rng = np.random.default_rng(7)
    R, t = camera_pose(rng)
    kw = dict(rot=R, trans=t, z_min=0.1, z_max=1.5, min_points=2)
    x, y, z, rgb = dg.frame_1280x720()
    g = plain(x, y, z, rgb, 0.02, kw)
    o = oracle.downsample_filtered(x, y, z, rgb, 0.02, **kw)
    assert_matches_oracle(g, o, 0.02)


def test_everything_cropped_and_all_sparse():
    x, y, z, rgb = dg.rgbd_frame(160, 120, seed=3)
    g = plain(x, y, z, rgb, 0.05, dict(z_min=50.0, z_max=60.0))
    assert g["m"] == 0 and (g["point_cell"] == -1).all()
    g = plain(x, y, z, rgb, 1e-4, dict(min_points=2))   # (almost) every cell holds one point
    o = oracle.downsample_filtered(x, y, z, rgb, 1e-4, min_points=2)
    assert_matches_oracle(g, o, 1e-4)


def _batch(seed, B=12):
    rng = np.random.default_rng(seed)
    frames, leaves, kws = [], [], []
    for b in range(B):
        W, H = [(64, 48), (160, 120), (200, 150), (320, 240)][b % 4]
        frames.append(dg.rgbd_frame(W, H, seed=seed * 100 + b))
        leaves.append(float(rng.choice([0.02, 0.05, 0.1])))
        kind = b % 4
        if kind == 0:
            kws.append(dict())
        elif kind == 1:
            R, t = camera_pose(rng)
            kws.append(dict(rot=R, trans=t))
        elif kind == 2:
            kws.append(dict(z_min=1.0, z_max=3.0, min_points=int(rng.integers(2, 5))))
        else:
            R, t = camera_pose(rng)
            kws.append(dict(rot=R, trans=t, z_min=0.0, z_max=1.0, min_points=2))
    offs = np.zeros(B + 1, np.int64)
    offs[1:] = np.cumsum([f[0].size for f in frames])
    cat = [np.concatenate([f[a] for f in frames]) for a in range(4)]
    return cat, offs, np.array(leaves, np.float32), kws


def _check_batch(g, cat, offs, leaves, kws):
    x, y, z, rgb = cat
    oo = g["out_offsets"]
    assert (g["frame_status"] == 0).all()
    for b in range(len(leaves)):
        s0, s1 = int(offs[b]), int(offs[b + 1])
        lo, hi = int(oo[b]), int(oo[b + 1])
        o = oracle.downsample_filtered(x[s0:s1], y[s0:s1], z[s0:s1], rgb[s0:s1], float(leaves[b]),
                                       **kws[b])
        fr = {k: g[k][lo:hi] for k in ("x", "y", "z", "rgb", "count", "key", "ref_index", "lx", "ly", "lz")}
        fr["point_cell"] = g["point_cell"][s0:s1]
        fr["m"] = hi - lo
        assert_matches_oracle(fr, o, float(leaves[b]), point_cell_offset=lo, ref_offset=s0)


@pytest.mark.parametrize("mode", [vg.EXEC_PHASED, vg.EXEC_PERSISTENT])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_filtered_matches_per_frame_oracle(mode, use_graph):
    print(f"case filtered batch, exec mode {mode}, graph {use_graph}", flush=True)
    cat, offs, leaves, kws = _batch(5)
    t = vg.launch_tuning(mode)
    plan = vg.BatchPlan(len(leaves), int(offs[-1]), vg.KEY_LINEAR, t, use_graph=use_graph)
    d = to_dev(cat[0], cat[1], cat[2], cat[3].reshape(-1))
    # an unfiltered call first (a graph then lacks the sparse-cell pass), then
    # filtered calls, then unfiltered again
    plain_g = host(plan.run(*d, offs, leaves))
    torch.cuda.synchronize()
    for rep in range(2):
        g = host(plan.run(*d, offs, leaves, filters=[vg.make_filter(**k) for k in kws]))
        torch.cuda.synchronize()
        _check_batch(g, cat, offs, leaves, kws)
    again = host(plan.run(*d, offs, leaves))
    torch.cuda.synchronize()
    plan.close()
    n = int(plain_g["out_offsets"][-1])
    for k in ("x", "y", "z", "count", "key", "ref_index", "point_cell", "out_offsets"):
        a, b = (plain_g[k], again[k]) if k in ("point_cell", "out_offsets") else (plain_g[k][:n], again[k][:n])
        assert np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8)), k


def test_batched_filtered_equals_plain_filtered_bitwise():
    cat, offs, leaves, kws = _batch(6, B=8)
    x, y, z, rgb = cat
    plan = vg.BatchPlan(len(leaves), int(offs[-1]))
    d = to_dev(x, y, z, rgb.reshape(-1))
    g = host(plan.run(*d, offs, leaves, filters=[vg.make_filter(**k) for k in kws]))
    torch.cuda.synchronize()
    plan.close()
    for b in range(len(leaves)):
        s0, s1 = int(offs[b]), int(offs[b + 1])
        lo, hi = int(g["out_offsets"][b]), int(g["out_offsets"][b + 1])
        p = plain(x[s0:s1], y[s0:s1], z[s0:s1], rgb[s0:s1], float(leaves[b]), kws[b])
        assert p["m"] == hi - lo, b
        for k in ("x", "y", "z", "rgb", "count", "key", "lx", "ly", "lz"):
            assert np.array_equal(p[k].view(np.uint8), g[k][lo:hi].view(np.uint8)), (b, k)
        pc = p["point_cell"].astype(np.int64)
        assert np.array_equal(np.where(pc >= 0, pc + lo, -1), g["point_cell"][s0:s1]), b


def test_min_points_without_count_output():
    """The sparse-cell pass needs counts; when the caller does not ask for
    them it keeps them internally and writes none."""
    x, y, z, rgb = dg.rgbd_frame(200, 150, seed=8)
    d = to_dev(x, y, z, rgb.reshape(-1))
    r = vg.voxel_downsample(*d, leaf=0.05, outputs=("xyz", "point_cell"),
                            filter=vg.make_filter(min_points=4))
    torch.cuda.synchronize()
    o = oracle.downsample_filtered(x, y, z, rgb, 0.05, min_points=4)
    assert r["m"] == o["m"]
    assert np.array_equal(r["point_cell"].cpu().numpy(), o["point_cell"])
    for a, k in (("x", "cx"), ("y", "cy"), ("z", "cz")):
        err = np.abs(r[a].cpu().numpy().astype(np.float64) - o[k])
        assert (err <= 1e-6 * 0.05 + np.spacing(np.abs(o[k]).astype(np.float32))).all()
