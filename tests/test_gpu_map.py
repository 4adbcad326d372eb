"""The global voxel map on the GPU against the oracle's map: the occupied
voxels and their stamps after every operation of seeded sequences of marks,
frustum clears and expiries, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import to_dev
from paper_2102_11084_amd import datagen as dg
from paper_2102_11084_amd import vg

pytestmark = pytest.mark.gpu


def same(g, o, ctx):
    gk, gs = g.export()
    ok, os_ = o.export()
    assert np.array_equal(gk, ok), (ctx, gk.size, ok.size)
    assert np.array_equal(gs, os_), ctx


def frustum_args(R, t, W=640, H=480, zn=0.3, zf=4.0):
    f = 525.0 * W / 640.0
    return (R, t, f, f, (W - 1) / 2.0, (H - 1) / 2.0, W, H, zn, zf)


@pytest.mark.parametrize("res", [0.05, 0.1])
def test_random_sequence_matches_oracle(res):
    rng = np.random.default_rng(int(res * 1000))
    g = vg.VoxelMap(1 << 20, res)
    o = oracle.VoxelMap(res)
    last = {"skipped": 0, "cleared": 0, "expired": 0}  # the oracle's count of the last op of each kind
    for step in range(12):
        op = step % 4
        if op in (0, 1):
            n = int(rng.integers(1, 200000))
            p = rng.uniform(-6, 6, size=(n, 3)).astype(np.float32)
            p[rng.integers(0, n, n // 50), rng.integers(0, 3)] = np.nan
            p[:3] = [[1e9, 0, 0], [-1e9, 1, 1], [0.0, 0.0, -0.0]]   # out of range; signed zero
            x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
            g.mark(*to_dev(x, y, z), step + 1)
            last["skipped"] = o.mark(x, y, z, step + 1)
        elif op == 2:
            R, t = dg.camera_pose(int(rng.integers(0, 1 << 30)))
            args = frustum_args(R, t)
            g.clear(vg.make_frustum(*args))
            last["cleared"] = o.clear(*args)
        else:
            g.expire(step - 1)
            last["expired"] = o.expire(step - 1)
        torch.cuda.synchronize()
        same(g, o, (res, step))
        info = g.stats()
        assert info.full == 0
        got = {"skipped": info.last_skipped, "cleared": info.last_cleared,
               "expired": info.last_expired}
        assert got == last, (res, step, got, last)
    g.compact()
    torch.cuda.synchronize()
    same(g, o, (res, "compact"))
    info = g.stats()
    assert info.used_slots == info.occupied
    g.close()
    o.close()


def test_frames_marked_and_cleared_like_the_costmap():
    """Frames filtered into the global frame, each first clearing its own
    frustum then marking its cells (the layer's per-frame order)."""
    g = vg.VoxelMap(1 << 20, 0.05)
    o = oracle.VoxelMap(0.05)
    for b in range(6):
        x, y, z, rgb = dg.rgbd_frame(320, 240, seed=600 + b)
        R, t = dg.camera_pose(8000 + b)
        W, H = 320, 240
        args = frustum_args(R, t, W, H, 0.5, 4.0)
        d = to_dev(x, y, z, rgb.reshape(-1))
        r = vg.voxel_downsample(*d, leaf=0.05, filter=vg.make_filter(rot=R, trans=t, z_min=0.05, z_max=2.0),
                                outputs=("xyz",))
        g.clear(vg.make_frustum(*args))
        o.clear(*args)
        g.mark(r["x"], r["y"], r["z"], b + 1)
        o.mark(r["x"].cpu().numpy(), r["y"].cpu().numpy(), r["z"].cpu().numpy(), b + 1)
        torch.cuda.synchronize()
        same(g, o, b)
    g.close()
    o.close()


def test_argument_checks():
    with pytest.raises(vg.VGError):
        vg.VoxelMap(1 << 10, 0.0)
    g = vg.VoxelMap(1 << 10, 0.1)
    e = torch.zeros(4, device="cuda")
    with pytest.raises(vg.VGError):
        g.mark(e, e, e, 0)   # stamp 0 is reserved for free voxels
    bad = vg.make_frustum(np.eye(3), np.zeros(3), 1, 1, 0, 0, 0, 10, 0.1, 1.0)
    with pytest.raises(vg.VGError):
        g.clear(bad)
    g.close()
