"""Backward kernel and autograd function against the oracle gradient.

The oracle gradient is itself pinned by FP64 finite differences on the CPU;
here the GPU gradient is also checked directly against finite differences of
the oracle's fixed-assignment centroids.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import to_dev
from paper_2102_11084_amd import datagen as dg
from paper_2102_11084_amd import vg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("c", [0, 1, 2, 31])
def test_backward_cloud_matches_oracle(c):
    x, y, z, _ = dg.uniform_cloud(100_000, seed=5000 + c)
    leaf = 0.05
    xs = [t.requires_grad_(True) for t in to_dev(x, y, z)]
    cx, cy, cz, cnt = vg.voxel_downsample_autograd(*xs, leaf)
    m = cx.numel()
    G = dg.upstream_grad(m, seed=6000 + c)
    Gd = torch.from_numpy(G).cuda()
    (cx * Gd[:, 0] + cy * Gd[:, 1] + cz * Gd[:, 2]).sum().backward()
    gpu = np.stack([t.grad.cpu().numpy() for t in xs], 1).astype(np.float64)
    o = oracle.downsample(x, y, z, None, leaf)
    assert o["m"] == m
    ref = np.stack(oracle.backward(G[:, 0], G[:, 1], G[:, 2], o["count"], o["point_cell"]), 1)
    err = np.abs(gpu - ref)
    assert (err <= 1e-6 * np.maximum(np.abs(ref), 1e-30) + 1e-30).all(), err.max()
    # finite differences of the fixed-assignment centroids (FP64, h = 1e-4)
    P = np.stack([x, y, z], 1).astype(np.float64)
    pc = o["point_cell"]
    Gf = G.astype(np.float64)

    def loss(Q):
        cc = oracle.centroids_fixed(Q[:, 0], Q[:, 1], Q[:, 2], pc, m)
        return float(sum((Gf[:, a] * cc[a]).sum() for a in range(3)))

    rng = np.random.default_rng(c)
    for _ in range(16):
        i, a = int(rng.integers(0, x.size)), int(rng.integers(0, 3))
        Qp, Qm = P.copy(), P.copy()
        Qp[i, a] += 1e-4
        Qm[i, a] -= 1e-4
        fd = (loss(Qp) - loss(Qm)) / 2e-4
        assert abs(fd - gpu[i, a]) <= 1e-6 * max(1.0, abs(fd))


def test_backward_invalid_points_get_zero():
    x, y, z, rgb = dg.rgbd_frame(160, 120, seed=3)
    xs = [t.requires_grad_(True) for t in to_dev(x, y, z)]
    cx, cy, cz, cnt = vg.voxel_downsample_autograd(*xs, 0.05)
    (cx.sum() + cy.sum() + cz.sum()).backward()
    g = xs[0].grad.cpu().numpy()
    bad = ~np.isfinite(z)
    assert (g[bad] == 0).all()
    assert (g[~bad] > 0).all()
    # every valid point receives 1/count of its cell
    o = oracle.downsample(x, y, z, None, 0.05)
    exp = 1.0 / o["count"][o["point_cell"][~bad]].astype(np.float64)
    assert np.allclose(g[~bad], exp, rtol=1e-6, atol=0)


def test_backward_direct_call():
    m, n = 5, 12
    gx = torch.arange(m, dtype=torch.float32, device="cuda")
    gy, gz = gx * 2, gx * 3
    count = torch.tensor([1, 2, 3, 4, 2], dtype=torch.int32, device="cuda")
    pc = torch.tensor([0, 1, 1, -1, 2, 2, 2, 3, 3, 3, 3, 4], dtype=torch.int32, device="cuda")
    dx, dy, dz = vg.downsample_backward(gx, gy, gz, count, pc)
    exp = np.array([0, .5, .5, 0, 2 / 3, 2 / 3, 2 / 3, .75, .75, .75, .75, 2.0], np.float32)
    assert np.allclose(dx.cpu().numpy(), exp, rtol=1e-7, atol=0)
    assert np.allclose(dz.cpu().numpy(), 3 * exp, rtol=1e-6, atol=0)


@pytest.mark.slow
def test_all_clouds_batched_forward_and_backward():
    """The 32 x 100k clouds as the benchmark runs them: one batched forward
    (every cloud against the oracle), then the backward on the batch's rows
    against the oracle gradient of every cloud and FP64 finite differences of
    the fixed-assignment centroids at sampled coordinates of every cloud."""
    print("case 32 x 100k clouds, batched forward + backward", flush=True)
    leaf = 0.05
    clouds = [dg.uniform_cloud(100_000, seed=5000 + c) for c in range(32)]
    offs = np.arange(33, dtype=np.int64) * 100_000
    x, y, z = (np.concatenate([cl[a] for cl in clouds]) for a in range(3))
    d = to_dev(x, y, z)
    plan = vg.BatchPlan(32, x.size, vg.KEY_LINEAR)
    o = plan.run(d[0], d[1], d[2], None, offs, np.full(32, leaf, np.float32),
                 outputs=("xyz", "count", "key", "point_cell", "ref_index", "local"))
    torch.cuda.synchronize()
    plan.close()
    assert (o["frame_status"].cpu().numpy() == 0).all()
    oo = o["out_offsets"].cpu().numpy()
    mt = int(oo[-1])
    res = []
    Gs = []
    for c in range(32):
        s0, s1 = int(offs[c]), int(offs[c + 1])
        lo, hi = int(oo[c]), int(oo[c + 1])
        r = oracle.downsample(x[s0:s1], y[s0:s1], z[s0:s1], None, leaf)
        fr = {k: o[k][lo:hi].cpu().numpy() for k in ("x", "y", "z", "count", "key", "ref_index",
                                                     "lx", "ly", "lz")}
        fr["count"] = fr["count"].view(np.uint32)
        fr["key"] = fr["key"].view(np.uint64)
        fr["ref_index"] = fr["ref_index"].view(np.uint32)
        fr["point_cell"] = o["point_cell"][s0:s1].cpu().numpy()
        fr["m"] = hi - lo
        from gpu_util import assert_matches_oracle
        assert_matches_oracle(fr, r, leaf, point_cell_offset=lo, ref_offset=s0, check_rgb=False)
        res.append(r)
        Gs.append(dg.upstream_grad(r["m"], seed=6000 + c))
    G = np.concatenate(Gs)
    assert G.shape[0] == mt
    Gd = torch.from_numpy(G).cuda()
    gx, gy, gz = (Gd[:, a].contiguous() for a in range(3))
    dx, dy, dz = vg.downsample_backward(gx, gy, gz, o["count"][:mt], o["point_cell"])
    torch.cuda.synchronize()
    gpu = np.stack([t.cpu().numpy() for t in (dx, dy, dz)], 1).astype(np.float64)
    rng = np.random.default_rng(77)
    for c in range(32):
        s0, s1 = int(offs[c]), int(offs[c + 1])
        r, Gc = res[c], Gs[c]
        ref = np.stack(oracle.backward(Gc[:, 0], Gc[:, 1], Gc[:, 2], r["count"], r["point_cell"]), 1)
        err = np.abs(gpu[s0:s1] - ref)
        assert (err <= 1e-6 * np.maximum(np.abs(ref), 1e-30) + 1e-30).all(), (c, err.max())
        P = np.stack([x[s0:s1], y[s0:s1], z[s0:s1]], 1).astype(np.float64)
        pc, m = r["point_cell"], r["m"]
        Gf = Gc.astype(np.float64)

        def loss(Q):
            cc = oracle.centroids_fixed(Q[:, 0], Q[:, 1], Q[:, 2], pc, m)
            return float(sum((Gf[:, a] * cc[a]).sum() for a in range(3)))

        for _ in range(4):
            i, a = int(rng.integers(0, s1 - s0)), int(rng.integers(0, 3))
            Qp, Qm = P.copy(), P.copy()
            Qp[i, a] += 1e-4
            Qm[i, a] -= 1e-4
            fd = (loss(Qp) - loss(Qm)) / 2e-4
            assert abs(fd - gpu[s0 + i, a]) <= 1e-6 * max(1.0, abs(fd)), (c, i, a)
