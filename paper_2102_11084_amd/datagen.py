"""Seeded synthetic point clouds shaped like the paper's workloads.

The paper measures on RGB-D frames from a simulated corridor and from a depth
camera (Sec. II-D, Sec. II-E); neither recording exists here, so these seeded
generators stand in for them.  This module holds no arithmetic of the
downsampling method: it only draws clouds.  Both the oracle-side tests and the
GPU path consume what it returns, nothing else is shared between them.

RNG: numpy default_rng (PCG64).  Layout: structure of arrays (x, y, z float32,
rgb uint8 n x 3 interleaved), raster order (row v, then column u) for frames.
"""
from __future__ import annotations

import math

import numpy as np

LEAF_CHOICES_BATCH = (0.02, 0.05, 0.10)


def _intrinsics(W, H):
    # 640x480 gives fx = fy = 525, cx = 319.5, cy = 239.5; other sizes keep the
    # horizontal field of view.
    f = 525.0 * W / 640.0
    return f, f, (W - 1) / 2.0, (H - 1) / 2.0


def _scene(rng):
    planes = []
    for _ in range(6):
        nrm = np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6), -1.0])
        nrm /= np.linalg.norm(nrm)
        z0 = rng.uniform(1.5, 4.0)
        planes.append((nrm, z0))
    boxes = []
    for _ in range(10):
        c = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-1.0, 1.0), rng.uniform(1.0, 3.5)])
        h = rng.uniform(0.1, 0.5, size=3)
        boxes.append((c, h))
    colours = rng.integers(0, 256, size=(16, 3))
    return planes, boxes, colours


def rgbd_frame(W, H, seed, invalid_frac=0.10, z_range=(0.5, 4.0)):
    """One ray-cast RGB-D frame: 6 random planes + 10 random axis-aligned boxes.

    Depth z is the nearest positive hit along the pixel ray; no hit or z outside
    z_range gives NaN.  Depth noise sigma = 0.0012 z^2.  Exactly
    round(invalid_frac * W * H) further pixels are set to NaN.  Returns
    (x, y, z, rgb) with W*H points in raster order; invalid points have rgb 0.
    """
    rng = np.random.default_rng(seed)
    planes, boxes, colours = _scene(rng)
    fx, fy, cx, cy = _intrinsics(W, H)
    u = np.arange(W, dtype=np.float64)
    v = np.arange(H, dtype=np.float64)
    dx = np.broadcast_to(((u - cx) / fx)[None, :], (H, W)).reshape(-1)
    dy = np.broadcast_to(((v - cy) / fy)[:, None], (H, W)).reshape(-1)
    npx = W * H
    best = np.full(npx, np.inf)
    prim = np.full(npx, -1, np.int16)
    with np.errstate(divide="ignore", invalid="ignore"):
        for j, (nrm, z0) in enumerate(planes):
            den = nrm[0] * dx + nrm[1] * dy + nrm[2]
            t = (nrm[2] * z0) / den  # plane through (0, 0, z0); ray (dx, dy, 1)
            hit = (t > 0) & (t < best)
            best[hit] = t[hit]
            prim[hit] = j
        inv_dx = 1.0 / dx
        inv_dy = 1.0 / dy
        for j, (c, h) in enumerate(boxes):
            t1x = (c[0] - h[0]) * inv_dx
            t2x = (c[0] + h[0]) * inv_dx
            t1y = (c[1] - h[1]) * inv_dy
            t2y = (c[1] + h[1]) * inv_dy
            t1z, t2z = c[2] - h[2], c[2] + h[2]
            tmin = np.maximum(np.maximum(np.minimum(t1x, t2x), np.minimum(t1y, t2y)), min(t1z, t2z))
            tmax = np.minimum(np.minimum(np.maximum(t1x, t2x), np.maximum(t1y, t2y)), max(t1z, t2z))
            # rays parallel to a slab: inside iff the origin lies within it
            tmin = np.where(dx == 0, np.where(abs(c[0]) <= h[0], tmin, np.inf), tmin)
            tmin = np.where(dy == 0, np.where(abs(c[1]) <= h[1], tmin, np.inf), tmin)
            tnear = np.where(tmin > 0, tmin, tmax)
            hit = (tmax >= tmin) & (tnear > 0) & (tnear < best)
            best[hit] = tnear[hit]
            prim[hit] = 6 + j
    z = best
    valid = np.isfinite(z) & (z >= z_range[0]) & (z <= z_range[1])
    noise = rng.standard_normal(npx)
    z = z + noise * (0.0012 * z * z)
    n_drop = int(round(invalid_frac * npx))
    drop = rng.choice(npx, size=n_drop, replace=False) if n_drop > 0 else np.zeros(0, np.int64)
    valid[drop] = False
    col = colours[np.clip(prim, 0, 15)].astype(np.float64) + rng.normal(0.0, 8.0, size=(npx, 3))
    rgb = np.clip(np.rint(col), 0, 255).astype(np.uint8)
    xs = (dx * z).astype(np.float32)
    ys = (dy * z).astype(np.float32)
    zs = z.astype(np.float32)
    xs[~valid] = np.nan
    ys[~valid] = np.nan
    zs[~valid] = np.nan
    rgb[~valid] = 0
    return xs, ys, zs, rgb


def frame_640x480(seed=1001):
    """640x480 = 307,200 points, 10% invalid (the small single-frame workload)."""
    return rgbd_frame(640, 480, seed)


def frame_1280x720(seed=1002):
    """1280x720 = 921,600 points from the same generator (leaf-sweep workload)."""
    return rgbd_frame(1280, 720, seed)


def room_map(n=16_000_000, seed=1003, room=(20.0, 20.0, 5.0), n_boxes=200, jitter=0.01,
             outlier_frac=0.02, shuffle=True):
    """Accumulated map: floor + 4 walls + boxes on the floor, 1 cm jitter, 2% outliers.

    Surface points are area-proportional; the cloud is shuffled (an accumulated
    map has no raster locality).  Returns (x, y, z, rgb).
    """
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = room
    # surfaces as (origin, edge u, edge v, colour)
    surf = [
        ((0, 0, 0), (Lx, 0, 0), (0, Ly, 0)),
        ((0, 0, 0), (Lx, 0, 0), (0, 0, Lz)),
        ((0, Ly, 0), (Lx, 0, 0), (0, 0, Lz)),
        ((0, 0, 0), (0, Ly, 0), (0, 0, Lz)),
        ((Lx, 0, 0), (0, Ly, 0), (0, 0, Lz)),
    ]
    for _ in range(n_boxes):
        cxy = rng.uniform(1.0, Lx - 1.0, size=2)
        e = rng.uniform(0.2, 1.5, size=3)
        x0, y0 = cxy[0] - e[0] / 2, cxy[1] - e[1] / 2
        x1, y1, z1 = x0 + e[0], y0 + e[1], e[2]
        surf += [
            ((x0, y0, z1), (e[0], 0, 0), (0, e[1], 0)),  # top
            ((x0, y0, 0), (e[0], 0, 0), (0, 0, e[2])),
            ((x0, y1, 0), (e[0], 0, 0), (0, 0, e[2])),
            ((x0, y0, 0), (0, e[1], 0), (0, 0, e[2])),
            ((x1, y0, 0), (0, e[1], 0), (0, 0, e[2])),
        ]
    o = np.array([s[0] for s in surf], np.float64)
    eu = np.array([s[1] for s in surf], np.float64)
    ev = np.array([s[2] for s in surf], np.float64)
    area = np.linalg.norm(np.cross(eu, ev), axis=1)
    colours = rng.integers(0, 256, size=(len(surf), 3))
    n_out = int(round(outlier_frac * n))
    n_srf = n - n_out
    which = rng.choice(len(surf), size=n_srf, p=area / area.sum())
    a = rng.random(n_srf)[:, None]
    b = rng.random(n_srf)[:, None]
    pts = o[which] + a * eu[which] + b * ev[which] + rng.normal(0.0, jitter, size=(n_srf, 3))
    out = rng.random((n_out, 3)) * np.array(room)
    p = np.concatenate([pts, out])
    col = np.concatenate([colours[which], rng.integers(0, 256, size=(n_out, 3))]).astype(np.float64)
    col += rng.normal(0.0, 8.0, size=col.shape)
    rgb = np.clip(np.rint(col), 0, 255).astype(np.uint8)
    if shuffle:
        perm = rng.permutation(n)
        p, rgb = p[perm], rgb[perm]
    p = p.astype(np.float32)
    return (np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
            np.ascontiguousarray(p[:, 2]), np.ascontiguousarray(rgb))


def batch_frame_spec(b, seed_base=4000):
    """Size, valid count and leaf of frame b of the uneven 64-frame batch."""
    rng = np.random.default_rng(seed_base + b)
    v = int(rng.integers(50_000, 900_001))
    f = float(rng.uniform(0.05, 0.30))
    H = int(math.ceil(math.sqrt(v / (1.0 - f) / 0.9 * 0.75)))
    W = int(math.ceil(4 * H / 3))
    leaf = float(LEAF_CHOICES_BATCH[int(rng.integers(0, len(LEAF_CHOICES_BATCH)))])
    return dict(W=W, H=H, n_valid=v, leaf=leaf, frame_seed=int(rng.integers(0, 2**31)))


def batch_frame(b, seed_base=4000):
    """Frame b of the batch: exactly n_valid valid points (random valid pixels NaN'd)."""
    spec = batch_frame_spec(b, seed_base)
    seed = spec["frame_seed"]
    for _ in range(16):
        x, y, z, rgb = rgbd_frame(spec["W"], spec["H"], seed, invalid_frac=0.0)
        valid = np.flatnonzero(np.isfinite(z))
        if valid.size >= spec["n_valid"]:
            break
        seed += 1000
    else:
        raise RuntimeError("could not draw enough valid pixels")
    rng = np.random.default_rng(seed + 7)
    drop = rng.choice(valid, size=valid.size - spec["n_valid"], replace=False)
    x[drop] = np.nan
    y[drop] = np.nan
    z[drop] = np.nan
    rgb[drop] = 0
    return x, y, z, rgb, spec["leaf"]


def batch(n_frames=64, seed_base=4000):
    """Concatenated uneven batch: (x, y, z, rgb, frame_offsets[B+1] int64, leaves[B] float32)."""
    xs, ys, zs, cs, leaves = [], [], [], [], []
    for b in range(n_frames):
        x, y, z, rgb, leaf = batch_frame(b, seed_base)
        xs.append(x), ys.append(y), zs.append(z), cs.append(rgb), leaves.append(leaf)
    offs = np.zeros(n_frames + 1, np.int64)
    offs[1:] = np.cumsum([a.size for a in xs])
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), np.concatenate(cs), offs,
            np.array(leaves, np.float32))


def uniform_cloud(n=100_000, seed=5000, side=2.0):
    """xyz uniform in [0, side)^3 (float32) and uniform rgb."""
    rng = np.random.default_rng(seed)
    p = (rng.random((n, 3)) * side).astype(np.float32)
    rgb = rng.integers(0, 256, size=(n, 3), dtype=np.uint8)
    return (np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
            np.ascontiguousarray(p[:, 2]), rgb)


def upstream_grad(m, seed):
    """Upstream gradient dL/dcentroid ~ N(0, 1), shape (m, 3), float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, 3)).astype(np.float32)


def camera_pose(seed):
    """A depth camera on a ground robot, as a rigid transform of camera points
    into the global frame: optical axes (x right, y down, z forward) turned to
    the robot's (x forward, y left, z up), pitched by up to +-0.2 rad, yawed
    anywhere, mounted 0.3 m up at a random spot of a 10 x 10 m floor.  Returns
    (R 3x3 float32, t 3 float32) with p_global = R p_camera + t."""
    rng = np.random.default_rng(seed)
    yaw, pitch = rng.uniform(-np.pi, np.pi), rng.uniform(-0.2, 0.2)
    cam = np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]], np.float64)
    cp, sp = np.cos(pitch), np.sin(pitch)
    Ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]])
    cy, sy = np.cos(yaw), np.sin(yaw)
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    R = (Rz @ Ry @ cam).astype(np.float32)
    t = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), 0.3], np.float32)
    return R, t
