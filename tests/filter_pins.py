"""Pins of the oracle's filtered form (rigid transform into the global frame,
height limit, minimum points per cell), each against something that is not
the filtered oracle itself:

  * the plain voxel filter (pinned on its own in oracle_pins.py) on inputs
    whose transform numpy computes exactly: the identity, dyadic translations
    of dyadic lattices, quarter turns about z (only sign changes and swaps);
  * for a general rotation, the FP64 mean of the FP64-transformed points of a
    single cell (the binary32 transform is within a few ulps of it);
  * the height limit as the plain filter on the input with the points outside
    the limits (bounds included) made invalid;
  * the noise removal as the plain filter's rows with the sparse cells taken
    out and every point's row renumbered.
Each check takes an oracle library handle (test_oracle_mutants.py runs them
on broken builds).
"""
from __future__ import annotations

import numpy as np

import oracle

FIELDS = ("cx", "cy", "cz", "lx", "ly", "lz", "rgb", "count", "key", "ref_index", "point_cell")


def _same(a, b, ctx):
    assert a["m"] == b["m"], (ctx, a["m"], b["m"])
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), (ctx, k)


def _cloud(rng, n, step=1.0 / 64, lo=-2.0, hi=2.0):
    k = rng.integers(int(lo / step), int(hi / step) + 1, size=(n, 3))
    p = (k * step).astype(np.float32)
    p[rng.integers(0, n, max(1, n // 20)), rng.integers(0, 3)] = np.nan
    rgb = rng.integers(0, 256, size=(n, 3), dtype=np.uint8)
    return p, rgb


def pin_filter_identity(lib, seed=21):
    rng = np.random.default_rng(seed)
    for _ in range(5):
        p, rgb = _cloud(rng, int(rng.integers(1, 3000)))
        x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
        a = oracle.downsample_filtered(x, y, z, rgb, 0.25, rot=np.eye(3), trans=np.zeros(3), lib=lib)
        b = oracle.downsample(x, y, z, rgb, 0.25, lib=lib)
        _same(a, b, "identity")
        a = oracle.downsample_filtered(x, y, z, rgb, 0.25, lib=lib)
        _same(a, b, "no transform")


def pin_filter_exact_transforms(lib, seed=22):
    rng = np.random.default_rng(seed)
    quarter = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float32)   # +90 deg about z
    half = np.array([[-1, 0, 0], [0, -1, 0], [0, 0, 1]], np.float32)
    for trial in range(6):
        p, rgb = _cloud(rng, int(rng.integers(50, 3000)))
        x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
        t = (rng.integers(-64, 65, size=3) / 16.0).astype(np.float32)   # dyadic: sums stay exact
        for R in (np.eye(3, dtype=np.float32), quarter, half):
            q = (p.astype(np.float64) @ R.T.astype(np.float64) + t).astype(np.float32)
            a = oracle.downsample_filtered(x, y, z, rgb, 0.25, rot=R, trans=t, lib=lib)
            b = oracle.downsample(q[:, 0], q[:, 1], q[:, 2], rgb, 0.25, lib=lib)
            _same(a, b, (trial, R.tolist()))


def pin_filter_general_rotation(lib, seed=23):
    rng = np.random.default_rng(seed)
    for _ in range(5):
        # a random rotation (QR of a Gaussian matrix) and translation
        Q, _r = np.linalg.qr(rng.normal(size=(3, 3)))
        Q *= np.sign(np.linalg.det(Q))
        R = Q.astype(np.float32)
        t = rng.uniform(-5, 5, 3).astype(np.float32)
        p = rng.uniform(-1, 1, size=(2000, 3)).astype(np.float32)
        x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
        a = oracle.downsample_filtered(x, y, z, None, 64.0, rot=R, trans=t, lib=lib)
        q64 = p.astype(np.float64) @ R.astype(np.float64).T + t.astype(np.float64)
        assert a["m"] == 1 and a["count"][0] == 2000
        mean = q64.mean(0)
        for k, name in enumerate(("cx", "cy", "cz")):
            assert abs(a[name][0] - mean[k]) <= 1e-5, (name, a[name][0], mean[k])
        # a height limit on the transformed z: the kept count matches the FP64
        # transform except for points within rounding of the limits
        zq = q64[:, 2]
        zlo, zhi = np.float32(np.quantile(zq, 0.3)), np.float32(np.quantile(zq, 0.8))
        a = oracle.downsample_filtered(x, y, z, None, 64.0, rot=R, trans=t, z_min=zlo, z_max=zhi, lib=lib)
        inside = (zq >= zlo + 1e-5) & (zq <= zhi - 1e-5)
        border = (np.abs(zq - zlo) < 1e-5) | (np.abs(zq - zhi) < 1e-5)
        assert inside.sum() <= a["count"].sum() <= inside.sum() + border.sum()
        assert (a["point_cell"][inside] == 0).all()


def pin_filter_height_limit(lib, seed=24):
    rng = np.random.default_rng(seed)
    for _ in range(5):
        p, rgb = _cloud(rng, 3000)
        x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
        zlo, zhi = np.float32(-0.5), np.float32(1.25)   # lattice values: points lie on both limits
        assert ((z == zlo) | (z == zhi)).any()
        a = oracle.downsample_filtered(x, y, z, rgb, 0.25, z_min=zlo, z_max=zhi, lib=lib)
        out = ~((z >= zlo) & (z <= zhi))
        xb, yb, zb = x.copy(), y.copy(), z.copy()
        xb[out] = np.nan
        b = oracle.downsample(xb, yb, zb, rgb, 0.25, lib=lib)
        _same(a, b, "height limit")
        # one limit only; empty band
        a = oracle.downsample_filtered(x, y, z, rgb, 0.25, z_min=zlo, lib=lib)
        xb = x.copy()
        xb[~(z >= zlo)] = np.nan
        _same(a, oracle.downsample(xb, y, z, rgb, 0.25, lib=lib), "lower limit")
        a = oracle.downsample_filtered(x, y, z, rgb, 0.25, z_min=9.0, z_max=9.5, lib=lib)
        assert a["m"] == 0 and (a["point_cell"] == -1).all()


def pin_filter_min_points(lib, seed=25):
    rng = np.random.default_rng(seed)
    for k in (1, 2, 3, 7):
        p, rgb = _cloud(rng, 4000, lo=-1.0, hi=1.0)
        x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
        a = oracle.downsample_filtered(x, y, z, rgb, 0.25, min_points=k, lib=lib)
        b = oracle.downsample(x, y, z, rgb, 0.25, lib=lib)
        keep = b["count"] >= k
        assert a["m"] == keep.sum()
        for f in FIELDS[:-1]:
            assert np.array_equal(a[f], b[f][keep]), (k, f)
        new_row = np.cumsum(keep) - 1
        pc = b["point_cell"]
        exp = np.where(pc >= 0, np.where(keep[np.maximum(pc, 0)], new_row[np.maximum(pc, 0)], -1), -1)
        assert np.array_equal(a["point_cell"], exp)
        assert a["count"].astype(np.int64).sum() == (a["point_cell"] >= 0).sum()


def pin_filter_errors(lib):
    x = np.array([0.0, 1.0], np.float32)
    for kw in (dict(z_min=1.0, z_max=0.0), dict(z_min=np.nan), dict(rot=np.eye(3)),
               dict(rot=np.full((3, 3), np.inf), trans=np.zeros(3))):
        try:
            oracle.downsample_filtered(x, x, x, None, 0.5, lib=lib, **kw)
        except oracle.OracleError as e:
            assert e.status == oracle.ERR_ARG
        else:
            raise AssertionError(kw)


ALL_FILTER_PINS = [pin_filter_identity, pin_filter_exact_transforms, pin_filter_general_rotation,
                   pin_filter_height_limit, pin_filter_min_points, pin_filter_errors]
