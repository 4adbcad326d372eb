"""Pins of the oracle's global voxel map against facts that do not come from
the oracle:
  * voxel keys of dyadic points at a dyadic voxel size, where every binary32
    operation of the key is exact: floor(p / res) in exact rational arithmetic;
  * the frustum of a camera on the global axes or turned by quarter turns (all
    rotation entries 0 or +-1): every voxel centre classified in exact rational
    arithmetic, compared wherever the exact values are not within rounding
    distance of a bound;
  * marking twice keeps the later stamp; expiry by stamp; skipped points.
Each check takes an oracle library handle (test_oracle_mutants.py runs them
on broken builds)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import oracle

H = 1 << 20


def exact_key(p, res):
    k = [int(np.floor(Fraction(float(v)) / Fraction(res))) for v in p]
    if any(not (-H <= c < H) for c in k):
        return None
    return (k[0] + H) | ((k[1] + H) << 21) | ((k[2] + H) << 42)


def decode(key):
    return [int((int(key) >> (21 * a)) & ((1 << 21) - 1)) - H for a in range(3)]


def pin_map_keys(lib, seed=31):
    rng = np.random.default_rng(seed)
    res = 0.125
    p = (rng.integers(-4000, 4000, size=(3000, 3)) / 64.0).astype(np.float32)
    p[:10] = (np.arange(10)[:, None] * res).astype(np.float32)       # on voxel faces
    p[10:20] = -p[:10]
    p[20] = (2.0 ** 20 * res, 0, 0)                                  # first key out of range
    p[21] = (-(2.0 ** 20) * res, 0, 0)                               # last key in range
    p[22, 1] = np.nan
    m = oracle.VoxelMap(res, lib=lib)
    skipped = m.mark(p[:, 0], p[:, 1], p[:, 2], 5)
    keys, stamps = m.export()
    exp = {exact_key(q, res) for q in p if np.isfinite(q).all()}
    assert skipped == 2 and None in exp
    exp.discard(None)
    assert set(int(k) for k in keys) == exp and (stamps == 5).all()
    assert (keys[1:] > keys[:-1]).all()
    m.close()


def pin_map_restamp_and_expire(lib, seed=32):
    rng = np.random.default_rng(seed)
    res = 0.25
    a = (rng.integers(-200, 200, size=(500, 3)) / 16.0).astype(np.float32)
    b = (rng.integers(-200, 200, size=(500, 3)) / 16.0).astype(np.float32)
    b[:250] = a[:250]   # half of b re-marks voxels of a
    m = oracle.VoxelMap(res, lib=lib)
    m.mark(a[:, 0], a[:, 1], a[:, 2], 1)
    m.mark(b[:, 0], b[:, 1], b[:, 2], 2)
    ref = {}
    for q in a:
        ref[exact_key(q, res)] = 1
    for q in b:
        ref[exact_key(q, res)] = 2
    keys, stamps = m.export()
    assert dict(zip((int(k) for k in keys), (int(s) for s in stamps))) == ref
    gone = m.expire(2)
    keys, stamps = m.export()
    assert gone == sum(1 for v in ref.values() if v < 2)
    assert set(int(k) for k in keys) == {k for k, v in ref.items() if v >= 2}
    m.close()


QUARTERS = [np.eye(3), np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]]),   # optical axes on a robot
            np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]]), np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]])]


def exact_inside(key, res, R, t, fx, fy, cx, cy, W, Hh, zn, zf, eps):
    """Exact classification of a voxel centre; None when u or v is within eps
    of a bound.  (With quarter turns and dyadic centres and translations, the
    camera-frame coordinates are exact in binary32 too, so the depth limits
    are decided exactly, bounds included.)"""
    k = decode(key)
    c = [(Fraction(kk) + Fraction(1, 2)) * Fraction(res) for kk in k]
    d = [c[a] - Fraction(float(t[a])) for a in range(3)]
    q = [sum(Fraction(int(R[i][j])) * d[i] for i in range(3)) for j in range(3)]
    if not (Fraction(zn) <= q[2] <= Fraction(zf)):
        return False
    u = Fraction(fx) * q[0] / q[2] + Fraction(cx)
    v = Fraction(fy) * q[1] / q[2] + Fraction(cy)
    lo, hu, hv = Fraction(-1, 2), Fraction(W) - Fraction(1, 2), Fraction(Hh) - Fraction(1, 2)
    for val, hi in ((u, hu), (v, hv)):
        if abs(val - lo) < eps or abs(val - hi) < eps:
            return None
    return lo <= u <= hu and lo <= v <= hv


def pin_map_frustum(lib, seed=33):
    rng = np.random.default_rng(seed)
    res = 0.125
    p = (rng.integers(-64, 64, size=(6000, 3)) / 8.0).astype(np.float32)
    for ri, R in enumerate(QUARTERS):
        t = (rng.integers(-8, 8, size=3) / 4.0).astype(np.float32)
        fx = fy = 16.0
        W, Hh = 32, 24
        cx, cy = (W - 1) / 2.0, (Hh - 1) / 2.0
        m = oracle.VoxelMap(res, lib=lib)
        m.mark(p[:, 0], p[:, 1], p[:, 2], 1)
        before, _ = m.export()
        zn, zf = 0.5625, 5.9375   # odd sixteenths: voxel centres lie on both limits
        cleared = m.clear(R, t, fx, fy, cx, cy, W, Hh, zn, zf)
        after, _ = m.export()
        left = set(int(k) for k in after)
        assert len(before) - len(after) == cleared
        ins = outs = 0
        for key in before:
            e = exact_inside(int(key), res, R, t, fx, fy, cx, cy, W, Hh, zn, zf, Fraction(1, 10000))
            if e is None:
                continue
            if e:
                assert int(key) not in left, (ri, decode(key))
                ins += 1
            else:
                assert int(key) in left, (ri, decode(key))
                outs += 1
        assert ins > 50 and outs > 50, (ins, outs)
        m.close()


def pin_map_errors(lib):
    for res in (0.0, -1.0, float("nan"), float("inf")):
        try:
            oracle.VoxelMap(res, lib=lib)
        except oracle.OracleError:
            continue
        raise AssertionError(res)


ALL_MAP_PINS = [pin_map_keys, pin_map_restamp_and_expire, pin_map_frustum, pin_map_errors]
