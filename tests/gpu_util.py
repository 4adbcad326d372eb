"""Helpers shared by the GPU tests: run libvg and compare with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2102_11084_amd import vg


def to_dev(*arrs):
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def gpu_downsample(x, y, z, rgb, leaf, key_mode=vg.KEY_LINEAR, tuning=None):
    dx, dy, dz, drgb = to_dev(x, y, z, None if rgb is None else rgb.reshape(-1))
    r = vg.voxel_downsample(dx, dy, dz, drgb, leaf, key_mode, tuning)
    torch.cuda.synchronize()
    return host(r)


def host(r):
    out = {}
    for k, v in r.items():
        if k == "m":
            out[k] = v
            continue
        a = v.cpu().numpy()
        if k in ("count", "ref_index"):
            a = a.view(np.uint32)
        elif k == "key":
            a = a.view(np.uint64)
        out[k] = a
    return out


def ulp32(v):
    return np.spacing(np.abs(np.asarray(v, np.float64)).astype(np.float32)).astype(np.float64)


def centroid_tol(c64, leaf):
    """Tolerance for binary32 centroids against the FP64 oracle: 1e-6 of the
    cell edge plus one binary32 ulp of the centroid (the output is binary32)."""
    return 1e-6 * leaf + ulp32(c64)


def assert_matches_oracle(g, o, leaf, point_cell_offset=0, ref_offset=0, check_rgb=True):
    """Bit-exact cells/order/counts/refs/colours; centroids and local means to tolerance."""
    m = o["m"]
    assert g["m"] == m, (g["m"], m)
    assert np.array_equal(g["key"], o["key"]), "keys differ"
    assert np.array_equal(g["count"], o["count"]), "counts differ"
    assert np.array_equal(g["ref_index"].astype(np.int64), o["ref_index"] + ref_offset), "refs differ"
    pc = o["point_cell"].astype(np.int64)
    exp_pc = np.where(pc >= 0, pc + point_cell_offset, -1)
    assert np.array_equal(g["point_cell"].astype(np.int64), exp_pc), "point_cell differs"
    if check_rgb and "rgb" in g:
        assert np.array_equal(g["rgb"], o["rgb"]), "colours differ"
    for a, (gk, ok) in enumerate((("x", "cx"), ("y", "cy"), ("z", "cz"))):
        c32 = g[gk].astype(np.float64)
        err = np.abs(c32 - o[ok])
        tol = centroid_tol(o[ok], leaf)
        bad = np.flatnonzero(err > tol)
        assert bad.size == 0, f"centroid axis {a}: {bad.size} cells off, worst {err.max():.3e}"
    for gk, ok in (("lx", "lx"), ("ly", "ly"), ("lz", "lz")):
        if gk in g:
            err = np.abs(g[gk].astype(np.float64) - o[ok])
            assert (err <= 1e-6 * leaf).all(), f"local mean {gk}: worst {err.max() / leaf:.3e} l"


def frame_rows(o_list, status):
    rows = [0]
    for r, s in zip(o_list, status):
        rows.append(rows[-1] + (r["m"] if s == oracle.OK else 0))
    return rows
