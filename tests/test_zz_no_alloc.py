"""The entry point that allocates nothing, against vg_downsample_ex.

Two calls in a row on the one fixed device array, the second on a smaller
cloud (the array keeps the first call's contents), each compared bit for bit
with vg_downsample_ex on the same cloud and with the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_matches_oracle, gpu_downsample, host, to_dev
from paper_2102_11084_amd import datagen as dg
from paper_2102_11084_amd import vg


def test_noalloc_rejects_too_large_before_any_launch():
    # host-side size check: no device is touched, so this runs without a GPU
    L = vg.lib()
    dummy = ctypes.c_void_p(16)
    pts = vg.vg_points(dummy, dummy, dummy, None)
    cells = vg.vg_cells()
    st = L.vg_downsample_noalloc(ctypes.byref(pts), vg.NOALLOC_MAX_POINTS + 1, ctypes.c_float(0.05),
                                 0, ctypes.byref(cells), dummy, dummy, None)
    assert st == vg.VG_ERR_WORKSPACE
    assert L.vg_downsample_noalloc(None, 10, ctypes.c_float(0.05), 0, ctypes.byref(cells), dummy,
                                   dummy, None) == vg.VG_ERR_ARG
    # the documented maximum fits the fixed array
    assert vg.workspace_bytes(vg.NOALLOC_MAX_POINTS, 1) <= vg.NOALLOC_SCRATCH_BYTES


@pytest.mark.gpu
@pytest.mark.parametrize("key_mode", [vg.KEY_LINEAR, vg.KEY_MORTON])
def test_noalloc_matches_ex_twice_second_smaller(key_mode):
    cases = [(dg.frame_640x480(), 0.02), (dg.rgbd_frame(200, 150, seed=77), 0.05)]
    for i, ((x, y, z, rgb), leaf) in enumerate(cases):
        print(f"case noalloc call {i}: {x.size} points, leaf {leaf}, key mode {key_mode}", flush=True)
        d = to_dev(x, y, z, rgb.reshape(-1))
        o, dm, ds = vg.voxel_downsample_noalloc(*d, leaf=leaf, key_mode=key_mode)
        torch.cuda.synchronize()
        assert int(ds.item()) == vg.VG_OK
        m = int(dm.item())
        g = host({k: (v if k == "point_cell" else v[:m]) for k, v in o.items()})
        g["m"] = m
        e = gpu_downsample(x, y, z, rgb, leaf, key_mode=key_mode)
        assert e["m"] == m
        for k in ("x", "y", "z", "rgb", "count", "key", "ref_index", "point_cell", "lx", "ly", "lz"):
            assert np.array_equal(np.ascontiguousarray(g[k]).view(np.uint8),
                                  np.ascontiguousarray(e[k]).view(np.uint8)), (i, k)
        r = oracle.downsample(x, y, z, rgb, leaf, key_mode)
        assert_matches_oracle(g, r, leaf)


@pytest.mark.gpu
def test_noalloc_reports_overflow_on_device():
    x = np.array([0.0, 1e4, 5.0], np.float32)
    zz = np.zeros(3, np.float32)
    d = to_dev(x, zz, zz.copy(), None)
    o, dm, ds = vg.voxel_downsample_noalloc(d[0], d[1], d[2], None, leaf=1e-3)
    torch.cuda.synchronize()
    assert int(ds.item()) == vg.VG_ERR_GRID_OVERFLOW and int(dm.item()) == 0
    # and the next call on the same array is right again
    x, y, z, rgb = dg.rgbd_frame(64, 48, seed=5)
    d = to_dev(x, y, z, rgb.reshape(-1))
    o, dm, ds = vg.voxel_downsample_noalloc(*d, leaf=0.05)
    torch.cuda.synchronize()
    m = int(dm.item())
    g = host({k: (v if k == "point_cell" else v[:m]) for k, v in o.items()})
    g["m"] = m
    assert_matches_oracle(g, oracle.downsample(x, y, z, rgb, 0.05), 0.05)
