"""Points in mapped host memory (the zero-copy ingest): every output
bit-identical to the same call on device-resident points, with and without
graph replay, with and without filters, in both launch forms."""
import numpy as np
import pytest
import torch

from gpu_util import host, to_dev
from paper_2102_11084_amd import datagen as dg
from paper_2102_11084_amd import vg
from test_gpu_batched import small_batch

pytestmark = pytest.mark.gpu


def host_copy(x, y, z, rgb):
    n = x.size
    buf = vg.HostBuffer(15 * n)
    parts = []
    off = 0
    for a, dt in ((x, np.float32), (y, np.float32), (z, np.float32)):
        buf.view(dt, n, off)[:] = a
        parts.append(buf.device + off)
        off += 4 * n
    buf.view(np.uint8, 3 * n, off)[:] = rgb.reshape(-1)
    parts.append(buf.device + off)
    return buf, parts


def same(a, b):
    n = int(a["out_offsets"][-1])
    assert np.array_equal(a["out_offsets"], b["out_offsets"])
    assert np.array_equal(a["frame_status"], b["frame_status"])
    for k in ("x", "y", "z", "rgb", "count", "key", "ref_index", "lx", "ly", "lz"):
        assert np.array_equal(np.ascontiguousarray(a[k][:n]).view(np.uint8),
                              np.ascontiguousarray(b[k][:n]).view(np.uint8)), k
    assert np.array_equal(a["point_cell"], b["point_cell"])


@pytest.mark.parametrize("mode", [vg.EXEC_PHASED, vg.EXEC_PERSISTENT])
@pytest.mark.parametrize("use_graph", [False, True])
def test_host_input_bit_identical(mode, use_graph):
    print(f"case host input, exec mode {mode}, graph {use_graph}", flush=True)
    x, y, z, rgb, offs, leaves = small_batch(seed=11)
    n = x.size
    t = vg.launch_tuning(mode)
    dev_plan = vg.BatchPlan(len(leaves), n, vg.KEY_LINEAR, t, use_graph=use_graph)
    ref = host(dev_plan.run(*to_dev(x, y, z, rgb.reshape(-1)), offs, leaves))
    torch.cuda.synchronize()
    dev_plan.close()
    buf, ptrs = host_copy(x, y, z, rgb)
    plan = vg.BatchPlan(len(leaves), n, vg.KEY_LINEAR, t, use_graph=use_graph)
    plan.set_host_input(True)
    out = plan.alloc_outputs(n, len(leaves), torch.device("cuda"))
    stream = torch.cuda.current_stream()
    for rep in range(2):
        g = host(plan.run_host(*ptrs, n, offs, leaves, out, stream))
        torch.cuda.synchronize()
        same(g, ref)
    plan.close()
    buf.close()


def test_host_input_with_filters():
    x, y, z, rgb, offs, leaves = small_batch(seed=12)
    n = x.size
    rng = np.random.default_rng(3)
    filters = []
    for b in range(len(leaves)):
        R, t = dg.camera_pose(900 + b)
        filters.append(vg.make_filter(rot=R, trans=t, z_min=-0.5, z_max=1.5,
                                      min_points=int(rng.integers(1, 4))))
    dev_plan = vg.BatchPlan(len(leaves), n)
    ref = host(dev_plan.run(*to_dev(x, y, z, rgb.reshape(-1)), offs, leaves, filters=filters))
    torch.cuda.synchronize()
    dev_plan.close()
    buf, ptrs = host_copy(x, y, z, rgb)
    plan = vg.BatchPlan(len(leaves), n)
    plan.set_host_input(True)
    o, cells = plan.alloc_outputs(n, len(leaves), torch.device("cuda"))
    pts = vg.vg_points(*(vg.ctypes.c_void_p(p) for p in ptrs))
    offs64 = np.ascontiguousarray(offs, np.int64)
    lv = np.ascontiguousarray(leaves, np.float32)
    farr = (vg.vg_filter * len(leaves))(*filters)
    st = vg.lib().vg_downsample_batched_filtered(
        plan._h, vg.ctypes.byref(pts), vg.ctypes.c_void_p(offs64.ctypes.data),
        vg.ctypes.c_void_p(lv.ctypes.data), farr, len(leaves), vg.ctypes.byref(cells),
        vg._ptr(o["out_offsets"]), vg._ptr(o["frame_status"]),
        vg.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == vg.VG_OK
    torch.cuda.synchronize()
    same(host(o), ref)
    plan.close()
    buf.close()
