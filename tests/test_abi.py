"""The C ABI of libvg.so without a GPU: exports and host-side argument checks.

Every check below returns before anything touches a device, so it runs on the
CPU; calls that would need a device report VG_ERR_DEVICE instead of crashing.
"""
import ctypes
import re

import numpy as np
import pytest

from paper_2102_11084_amd import vg

FAKE = 0x10000  # never dereferenced: every call below fails its host checks first


def header_functions():
    src = open(vg.HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(vg_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_what_the_binding_binds():
    assert header_functions() == sorted(vg.EXPORTS)


@pytest.mark.parametrize("name", header_functions())
def test_library_exports_symbol(name):
    assert hasattr(vg.lib(), name)


def call(n=10, leaf=0.1, pts=None, cells=None, m=True, opts=None):
    L = vg.lib()
    pts = pts if pts is not None else vg.vg_points(FAKE, FAKE, FAKE, None)
    cells = cells if cells is not None else vg.vg_cells()
    mm = ctypes.c_int64(123)
    opts = opts if opts is not None else vg.vg_options(None, None, 0, 0, None)
    st = L.vg_downsample_ex(ctypes.byref(pts), n, ctypes.c_float(leaf), ctypes.byref(cells),
                            ctypes.byref(mm) if m else None, ctypes.byref(opts))
    return st, mm.value


def test_status_strings():
    L = vg.lib()
    for s in range(6):
        assert L.vg_status_string(s).startswith(b"VG_")
    assert L.vg_status_string(99) == b"VG_ERR_UNKNOWN"


@pytest.mark.parametrize("leaf", [0.0, -1.0, float("nan"), float("inf"), -float("inf"), 1e-45])
def test_bad_leaf(leaf):
    st, m = call(leaf=leaf)
    assert st == vg.VG_ERR_LEAF and m == 0


def test_subnormal_leaf_with_finite_reciprocal_passes_the_leaf_check():
    # 2^-127 is subnormal, 1/leaf = 2^127 is finite: not a leaf error (then no device)
    st, _ = call(leaf=2.0 ** -127)
    assert st == vg.VG_ERR_DEVICE


def test_bad_sizes_and_pointers():
    L = vg.lib()
    assert call(n=-1)[0] == vg.VG_ERR_ARG
    assert call(n=1 << 30)[0] == vg.VG_ERR_ARG
    assert call(pts=vg.vg_points(FAKE, None, FAKE, None))[0] == vg.VG_ERR_ARG
    assert call(m=False)[0] == vg.VG_ERR_ARG
    assert call(cells=vg.vg_cells(FAKE, None, None))[0] == vg.VG_ERR_ARG   # partial xyz triple
    assert call(opts=vg.vg_options(None, None, 0, 7, None))[0] == vg.VG_ERR_ARG  # key mode
    mm = ctypes.c_int64(0)
    opts = vg.vg_options(None, None, 0, 0, None)
    assert L.vg_downsample_ex(None, 10, ctypes.c_float(0.1), None, ctypes.byref(mm),
                              ctypes.byref(opts)) == vg.VG_ERR_ARG


def test_empty_cloud_needs_no_device():
    st, m = call(n=0)
    assert st == vg.VG_OK and m == 0


def test_workspace_too_small():
    st, _ = call(opts=vg.vg_options(None, FAKE, 64, 0, None))
    assert st == vg.VG_ERR_WORKSPACE


def test_workspace_bytes():
    t = vg.default_tuning()
    a, b = vg.workspace_bytes(1000, 1, t), vg.workspace_bytes(2_000_000, 1, t)
    assert 0 < a < b
    assert vg.workspace_bytes(-1, 1, t) == 0
    assert vg.workspace_bytes(10, 0, t) == 0
    assert vg.workspace_bytes(2 ** 31, 1, t) == 0


def test_tunings():
    t = vg.default_tuning()
    assert vg.tuning_supported(t)
    t2 = vg.default_tuning()
    t2.reduce_block = t2.sort_block * 2
    assert not vg.tuning_supported(t2)  # one block size for every phase
    assert not vg.tuning_supported(vg.default_tuning(sort_items=5))
    assert not vg.tuning_supported(vg.default_tuning(exec_mode=3))
    bad = vg.default_tuning(sort_items=5)
    assert call(opts=vg.vg_options(None, None, 0, 0, ctypes.pointer(bad)))[0] == vg.VG_ERR_ARG


def test_backward_checks():
    L = vg.lib()
    s = None
    assert L.vg_downsample_backward(None, None, None, None, 0, None, 0, None, None, None, s) == vg.VG_OK
    assert L.vg_downsample_backward(FAKE, FAKE, FAKE, FAKE, 1, FAKE, -1, FAKE, FAKE, FAKE, s) == vg.VG_ERR_ARG
    assert L.vg_downsample_backward(FAKE, FAKE, FAKE, FAKE, 1, None, 5, FAKE, FAKE, FAKE, s) == vg.VG_ERR_ARG
    assert L.vg_downsample_backward(None, FAKE, FAKE, FAKE, 1, FAKE, 5, FAKE, FAKE, FAKE, s) == vg.VG_ERR_ARG


def test_batch_plan_checks():
    L = vg.lib()
    h = ctypes.c_void_p()
    assert L.vg_batch_plan_create(0, 100, 0, None, ctypes.byref(h)) == vg.VG_ERR_ARG
    assert L.vg_batch_plan_create(4, -1, 0, None, ctypes.byref(h)) == vg.VG_ERR_ARG
    assert L.vg_batch_plan_create(4, 100, 5, None, ctypes.byref(h)) == vg.VG_ERR_ARG
    assert L.vg_batch_plan_create(4, 100, 0, None, None) == vg.VG_ERR_ARG
    assert L.vg_downsample_batched(None, None, None, None, 1, None, None, None, None) == vg.VG_ERR_ARG
    assert L.vg_batch_plan_destroy(None) == vg.VG_ERR_ARG
    assert L.vg_batch_plan_set_graph(None, 1) == vg.VG_ERR_ARG
    assert L.vg_batch_plan_set_timing(None, 1) == vg.VG_ERR_ARG
    assert L.vg_batch_plan_set_fail_waits(None, 1) == vg.VG_ERR_ARG
    cnt = ctypes.c_int(5)
    assert L.vg_batch_plan_kernel_times(None, None, None, 0, ctypes.byref(cnt)) == vg.VG_ERR_ARG


def test_filter_arguments_rejected_before_any_launch():
    import ctypes
    L = vg.lib()
    dummy = ctypes.c_void_p(16)
    pts = vg.vg_points(dummy, dummy, dummy, None)
    cells = vg.vg_cells()
    m = ctypes.c_int64(7)
    opts = vg.vg_options()
    for f in (vg.make_filter(z_min=1.0, z_max=0.0), vg.make_filter(z_min=float("nan")),
              vg.make_filter(rot=np.full((3, 3), np.inf), trans=np.zeros(3))):
        st = L.vg_downsample_filtered(ctypes.byref(pts), 10, ctypes.c_float(0.1), ctypes.byref(f),
                                      ctypes.byref(cells), ctypes.byref(m), ctypes.byref(opts))
        assert st == vg.VG_ERR_ARG and m.value == 0
    bad = vg.make_filter()
    bad.flags = 8
    assert L.vg_downsample_filtered(ctypes.byref(pts), 10, ctypes.c_float(0.1), ctypes.byref(bad),
                                    ctypes.byref(cells), ctypes.byref(m),
                                    ctypes.byref(opts)) == vg.VG_ERR_ARG
    assert L.vg_downsample_filtered(ctypes.byref(pts), 10, ctypes.c_float(0.1), None,
                                    ctypes.byref(cells), ctypes.byref(m),
                                    ctypes.byref(opts)) == vg.VG_ERR_ARG


def test_one_launch_form_only_where_built():
    # the one-launch form is built for the shapes with 4 reduce items per thread
    assert vg.tuning_supported(vg.default_tuning(reduce_items=4, exec_mode=vg.EXEC_PERSISTENT))
    assert not vg.tuning_supported(vg.default_tuning(exec_mode=vg.EXEC_PERSISTENT))
    assert vg.tuning_supported(vg.launch_tuning(vg.EXEC_PERSISTENT))
    assert vg.tuning_supported(vg.launch_tuning(vg.EXEC_PHASED))
