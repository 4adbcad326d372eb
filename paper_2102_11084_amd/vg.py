"""Thin Python binding of libvg.so (ctypes): argument marshalling only.

Every step of the downsampling runs in the HIP library; torch provides the
device memory (outputs, workspace) and the current stream.  If libvg.so is
missing the calls raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvg.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "vg.h")

VG_OK, VG_ERR_ARG, VG_ERR_LEAF, VG_ERR_GRID_OVERFLOW, VG_ERR_WORKSPACE, VG_ERR_DEVICE = range(6)
KEY_LINEAR, KEY_MORTON = 0, 1
EXEC_PERSISTENT, EXEC_PHASED = 0, 1

P = ctypes.c_void_p


class vg_points(ctypes.Structure):
    _fields_ = [("x", P), ("y", P), ("z", P), ("rgb", P)]


class vg_cells(ctypes.Structure):
    _fields_ = [("x", P), ("y", P), ("z", P), ("rgb", P), ("count", P), ("key", P),
                ("point_cell", P), ("ref_index", P), ("lx", P), ("ly", P), ("lz", P)]


class vg_tuning(ctypes.Structure):
    _fields_ = [("sort_block", ctypes.c_int), ("sort_items", ctypes.c_int),
                ("radix_bits", ctypes.c_int), ("reduce_block", ctypes.c_int),
                ("reduce_items", ctypes.c_int), ("blocks_per_cu", ctypes.c_int),
                ("exec_mode", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vg_options(ctypes.Structure):
    _fields_ = [("stream", P), ("workspace", P), ("workspace_bytes", ctypes.c_size_t),
                ("key_mode", ctypes.c_int), ("tuning", ctypes.POINTER(vg_tuning))]


class vg_nbd_params(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_float), ("radius", ctypes.c_float), ("umbral", ctypes.c_uint32),
                ("round_size", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


NBD_EXACT_SELECT = 1


class vg_nbd_out(ctypes.Structure):
    _fields_ = [("keep_index", P), ("x", P), ("y", P), ("z", P), ("rgb", P), ("count0", P),
                ("marked", P), ("marked_cap", ctypes.c_int64)]


class vg_filter(ctypes.Structure):
    _fields_ = [("rot", ctypes.c_float * 9), ("trans", ctypes.c_float * 3), ("z_min", ctypes.c_float),
                ("z_max", ctypes.c_float), ("min_points", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


FILTER_TRANSFORM = 1


def make_filter(rot=None, trans=None, z_min=-np.inf, z_max=np.inf, min_points=1):
    """vg_filter for one cloud: rot (3x3) and trans (3) together or neither."""
    f = vg_filter()
    if rot is not None or trans is not None:
        R = np.asarray(rot, dtype=np.float32).reshape(9)
        T = np.asarray(trans, dtype=np.float32).reshape(3)
        for k in range(9):
            f.rot[k] = float(R[k])
        for k in range(3):
            f.trans[k] = float(T[k])
        f.flags = FILTER_TRANSFORM
    f.z_min, f.z_max = float(z_min), float(z_max)
    f.min_points = int(min_points)
    return f


class vg_frustum(ctypes.Structure):
    _fields_ = [("rot", ctypes.c_float * 9), ("trans", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("z_near", ctypes.c_float),
                ("z_far", ctypes.c_float)]


class vg_map_info(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("occupied", ctypes.c_int64),
                ("used_slots", ctypes.c_int64), ("last_skipped", ctypes.c_int64),
                ("last_cleared", ctypes.c_int64), ("last_expired", ctypes.c_int64),
                ("full", ctypes.c_int32)]


def make_frustum(rot, trans, fx, fy, cx, cy, width, height, z_near, z_far):
    f = vg_frustum()
    R = np.asarray(rot, dtype=np.float32).reshape(9)
    T = np.asarray(trans, dtype=np.float32).reshape(3)
    for k in range(9):
        f.rot[k] = float(R[k])
    for k in range(3):
        f.trans[k] = float(T[k])
    f.fx, f.fy, f.cx, f.cy = float(fx), float(fy), float(cx), float(cy)
    f.width, f.height = int(width), int(height)
    f.z_near, f.z_far = float(z_near), float(z_far)
    return f


class VGError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = _lib_handle.vg_status_string(status).decode() if _lib_handle else str(status)
        super().__init__(f"{where}: {msg}" if where else msg)


_lib_handle = None

EXPORTS = ["vg_status_string", "vg_default_tuning", "vg_tuning_supported", "vg_workspace_bytes",
           "vg_downsample", "vg_downsample_ex", "vg_downsample_backward", "vg_batch_plan_create",
           "vg_batch_plan_set_graph", "vg_downsample_batched", "vg_batch_plan_set_timing",
           "vg_batch_plan_kernel_times", "vg_batch_plan_set_fail_waits", "vg_batch_plan_destroy",
           "vg_downsample_noalloc", "vg_nbd_workspace_bytes", "vg_nbd_decimate",
           "vg_downsample_filtered", "vg_downsample_batched_filtered", "vg_host_alloc",
           "vg_host_free", "vg_batch_plan_set_host_input", "vg_map_create", "vg_map_destroy",
           "vg_map_mark", "vg_map_clear_frustum", "vg_map_expire", "vg_map_export", "vg_map_compact",
           "vg_map_stats"]

# Largest cloud of vg_downsample_noalloc and the size of its fixed device array.
NOALLOC_MAX_POINTS = 1048576
NOALLOC_SCRATCH_BYTES = 64 << 20

# vg_kernel_kind
KERNEL_KINDS = ("init", "bbox", "hist", "sort", "reduce", "fixup", "pipeline")


def lib():
    """The loaded libvg.so (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.vg_status_string.argtypes = [ctypes.c_int]
        L.vg_status_string.restype = ctypes.c_char_p
        L.vg_default_tuning.argtypes = [ctypes.POINTER(vg_tuning)]
        L.vg_tuning_supported.argtypes = [ctypes.POINTER(vg_tuning)]
        L.vg_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.POINTER(vg_tuning)]
        L.vg_workspace_bytes.restype = ctypes.c_size_t
        L.vg_downsample.argtypes = [ctypes.POINTER(vg_points), ctypes.c_int64, ctypes.c_float,
                                    ctypes.POINTER(vg_cells), ctypes.POINTER(ctypes.c_int64)]
        L.vg_downsample_ex.argtypes = L.vg_downsample.argtypes + [ctypes.POINTER(vg_options)]
        L.vg_downsample_backward.argtypes = [P, P, P, P, ctypes.c_int64, P, ctypes.c_int64, P, P,
                                             P, P]
        L.vg_batch_plan_create.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                           ctypes.POINTER(vg_tuning), ctypes.POINTER(P)]
        L.vg_batch_plan_set_graph.argtypes = [P, ctypes.c_int]
        L.vg_downsample_batched.argtypes = [P, ctypes.POINTER(vg_points), P, P, ctypes.c_int,
                                            ctypes.POINTER(vg_cells), P, P, P]
        L.vg_batch_plan_set_timing.argtypes = [P, ctypes.c_int]
        L.vg_batch_plan_kernel_times.argtypes = [P, P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.vg_batch_plan_set_fail_waits.argtypes = [P, ctypes.c_int]
        L.vg_batch_plan_destroy.argtypes = [P]
        L.vg_downsample_noalloc.argtypes = [ctypes.POINTER(vg_points), ctypes.c_int64,
                                            ctypes.c_float, ctypes.c_int, ctypes.POINTER(vg_cells),
                                            P, P, P]
        L.vg_downsample_filtered.argtypes = [ctypes.POINTER(vg_points), ctypes.c_int64,
                                             ctypes.c_float, ctypes.POINTER(vg_filter),
                                             ctypes.POINTER(vg_cells), ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(vg_options)]
        L.vg_downsample_batched_filtered.argtypes = [P, ctypes.POINTER(vg_points), P, P,
                                                     ctypes.POINTER(vg_filter), ctypes.c_int,
                                                     ctypes.POINTER(vg_cells), P, P, P]
        L.vg_host_alloc.argtypes = [ctypes.c_size_t, ctypes.POINTER(P), ctypes.POINTER(P)]
        L.vg_host_free.argtypes = [P]
        L.vg_batch_plan_set_host_input.argtypes = [P, ctypes.c_int]
        L.vg_map_create.argtypes = [ctypes.c_int64, ctypes.c_float, ctypes.POINTER(P)]
        L.vg_map_destroy.argtypes = [P]
        L.vg_map_mark.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_uint32, P]
        L.vg_map_clear_frustum.argtypes = [P, ctypes.POINTER(vg_frustum), P]
        L.vg_map_expire.argtypes = [P, ctypes.c_uint32, P]
        L.vg_map_export.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P]
        L.vg_map_compact.argtypes = [P, P]
        L.vg_map_stats.argtypes = [P, ctypes.POINTER(vg_map_info), P]
        L.vg_nbd_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
        L.vg_nbd_workspace_bytes.restype = ctypes.c_size_t
        L.vg_nbd_decimate.argtypes = [ctypes.POINTER(vg_points), ctypes.c_int64,
                                      ctypes.POINTER(vg_nbd_params), ctypes.POINTER(vg_nbd_out),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(vg_options)]
        for name in EXPORTS:
            if name not in ("vg_status_string", "vg_workspace_bytes", "vg_nbd_workspace_bytes"):
                getattr(L, name).restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def default_tuning(**over) -> vg_tuning:
    t = vg_tuning()
    lib().vg_default_tuning(ctypes.byref(t))
    for k, v in over.items():
        setattr(t, k, int(v))
    return t


def launch_tuning(exec_mode: int) -> vg_tuning:
    """A built tuning for the given launch form: the default for the phased
    form, the default's shape with 4 reduce items per thread for the one-launch
    form (the shapes it is built for)."""
    if exec_mode == EXEC_PERSISTENT:
        return default_tuning(reduce_items=4, exec_mode=EXEC_PERSISTENT)
    return default_tuning(exec_mode=exec_mode)


def load_tuning(path: str) -> vg_tuning:
    """Tuning written by the autotuner (JSON object with vg_tuning's fields)."""
    import json
    with open(path) as f:
        d = json.load(f)
    d = d.get("tuning", d)
    return default_tuning(**{k: d[k] for k, _ in vg_tuning._fields_ if k in d})


def tuning_supported(t: vg_tuning) -> bool:
    return lib().vg_tuning_supported(ctypes.byref(t)) == VG_OK


def workspace_bytes(n_total: int, n_frames: int = 1, tuning: vg_tuning | None = None) -> int:
    return int(lib().vg_workspace_bytes(int(n_total), int(n_frames),
                                        ctypes.byref(tuning) if tuning is not None else None))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_points(x, y, z, rgb):
    n = x.numel()
    for t in (x, y, z):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n):
            raise ValueError("x, y, z must be contiguous float32 CUDA tensors of equal length")
    if rgb is not None and not (rgb.is_cuda and rgb.dtype == torch.uint8 and rgb.is_contiguous()
                                and rgb.numel() == 3 * n):
        raise ValueError("rgb must be a contiguous uint8 CUDA tensor of n x 3 values")
    return n


ALL_OUTPUTS = ("xyz", "rgb", "count", "key", "point_cell", "ref_index", "local")


def _alloc_cells(cap, n_points, dev, outputs, have_rgb):
    o = {}
    f32 = dict(dtype=torch.float32, device=dev)
    if "xyz" in outputs:
        o["x"], o["y"], o["z"] = (torch.empty(cap, **f32) for _ in range(3))
    if "rgb" in outputs and have_rgb:
        o["rgb"] = torch.empty((cap, 3), dtype=torch.uint8, device=dev)
    if "count" in outputs:
        o["count"] = torch.empty(cap, dtype=torch.int32, device=dev)  # holds uint32
    if "key" in outputs:
        o["key"] = torch.empty(cap, dtype=torch.int64, device=dev)    # holds uint64
    if "point_cell" in outputs:
        o["point_cell"] = torch.empty(n_points, dtype=torch.int32, device=dev)
    if "ref_index" in outputs:
        o["ref_index"] = torch.empty(cap, dtype=torch.int32, device=dev)  # holds uint32
    if "local" in outputs:
        o["lx"], o["ly"], o["lz"] = (torch.empty(cap, **f32) for _ in range(3))
    cells = vg_cells(*(_ptr(o.get(k)) for k in ("x", "y", "z", "rgb", "count", "key",
                                                    "point_cell", "ref_index", "lx", "ly", "lz")))
    return o, cells


def voxel_downsample(x, y, z, rgb=None, leaf=0.05, key_mode=KEY_LINEAR, tuning=None,
                     outputs=ALL_OUTPUTS, workspace=None, filter=None):
    """Voxel-grid centroid filter of one cloud on the GPU (libvg: vg_downsample_ex).

    x, y, z: float32 CUDA tensors [n]; rgb: uint8 CUDA tensor [n, 3] or None.
    Returns a dict of tensors trimmed to the m occupied cells (point_cell has n
    entries) plus "m".  count/ref_index are int32 views of uint32 values; key
    is an int64 view of the uint64 key.
    """
    n = _check_points(x, y, z, rgb)
    dev = x.device
    o, cells = _alloc_cells(max(n, 1), n, dev, outputs, rgb is not None)
    pts = vg_points(_ptr(x), _ptr(y), _ptr(z), _ptr(rgb))
    wsb = workspace_bytes(max(n, 1), 1, tuning)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opts = vg_options(ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream),
                      ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), int(key_mode),
                      ctypes.pointer(tuning) if tuning is not None else None)
    m = ctypes.c_int64(0)
    if filter is None:
        st = lib().vg_downsample_ex(ctypes.byref(pts), n, ctypes.c_float(leaf), ctypes.byref(cells),
                                    ctypes.byref(m), ctypes.byref(opts))
    else:
        st = lib().vg_downsample_filtered(ctypes.byref(pts), n, ctypes.c_float(leaf),
                                          ctypes.byref(filter), ctypes.byref(cells), ctypes.byref(m),
                                          ctypes.byref(opts))
    if st != VG_OK:
        raise VGError(st, "vg_downsample_ex" if filter is None else "vg_downsample_filtered")
    mm = int(m.value)
    res = {k: (v if k == "point_cell" else v[:mm]) for k, v in o.items()}
    res["m"] = mm
    return res


def voxel_downsample_noalloc(x, y, z, rgb=None, leaf=0.05, key_mode=KEY_LINEAR,
                             outputs=ALL_OUTPUTS, out=None):
    """vg_downsample_noalloc: the library allocates nothing (its workspace is a
    fixed device array); fully asynchronous.  `out` = (tensors, vg_cells) from
    an earlier call to reuse outputs; else they are allocated here (by torch,
    for the caller).  Returns (untrimmed output tensors, m, status), m and
    status as one-element device tensors."""
    n = _check_points(x, y, z, rgb)
    dev = x.device
    o, cells = out if out is not None else _alloc_cells(max(n, 1), n, dev, outputs, rgb is not None)
    dm = torch.empty(1, dtype=torch.int64, device=dev)
    ds = torch.empty(1, dtype=torch.int32, device=dev)
    pts = vg_points(_ptr(x), _ptr(y), _ptr(z), _ptr(rgb))
    st = lib().vg_downsample_noalloc(ctypes.byref(pts), n, ctypes.c_float(leaf), int(key_mode),
                                     ctypes.byref(cells), _ptr(dm), _ptr(ds),
                                     ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    if st != VG_OK:
        raise VGError(st, "vg_downsample_noalloc")
    return o, dm, ds


def nbd_decimate(x, y, z, rgb=None, leaf=0.02, radius=None, umbral=16, seed=1, round_size=1000,
                 with_points=True, with_count0=False, workspace=None, tuning=None, marked_cap=1 << 16,
                 exact_select=False):
    """Neighbour-bucket decimation (libvg: vg_nbd_decimate; the paper's Alg. 1).

    Returns dict: keep_index (int32 view of uint32 input indices of the
    survivors, ascending), x/y/z/rgb of the survivors (if with_points),
    count0 (every point's neighbours before any deletion, if with_count0),
    marked (numpy int64, points marked per round), rounds, n_keep."""
    n = _check_points(x, y, z, rgb)
    dev = x.device
    radius = leaf if radius is None else radius
    o = {"keep_index": torch.empty(max(n, 1), dtype=torch.int32, device=dev)}
    if with_points:
        o["x"], o["y"], o["z"] = (torch.empty(max(n, 1), dtype=torch.float32, device=dev)
                                  for _ in range(3))
        if rgb is not None:
            o["rgb"] = torch.empty((max(n, 1), 3), dtype=torch.uint8, device=dev)
    if with_count0:
        o["count0"] = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    marked = np.zeros(marked_cap, np.int64)
    out = vg_nbd_out(_ptr(o["keep_index"]), _ptr(o.get("x")), _ptr(o.get("y")), _ptr(o.get("z")),
                     _ptr(o.get("rgb")), _ptr(o.get("count0")), ctypes.c_void_p(marked.ctypes.data),
                     marked_cap)
    prm = vg_nbd_params(float(leaf), float(radius), int(umbral), int(round_size), int(seed),
                        NBD_EXACT_SELECT if exact_select else 0, 0)
    wsb = int(lib().vg_nbd_workspace_bytes(max(n, 1), int(round_size)))
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    opts = vg_options(ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream),
                      ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), KEY_LINEAR,
                      ctypes.pointer(tuning) if tuning is not None else None)
    nk, nr = ctypes.c_int64(0), ctypes.c_int64(0)
    pts = vg_points(_ptr(x), _ptr(y), _ptr(z), _ptr(rgb))
    st = lib().vg_nbd_decimate(ctypes.byref(pts), n, ctypes.byref(prm), ctypes.byref(out),
                               ctypes.byref(nk), ctypes.byref(nr), ctypes.byref(opts))
    if st != VG_OK:
        raise VGError(st, "vg_nbd_decimate")
    k, r = int(nk.value), int(nr.value)
    res = {key: (v if key == "count0" else v[:k]) for key, v in o.items()}
    res["n_keep"], res["rounds"] = k, r
    res["marked"] = marked[:min(r, marked_cap)].copy()
    return res


def downsample_backward(gx, gy, gz, count, point_cell):
    """dL/dxyz for upstream dL/dcentroid (libvg: vg_downsample_backward)."""
    n = point_cell.numel()
    m = count.numel()
    dev = point_cell.device
    dx, dy, dz = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3))
    for t in (gx, gy, gz):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == m):
            raise ValueError("gradients must be contiguous float32 CUDA tensors [m]")
    st = lib().vg_downsample_backward(_ptr(gx), _ptr(gy), _ptr(gz), _ptr(count), m,
                                      _ptr(point_cell), n, _ptr(dx), _ptr(dy), _ptr(dz),
                                      ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    if st != VG_OK:
        raise VGError(st, "vg_downsample_backward")
    return dx, dy, dz


class VoxelDownsampleFn(torch.autograd.Function):
    """Centroids of the voxel grid as a differentiable function of x, y, z.

    The cell assignment (and so the grid) is held fixed in the backward pass:
    dL/dp_i = dL/dc[cell(i)] / count[cell(i)], zero for invalid points.
    """

    @staticmethod
    def forward(ctx, x, y, z, leaf, key_mode=KEY_LINEAR):
        r = voxel_downsample(x, y, z, None, leaf, key_mode,
                             outputs=("xyz", "count", "point_cell"))
        ctx.save_for_backward(r["count"], r["point_cell"])
        ctx.mark_non_differentiable(r["count"])
        return r["x"], r["y"], r["z"], r["count"]

    @staticmethod
    def backward(ctx, gx, gy, gz, gcount):
        count, pc = ctx.saved_tensors
        m = count.numel()
        dev = pc.device
        gx, gy, gz = (g.contiguous() if g is not None else torch.zeros(m, device=dev)
                      for g in (gx, gy, gz))
        dx, dy, dz = downsample_backward(gx, gy, gz, count, pc)
        return dx, dy, dz, None, None


def voxel_downsample_autograd(x, y, z, leaf, key_mode=KEY_LINEAR):
    return VoxelDownsampleFn.apply(x, y, z, leaf, key_mode)


class HostBuffer:
    """Pinned host memory mapped into the device (vg_host_alloc): `array` is a
    numpy view for filling it on the host, `device` the address the library
    reads it at."""

    def __init__(self, nbytes):
        h, d = ctypes.c_void_p(), ctypes.c_void_p()
        st = lib().vg_host_alloc(int(nbytes), ctypes.byref(h), ctypes.byref(d))
        if st != VG_OK:
            raise VGError(st, "vg_host_alloc")
        self._h, self.device, self.nbytes = h, int(d.value), int(nbytes)
        self.array = np.ctypeslib.as_array((ctypes.c_uint8 * max(int(nbytes), 1)).from_address(h.value))

    def view(self, dtype, count, offset=0):
        return self.array[offset:offset + count * np.dtype(dtype).itemsize].view(dtype)

    def close(self):
        if self._h:
            self.array = None
            lib().vg_host_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Many frames of uneven size and leaf in one launch (vg_downsample_batched)."""

    def __init__(self, max_frames, max_total_points, key_mode=KEY_LINEAR, tuning=None,
                 use_graph=False):
        self._h = ctypes.c_void_p()
        self.tuning = tuning
        st = lib().vg_batch_plan_create(int(max_frames), int(max_total_points), int(key_mode),
                                        ctypes.byref(tuning) if tuning is not None else None,
                                        ctypes.byref(self._h))
        if st != VG_OK:
            raise VGError(st, "vg_batch_plan_create")
        self.max_frames = int(max_frames)
        self.max_total_points = int(max_total_points)
        self.set_graph(use_graph)

    def set_graph(self, use_graph: bool):
        st = lib().vg_batch_plan_set_graph(self._h, 1 if use_graph else 0)
        if st != VG_OK:
            raise VGError(st, "vg_batch_plan_set_graph")

    def set_timing(self, enable: bool):
        """Per-launch HIP event timing of later runs (launches bypass the graph)."""
        st = lib().vg_batch_plan_set_timing(self._h, 1 if enable else 0)
        if st != VG_OK:
            raise VGError(st, "vg_batch_plan_set_timing")

    def set_fail_waits(self, enable: bool):
        """Test support: later runs start with the device time-out flag raised."""
        st = lib().vg_batch_plan_set_fail_waits(self._h, 1 if enable else 0)
        if st != VG_OK:
            raise VGError(st, "vg_batch_plan_set_fail_waits")

    def set_host_input(self, on: bool):
        """Later runs read their points from mapped host memory (run_host)."""
        st = lib().vg_batch_plan_set_host_input(self._h, 1 if on else 0)
        if st != VG_OK:
            raise VGError(st, "vg_batch_plan_set_host_input")

    def run_host(self, xp, yp, zp, rgbp, n, frame_offsets, leaves, out, stream):
        """run() with the points at device addresses of host memory (HostBuffer.device
        plus an offset); `out` from alloc_outputs; `stream` a torch stream."""
        offs = np.ascontiguousarray(frame_offsets, dtype=np.int64)
        lv = np.ascontiguousarray(leaves, dtype=np.float32)
        B = lv.size
        if offs.size != B + 1 or offs[-1] != n:
            raise ValueError("frame_offsets must have B+1 entries ending at n")
        o, cells = out
        pts = vg_points(ctypes.c_void_p(xp), ctypes.c_void_p(yp), ctypes.c_void_p(zp),
                        ctypes.c_void_p(rgbp) if rgbp else None)
        st = lib().vg_downsample_batched(
            self._h, ctypes.byref(pts), ctypes.c_void_p(offs.ctypes.data),
            ctypes.c_void_p(lv.ctypes.data), B, ctypes.byref(cells), _ptr(o["out_offsets"]),
            _ptr(o["frame_status"]), ctypes.c_void_p(stream.cuda_stream))
        if st != VG_OK:
            raise VGError(st, "vg_downsample_batched")
        return o

    def kernel_times(self):
        """[(kind name, ms)] of the last run's kernel launches, in launch order (waits)."""
        cap = 64
        kinds = (ctypes.c_int * cap)()
        ms = (ctypes.c_float * cap)()
        cnt = ctypes.c_int(0)
        st = lib().vg_batch_plan_kernel_times(self._h, ctypes.cast(kinds, ctypes.c_void_p),
                                              ctypes.cast(ms, ctypes.c_void_p), cap,
                                              ctypes.byref(cnt))
        if st != VG_OK:
            raise VGError(st, "vg_batch_plan_kernel_times")
        return [(KERNEL_KINDS[kinds[i]], float(ms[i])) for i in range(cnt.value)]

    def alloc_outputs(self, n_total, B, dev, outputs=ALL_OUTPUTS, have_rgb=True):
        o, cells = _alloc_cells(max(n_total, 1), n_total, dev, outputs, have_rgb)
        o["out_offsets"] = torch.empty(B + 1, dtype=torch.int64, device=dev)
        o["frame_status"] = torch.empty(B, dtype=torch.int32, device=dev)
        return o, cells

    def run(self, x, y, z, rgb, frame_offsets, leaves, outputs=ALL_OUTPUTS, out=None, filters=None):
        """Asynchronous launch; returns untrimmed output tensors (see out_offsets).
        filters: None or a list of vg_filter, one per frame."""
        n = _check_points(x, y, z, rgb)
        offs = np.ascontiguousarray(frame_offsets, dtype=np.int64)
        lv = np.ascontiguousarray(leaves, dtype=np.float32)
        B = lv.size
        if offs.size != B + 1 or offs[-1] != n:
            raise ValueError("frame_offsets must have B+1 entries ending at n")
        if out is None:
            out = self.alloc_outputs(n, B, x.device, outputs, rgb is not None)
        o, cells = out
        pts = vg_points(_ptr(x), _ptr(y), _ptr(z), _ptr(rgb))
        stream = ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
        if filters is None:
            st = lib().vg_downsample_batched(
                self._h, ctypes.byref(pts), ctypes.c_void_p(offs.ctypes.data),
                ctypes.c_void_p(lv.ctypes.data), B, ctypes.byref(cells), _ptr(o["out_offsets"]),
                _ptr(o["frame_status"]), stream)
        else:
            if len(filters) != B:
                raise ValueError("one filter per frame")
            farr = (vg_filter * B)(*filters)
            st = lib().vg_downsample_batched_filtered(
                self._h, ctypes.byref(pts), ctypes.c_void_p(offs.ctypes.data),
                ctypes.c_void_p(lv.ctypes.data), farr, B, ctypes.byref(cells),
                _ptr(o["out_offsets"]), _ptr(o["frame_status"]), stream)
        if st != VG_OK:
            raise VGError(st, "vg_downsample_batched" if filters is None else
                          "vg_downsample_batched_filtered")
        return o

    def close(self):
        if self._h:
            lib().vg_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VoxelMap:
    """Global voxel map on the GPU (vg_map_*): mark a cloud's voxels with a
    time stamp, clear the voxels in a camera frustum, expire old voxels."""

    def __init__(self, capacity, res):
        self._h = ctypes.c_void_p()
        st = lib().vg_map_create(int(capacity), ctypes.c_float(res), ctypes.byref(self._h))
        if st != VG_OK:
            raise VGError(st, "vg_map_create")

    @staticmethod
    def _stream():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def mark(self, x, y, z, stamp):
        n = x.numel()
        for t in (x, y, z):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n):
                raise ValueError("x, y, z must be contiguous float32 CUDA tensors of equal length")
        st = lib().vg_map_mark(self._h, _ptr(x), _ptr(y), _ptr(z), n, int(stamp), self._stream())
        if st != VG_OK:
            raise VGError(st, "vg_map_mark")

    def clear(self, frustum):
        st = lib().vg_map_clear_frustum(self._h, ctypes.byref(frustum), self._stream())
        if st != VG_OK:
            raise VGError(st, "vg_map_clear_frustum")

    def expire(self, min_stamp):
        st = lib().vg_map_expire(self._h, int(min_stamp), self._stream())
        if st != VG_OK:
            raise VGError(st, "vg_map_expire")

    def compact(self):
        st = lib().vg_map_compact(self._h, self._stream())
        if st != VG_OK:
            raise VGError(st, "vg_map_compact")

    def export(self):
        """(keys uint64, stamps uint32) of the occupied voxels, sorted by key (numpy)."""
        info = self.stats()
        cap = max(int(info.occupied), 1)
        keys = torch.empty(cap, dtype=torch.int64, device="cuda")
        stamps = torch.empty(cap, dtype=torch.int32, device="cuda")
        n = ctypes.c_int64(0)
        st = lib().vg_map_export(self._h, _ptr(keys), _ptr(stamps), cap, ctypes.byref(n), self._stream())
        if st != VG_OK:
            raise VGError(st, "vg_map_export")
        k = keys[:n.value].cpu().numpy().view(np.uint64)
        s = stamps[:n.value].cpu().numpy().view(np.uint32)
        order = np.argsort(k, kind="stable")
        return k[order], s[order]

    def stats(self):
        info = vg_map_info()
        st = lib().vg_map_stats(self._h, ctypes.byref(info), self._stream())
        if st != VG_OK:
            raise VGError(st, "vg_map_stats")
        return info

    def close(self):
        if self._h:
            lib().vg_map_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
