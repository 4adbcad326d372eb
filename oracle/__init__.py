"""CPU oracle for voxel-grid centroid downsampling (arXiv 2102.11084, Sec. II-C).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package never imports the product.

`vgo.cpp` holds the arithmetic (std::map grouping, FP64 accumulation, see its
header for the readings of the paper it takes); this module only builds it with
g++ and marshals numpy arrays through ctypes.  Batched clouds are handled by
calling the single-cloud oracle once per frame, which is what a batch means.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vgo.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_LEAF, ERR_GRID_OVERFLOW = 0, 1, 2, 3
KEY_LINEAR, KEY_MORTON = 0, 1

# Flags fixed by the oracle's numerics: no FMA contraction, no fast-math.
CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]


def build(src: str = _SRC, out: str = _LIB, extra: tuple = ()) -> str:
    """Compile the oracle into a shared library (always recompiles)."""
    tmp = out + ".tmp"
    subprocess.run(["g++", *CXXFLAGS, *extra, src, "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


_lib = None


def load(path: str | None = None):
    """Load (building first if absent) the oracle library; a path loads another build."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    i64, f32, c_int = ctypes.c_int64, ctypes.c_float, ctypes.c_int
    lib.vgo_grid.argtypes = [P, P, P, i64, f32, c_int, P, P, P, P, P, P]
    lib.vgo_grid.restype = c_int
    lib.vgo_downsample.argtypes = [P, P, P, P, i64, f32, c_int] + [P] * 12
    lib.vgo_downsample.restype = c_int
    lib.vgo_backward.argtypes = [P, P, P, P, i64, P, i64, P, P, P]
    lib.vgo_backward.restype = c_int
    lib.vgo_centroids_fixed.argtypes = [P, P, P, i64, P, i64, P, P, P]
    lib.vgo_centroids_fixed.restype = c_int
    lib.vgo_philox4x64.argtypes = [P, P, P]
    lib.vgo_philox4x64.restype = None
    lib.vgo_nbd.argtypes = [P, P, P, i64, f32, f32, ctypes.c_uint32, ctypes.c_uint64, i64, P, P, P,
                            i64, P]
    lib.vgo_nbd.restype = c_int
    lib.vgo_downsample_filtered.argtypes = [P, P, P, P, i64, f32, c_int, P, P, f32, f32,
                                            ctypes.c_uint32] + [P] * 12
    lib.vgo_downsample_filtered.restype = c_int
    lib.vgo_map_create.argtypes = [f32]
    lib.vgo_map_create.restype = P
    lib.vgo_map_destroy.argtypes = [P]
    lib.vgo_map_destroy.restype = None
    lib.vgo_map_mark.argtypes = [P, P, P, P, i64, ctypes.c_uint32]
    lib.vgo_map_mark.restype = i64
    lib.vgo_map_clear.argtypes = [P, P, P, f32, f32, f32, f32, ctypes.c_int32, ctypes.c_int32, f32, f32]
    lib.vgo_map_clear.restype = i64
    lib.vgo_map_expire.argtypes = [P, ctypes.c_uint32]
    lib.vgo_map_expire.restype = i64
    lib.vgo_map_export.argtypes = [P, P, P, i64]
    lib.vgo_map_export.restype = i64
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def grid(x, y, z, leaf, key_mode=KEY_LINEAR, lib=None):
    """Bounding box, cells per axis, valid count, per-point keys and validity."""
    lib = lib or load()
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.size
    mn = np.zeros(3, np.float32)
    mx = np.zeros(3, np.float32)
    d = np.zeros(3, np.uint32)
    nv = np.zeros(1, np.int64)
    keys = np.zeros(max(n, 1), np.uint64)
    valid = np.zeros(max(n, 1), np.uint8)
    st = lib.vgo_grid(_ptr(x), _ptr(y), _ptr(z), n, np.float32(leaf), key_mode, _ptr(mn), _ptr(mx),
                      _ptr(d), _ptr(nv), _ptr(keys), _ptr(valid))
    if st != OK:
        raise OracleError(st)
    return dict(min=mn, max=mx, dims=d, n_valid=int(nv[0]), keys=keys[:n], valid=valid[:n].astype(bool))


def downsample(x, y, z, rgb, leaf, key_mode=KEY_LINEAR, lib=None):
    """Voxel-grid centroid filter of one cloud; returns a dict of numpy arrays.

    Keys: cx, cy, cz (FP64 centroids), lx, ly, lz (FP64 means of p - p_ref),
    rgb (m x 3 uint8), count (uint32), key (uint64), ref_index (int64),
    point_cell (int32, -1 for invalid points), m.
    """
    lib = lib or load()
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.size
    cap = max(n, 1)
    if rgb is not None:
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8).reshape(-1)
        assert rgb.size == 3 * n
    out = dict(
        cx=np.zeros(cap), cy=np.zeros(cap), cz=np.zeros(cap),
        lx=np.zeros(cap), ly=np.zeros(cap), lz=np.zeros(cap),
        rgb=np.zeros((cap, 3), np.uint8), count=np.zeros(cap, np.uint32),
        key=np.zeros(cap, np.uint64), ref_index=np.zeros(cap, np.int64),
        point_cell=np.zeros(cap, np.int32),
    )
    m = np.zeros(1, np.int64)
    st = lib.vgo_downsample(
        _ptr(x), _ptr(y), _ptr(z), _ptr(rgb), n, np.float32(leaf), key_mode,
        _ptr(out["cx"]), _ptr(out["cy"]), _ptr(out["cz"]), _ptr(out["lx"]), _ptr(out["ly"]),
        _ptr(out["lz"]), _ptr(out["rgb"]), _ptr(out["count"]), _ptr(out["key"]),
        _ptr(out["ref_index"]), _ptr(out["point_cell"]), _ptr(m))
    if st != OK:
        raise OracleError(st)
    mm = int(m[0])
    res = {k: v[:mm] for k, v in out.items() if k != "point_cell"}
    res["point_cell"] = out["point_cell"][:n]
    res["m"] = mm
    return res


def downsample_filtered(x, y, z, rgb, leaf, rot=None, trans=None, z_min=-np.inf, z_max=np.inf,
                        min_points=1, key_mode=KEY_LINEAR, lib=None):
    """The voxel filter after a rigid transform into the global frame (rot:
    3x3 row-major, trans: 3; both or neither), a height limit z_min <= z' <=
    z_max and the removal of cells with fewer than min_points points (see
    vgo.cpp).  Same result layout as downsample."""
    lib = lib or load()
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.size
    cap = max(n, 1)
    if rgb is not None:
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8).reshape(-1)
    R = None if rot is None else np.ascontiguousarray(rot, dtype=np.float32).reshape(9)
    T = None if trans is None else np.ascontiguousarray(trans, dtype=np.float32).reshape(3)
    out = dict(
        cx=np.zeros(cap), cy=np.zeros(cap), cz=np.zeros(cap),
        lx=np.zeros(cap), ly=np.zeros(cap), lz=np.zeros(cap),
        rgb=np.zeros((cap, 3), np.uint8), count=np.zeros(cap, np.uint32),
        key=np.zeros(cap, np.uint64), ref_index=np.zeros(cap, np.int64),
        point_cell=np.zeros(cap, np.int32),
    )
    m = np.zeros(1, np.int64)
    st = lib.vgo_downsample_filtered(
        _ptr(x), _ptr(y), _ptr(z), _ptr(rgb), n, np.float32(leaf), key_mode, _ptr(R), _ptr(T),
        np.float32(z_min), np.float32(z_max), int(min_points),
        _ptr(out["cx"]), _ptr(out["cy"]), _ptr(out["cz"]), _ptr(out["lx"]), _ptr(out["ly"]),
        _ptr(out["lz"]), _ptr(out["rgb"]), _ptr(out["count"]), _ptr(out["key"]),
        _ptr(out["ref_index"]), _ptr(out["point_cell"]), _ptr(m))
    if st != OK:
        raise OracleError(st)
    mm = int(m[0])
    res = {k: v[:mm] for k, v in out.items() if k != "point_cell"}
    res["point_cell"] = out["point_cell"][:n]
    res["m"] = mm
    return res


def downsample_batched(x, y, z, rgb, frame_offsets, leaves, key_mode=KEY_LINEAR, lib=None):
    """Frames of a concatenated cloud, each filtered on its own (own box, own leaf).

    Returns per-frame results (indices frame-local) and a status per frame;
    a frame whose grid overflows yields status ERR_GRID_OVERFLOW and no cells.
    """
    res, status = [], []
    for b in range(len(leaves)):
        s, e = int(frame_offsets[b]), int(frame_offsets[b + 1])
        try:
            r = downsample(x[s:e], y[s:e], z[s:e], None if rgb is None else rgb[s:e], leaves[b],
                           key_mode, lib)
            status.append(OK)
        except OracleError as err:
            if err.status != ERR_GRID_OVERFLOW:
                raise
            r = None
            status.append(err.status)
        res.append(r)
    return res, status


def backward(gx, gy, gz, count, point_cell, lib=None):
    """dL/dp of the centroids for upstream gradient G (FP64), assignment fixed."""
    lib = lib or load()
    gx, gy, gz = (np.ascontiguousarray(g, dtype=np.float64) for g in (gx, gy, gz))
    count = np.ascontiguousarray(count, dtype=np.uint32)
    pc = np.ascontiguousarray(point_cell, dtype=np.int32)
    n, m = pc.size, count.size
    dx, dy, dz = (np.zeros(max(n, 1)) for _ in range(3))
    st = lib.vgo_backward(_ptr(gx), _ptr(gy), _ptr(gz), _ptr(count), m, _ptr(pc), n, _ptr(dx),
                          _ptr(dy), _ptr(dz))
    if st != OK:
        raise OracleError(st)
    return dx[:n], dy[:n], dz[:n]


def centroids_fixed(x, y, z, point_cell, m, lib=None):
    """FP64 centroids of FP64 points under a fixed assignment."""
    lib = lib or load()
    x, y, z = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z))
    pc = np.ascontiguousarray(point_cell, dtype=np.int32)
    cx, cy, cz = (np.zeros(max(m, 1)) for _ in range(3))
    st = lib.vgo_centroids_fixed(_ptr(x), _ptr(y), _ptr(z), pc.size, _ptr(pc), m, _ptr(cx),
                                 _ptr(cy), _ptr(cz))
    if st != OK:
        raise OracleError(st)
    return cx[:m], cy[:m], cz[:m]


def philox4x64(counter, key, lib=None):
    """Philox4x64-10 of one 4-word counter under a 2-word key (4 uint64 words)."""
    lib = lib or load()
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib.vgo_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def nbd_decimate(x, y, z, leaf, radius, umbral, seed, round_size=1000, lib=None):
    """Neighbour-bucket decimation (Alg. 1 of the paper, with the readings in
    vgo.cpp): returns keep (bool [n]), count0 (neighbours before any deletion,
    uint32 [n]), marked (points marked per round), rounds."""
    lib = lib or load()
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.size
    keep = np.zeros(max(n, 1), np.uint8)
    count0 = np.zeros(max(n, 1), np.uint32)
    cap = 1 << 16
    marked = np.zeros(cap, np.int64)
    rounds = np.zeros(1, np.int64)
    st = lib.vgo_nbd(_ptr(x), _ptr(y), _ptr(z), n, np.float32(leaf), np.float32(radius),
                     int(umbral), int(seed), int(round_size), _ptr(keep), _ptr(count0),
                     _ptr(marked), cap, _ptr(rounds))
    if st != OK:
        raise OracleError(st)
    r = int(rounds[0])
    return dict(keep=keep[:n].astype(bool), count0=count0[:n], marked=marked[:min(r, cap)],
                rounds=r)


class VoxelMap:
    """The global voxel map (mark / clear in a camera frustum / expire; see
    vgo.cpp for the readings)."""

    def __init__(self, res, lib=None):
        self.lib = lib or load()
        self.h = self.lib.vgo_map_create(np.float32(res))
        if not self.h:
            raise OracleError(ERR_ARG)

    def mark(self, x, y, z, stamp):
        x, y, z = _f32(x), _f32(y), _f32(z)
        return int(self.lib.vgo_map_mark(self.h, _ptr(x), _ptr(y), _ptr(z), x.size, int(stamp)))

    def clear(self, rot, trans, fx, fy, cx, cy, width, height, z_near, z_far):
        R = np.ascontiguousarray(rot, dtype=np.float32).reshape(9)
        T = np.ascontiguousarray(trans, dtype=np.float32).reshape(3)
        return int(self.lib.vgo_map_clear(self.h, _ptr(R), _ptr(T), np.float32(fx), np.float32(fy),
                                          np.float32(cx), np.float32(cy), int(width), int(height),
                                          np.float32(z_near), np.float32(z_far)))

    def expire(self, min_stamp):
        return int(self.lib.vgo_map_expire(self.h, int(min_stamp)))

    def export(self):
        n = int(self.lib.vgo_map_export(self.h, None, None, 0))
        keys = np.zeros(max(n, 1), np.uint64)
        stamps = np.zeros(max(n, 1), np.uint32)
        self.lib.vgo_map_export(self.h, _ptr(keys), _ptr(stamps), n)
        return keys[:n], stamps[:n]

    def close(self):
        if self.h:
            self.lib.vgo_map_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
