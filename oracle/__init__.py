"""CPU oracle for TSDF integration (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it: the GPU path and the
oracle share no code.

The oracle itself is plain C (``vbx_oracle.c``), compiled with gcc by
:func:`build` and loaded here with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vbx_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")

CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-mfpmath=sse", "-msse2", "-Wall", "-Wno-unused-function"]


def build(extra_flags=(), out: Optional[str] = None) -> str:
    """Compile the oracle with gcc; returns the path of the shared library."""
    out = out or _LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", *CFLAGS, *extra_flags, _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Params(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_float), ("trunc", ctypes.c_float),
                ("w_max", ctypes.c_float), ("max_range", ctypes.c_float),
                ("z_min", ctypes.c_float), ("weighting", ctypes.c_int),
                ("merge", ctypes.c_int), ("fp16", ctypes.c_int), ("dist", ctypes.c_int),
                ("world64", ctypes.c_int), ("full_ray", ctypes.c_int), ("color", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("points", "valid", "invalid", "out_of_bounds", "rays", "touches", "voxels",
                 "new_blocks")]


_libs = {}


def load(path: Optional[str] = None):
    path = path or _LIB
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        if path != _LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [P(_Params)]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_integrate.restype = ctypes.c_int
    lib.orc_integrate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p, P(_Stats)]
    lib.orc_num_blocks.restype = ctypes.c_size_t
    lib.orc_num_blocks.argtypes = [ctypes.c_void_p]
    lib.orc_integrate_color.restype = ctypes.c_int
    lib.orc_integrate_color.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, P(_Stats)]
    lib.orc_export_color.restype = ctypes.c_size_t
    lib.orc_export_color.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    lib.orc_integrate_projective.restype = ctypes.c_int
    lib.orc_integrate_projective.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                             ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                             P(_Stats)]
    lib.orc_export.restype = ctypes.c_size_t
    lib.orc_export.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [ctypes.c_size_t]
    lib.orc_export_ramp.restype = ctypes.c_size_t
    lib.orc_export_ramp.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    lib.orc_last_touches.restype = ctypes.c_size_t
    lib.orc_last_touches.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_size_t]
    lib.orc_dda.restype = ctypes.c_int
    lib.orc_dda.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.orc_group_mean.restype = None
    lib.orc_group_mean.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_float, ctypes.c_int, ctypes.c_void_p]
    lib.orc_round_half.restype = ctypes.c_double
    lib.orc_round_half.argtypes = [ctypes.c_double]
    lib.orc_round_s16.restype = ctypes.c_double
    lib.orc_round_s16.argtypes = [ctypes.c_double]
    _libs[path] = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


WEIGHTING = {"const": 0, "quad": 1}
MERGE = {"simple": 0, "grouped": 1}
DIST = {"eq1": 0, "ray": 1}
# value storage emulated after every frame: none (binary64), binary16 D/delta and W, or D/delta
# to the nearest multiple of 1/32767 with binary16 W
STORAGE = {"f32": 0, "f16": 1, "s16": 2}


def weight_bits(weighting: str, z_min: float) -> int:
    """Fractional bits of the fixed-point point weights in the grouped mean (0: weights are 1)."""
    if weighting == "const":
        return 0
    zf = np.float32(z_min)
    wmax = np.float32(1.0) / (zf * zf)
    c = 0
    while np.float32(2.0 ** c) < wmax:
        c += 1
    return 32 - c


class OracleMap:
    """One TSDF map integrated frame by frame on the CPU."""

    def __init__(self, voxel_size: float, trunc: float, weighting: str = "const",
                 merge: str = "simple", w_max: float = 1e4, max_range: float = 5.0,
                 z_min: float = 0.1, storage: str = "f32", dist: str = "eq1",
                 world64: bool = False, full_ray: bool = False, color: bool = False,
                 lib_path: Optional[str] = None):
        """world64: measure distances from the binary64 transform of each sensor point (and a
        group's exact binary64 mean) instead of the binary32 ray end point."""
        self.lib = load(lib_path)
        self.params = dict(voxel_size=voxel_size, trunc=trunc, weighting=weighting,
                           merge=merge, w_max=w_max, max_range=max_range, z_min=z_min,
                           storage=storage, dist=dist, world64=world64, full_ray=full_ray, color=color)
        p = _Params(voxel_size, trunc, w_max, max_range, z_min, WEIGHTING[weighting],
                    MERGE[merge], STORAGE[storage], DIST[dist], 1 if world64 else 0,
                    1 if full_ray else 0, 1 if color else 0)
        self._h = self.lib.orc_create(ctypes.byref(p))

    def close(self):
        if self._h:
            self.lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def integrate(self, points: np.ndarray, pose: np.ndarray, colors: Optional[np.ndarray] = None) -> dict:
        """colors: uint32 [n] RGBA8 (red in the low byte) for a colour map."""
        pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
        ps = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
        st = _Stats()
        if colors is not None:
            col = np.ascontiguousarray(colors, dtype=np.uint32).reshape(-1)
            assert col.shape[0] == pts.shape[0]
            self.lib.orc_integrate_color(self._h, _ptr(pts), _ptr(col), pts.shape[0], _ptr(ps), ctypes.byref(st))
        else:
            self.lib.orc_integrate(self._h, _ptr(pts), pts.shape[0], _ptr(ps), ctypes.byref(st))
        return {n: int(getattr(st, n)) for n, _ in _Stats._fields_}

    def integrate_projective(self, points: np.ndarray, pose: np.ndarray, width: int,
                             intrinsics) -> dict:
        """Projection mapping of one organised frame (Sec. IV-B): points [H*W, 3] in the sensor
        frame, intrinsics (fx, fy, cx, cy) mapping camera points to pixel coordinates."""
        pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
        ps = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
        intr = np.ascontiguousarray(intrinsics, dtype=np.float32).reshape(4)
        st = _Stats()
        rc = self.lib.orc_integrate_projective(self._h, _ptr(pts), pts.shape[0], int(width), _ptr(ps),
                                               _ptr(intr), ctypes.byref(st))
        if rc != 0:
            raise ValueError("projection mapping needs an organised frame (n a multiple of width)")
        return {n: int(getattr(st, n)) for n, _ in _Stats._fields_}

    def num_blocks(self) -> int:
        return int(self.lib.orc_num_blocks(self._h))

    def export(self, with_mass: bool = True):
        """(coords int32 [B,3] ascending, D f64 [B,4096] metres, W f64 [B,4096], mass f64 [B,4096],
        ramp f64 [B,4096]).  mass: the summed weight of every ray that saw the voxel; ramp: that of
        the rays that saw it on the Eq. (5) drop-off ramp (comparison diagnostics)."""
        nb = self.num_blocks()
        coords = np.zeros((nb, 3), np.int32)
        D = np.zeros((nb, 4096), np.float64)
        W = np.zeros((nb, 4096), np.float64)
        M = np.zeros((nb, 4096), np.float64) if with_mass else None
        R = np.zeros((nb, 4096), np.float64) if with_mass else None
        self.lib.orc_export(self._h, _ptr(coords), _ptr(D), _ptr(W),
                            _ptr(M) if with_mass else None, nb)
        if with_mass:
            self.lib.orc_export_ramp(self._h, _ptr(R), nb)
        return coords, D, W, M, R

    def export_colors(self) -> np.ndarray:
        """Packed RGB8 colours [B, 4096] (red in the low byte), in export()'s block order."""
        nb = self.num_blocks()
        rgb = np.zeros((nb, 4096), np.uint32)
        self.lib.orc_export_color(self._h, _ptr(rgb), nb)
        return rgb

    def last_touches(self):
        """Voxels touched by the last frame: (coords int32 [T,3], ray counts uint32 [T])."""
        n = int(self.lib.orc_last_touches(self._h, None, None, 0))
        coords = np.zeros((n, 3), np.int32)
        counts = np.zeros(n, np.uint32)
        self.lib.orc_last_touches(self._h, _ptr(coords), _ptr(counts), n)
        return coords, counts


def dda(A, B, lib_path: Optional[str] = None) -> np.ndarray:
    """Voxels visited between voxel-space points A and B (float32), in visiting order."""
    lib = load(lib_path)
    a = np.ascontiguousarray(A, np.float32).reshape(3)
    b = np.ascontiguousarray(B, np.float32).reshape(3)
    n = lib.orc_dda(_ptr(a), _ptr(b), None, 0)
    out = np.zeros((n, 3), np.int32)
    lib.orc_dda(_ptr(a), _ptr(b), _ptr(out), n)
    return out


def group_mean(p32, w32, voxel_size: float, wbits: int, lib_path: Optional[str] = None):
    """Binary32 ray end point of a group of points (grouped raycasting)."""
    lib = load(lib_path)
    p = np.ascontiguousarray(p32, np.float32).reshape(-1, 3)
    w = np.ascontiguousarray(w32, np.float32).reshape(-1)
    out = np.zeros(3, np.float32)
    lib.orc_group_mean(_ptr(p), _ptr(w), p.shape[0], voxel_size, wbits, _ptr(out))
    return out


def round_half(x: float, lib_path: Optional[str] = None) -> float:
    return float(load(lib_path).orc_round_half(float(x)))


def round_s16(x: float, lib_path: Optional[str] = None) -> float:
    return float(load(lib_path).orc_round_s16(float(x)))
