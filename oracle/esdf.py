"""CPU oracle for the ESDF built from a TSDF (test infrastructure).

Only the test-suite and the benchmark's CPU-baseline leg may import this module; the
product library never loads it.  The oracle is plain C (``esdf_oracle.c``, Algorithm 1 of
Sec. V-A with FIFO or bucketed priority queues, binary64), compiled with gcc by
:func:`build` and loaded with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esdf_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle_esdf.so")
CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall"]

# neighbour index n = (dx + 1) + 3 (dy + 1) + 9 (dz + 1); 13 is the voxel itself ("no parent")
OFFSETS = np.array([[n % 3 - 1, (n // 3) % 3 - 1, n // 9 - 1] for n in range(27)], np.int32)
NO_PARENT = 13

_libs = {}


def build(extra_flags=(), out: Optional[str] = None, src: Optional[str] = None) -> str:
    out = out or _LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    subprocess.run(["gcc", *CFLAGS, *extra_flags, src or _SRC, "-o", out, "-lm"], check=True)
    return out


def load(path: Optional[str] = None):
    path = path or _LIB
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        if path != _LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.orc_esdf_create.restype = vp
    lib.orc_esdf_create.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.orc_esdf_destroy.argtypes = [vp]
    lib.orc_esdf_update.argtypes = [vp, sz, vp, vp, vp]
    lib.orc_esdf_export.restype = sz
    lib.orc_esdf_export.argtypes = [vp, vp, vp, vp, sz]
    lib.orc_esdf_counts.argtypes = [vp, vp]
    _libs[path] = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleESDF:
    """The ESDF of one TSDF map, updated call by call on the CPU."""

    def __init__(self, voxel_size: float, gamma: float, d_max: float, queue: str = "fifo",
                 lib_path: Optional[str] = None):
        self.lib = load(lib_path)
        self.voxel_size, self.gamma, self.d_max = float(voxel_size), float(gamma), float(d_max)
        self._h = self.lib.orc_esdf_create(self.voxel_size, self.gamma, self.d_max,
                                           1 if queue == "priority" else 0)

    def close(self):
        if self._h:
            self.lib.orc_esdf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, coords, d, w):
        """coords int [n,3] voxel indices of changed TSDF voxels, d their distance (metres), w
        their weight (0: unknown)."""
        c = np.ascontiguousarray(coords, np.int32).reshape(-1, 3)
        dd = np.ascontiguousarray(d, np.float64).reshape(-1)
        ww = np.ascontiguousarray(w, np.float64).reshape(-1)
        self.lib.orc_esdf_update(self._h, c.shape[0], _ptr(c), _ptr(dd), _ptr(ww))

    def update_from_blocks(self, coords, D, W):
        """Every voxel of the given TSDF blocks (coords [B,3], D and W [B,4096], x fastest) as
        changed voxels."""
        c = voxel_coords(coords)
        self.update(c, np.asarray(D, np.float64).reshape(-1), np.asarray(W, np.float64).reshape(-1))

    def export(self):
        """(coords int32 [n,3], d f64 [n], info uint8 [n]) of the observed voxels, sorted by
        (x, y, z); info bit 0 observed, bit 1 fixed, bits 2..6 parent neighbour index, bit 7
        negative side."""
        n = int(self.lib.orc_esdf_export(self._h, None, None, None, 0))
        c = np.zeros((n, 3), np.int32)
        d = np.zeros(n, np.float64)
        info = np.zeros(n, np.uint8)
        self.lib.orc_esdf_export(self._h, _ptr(c), _ptr(d), _ptr(info), n)
        order = np.lexsort((c[:, 2], c[:, 1], c[:, 0]))
        return c[order], d[order], info[order]

    def counts(self):
        out = np.zeros(3, np.uint64)
        self.lib.orc_esdf_counts(self._h, _ptr(out))
        return {"raise_pops": int(out[0]), "lower_pops": int(out[1]), "updates": int(out[2])}


def voxel_coords(block_coords) -> np.ndarray:
    """Voxel indices [B*4096, 3] of blocks [B,3] (16^3 voxels each, x fastest)."""
    b = np.asarray(block_coords, np.int64).reshape(-1, 1, 3)
    l = np.arange(4096)
    loc = np.stack([l & 15, (l >> 4) & 15, l >> 8], axis=1)[None, :, :]
    return (16 * b + loc).reshape(-1, 3).astype(np.int32)


def chamfer(offsets, v: float) -> np.ndarray:
    """Quasi-Euclidean (26-neighbour) path length of integer offsets [n,3]: with the absolute
    components sorted a >= b >= c, sqrt(3) c + sqrt(2) (b - c) + (a - b), times v."""
    a = np.sort(np.abs(np.asarray(offsets, np.int64)), axis=1)[:, ::-1].astype(np.float64)
    return v * (np.sqrt(3.0) * a[:, 2] + np.sqrt(2.0) * (a[:, 1] - a[:, 2]) + (a[:, 0] - a[:, 1]))
