"""vbx: TSDF integration into hashed 16^3-voxel blocks on AMD MI355X.

A thin ctypes binding over the C ABI of libvbx.so (include/vbx.h).  It only marshals
arguments: every step of the integration runs in the library's HIP kernels.  PyTorch
provides device memory and streams; torch is imported first so that the library shares
torch's HIP runtime.

If the library has not been built, or cannot be loaded, every entry point raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np
import torch  # noqa: F401  (shares its HIP runtime with libvbx)

from .build import LIB as _LIB_PATH, build as build_library  # noqa: F401

# ---------------------------------------------------------------------------
# C structures (mirror include/vbx.h)
# ---------------------------------------------------------------------------
W_CONST, W_QUAD = 0, 1
MERGE_NONE, MERGE_GROUPED = 0, 1
F32, F16, S16 = 0, 1, 2
DIST_EQ1, DIST_ALONG_RAY = 0, 1
FLAG_KEEP_TOUCHES = 1
FLAG_FULL_RAY = 2
FLAG_COLOR = 4

STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "block pool full",
          -4: "buffer too small", -5: "device error", -6: "limit exceeded"}
ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_POOL_FULL, ERR_LIMIT = -1, -2, -3, -6


class VbxError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"vbx: {what}: {STATUS.get(status, status)} ({status})")


# Allocator hook of a map's own device memory: alloc(bytes, ctx) -> device pointer or NULL;
# free(ptr, ctx).
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class MapParams(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_float), ("trunc", ctypes.c_float),
                ("w_max", ctypes.c_float), ("max_range", ctypes.c_float),
                ("z_min", ctypes.c_float), ("weighting", ctypes.c_int32),
                ("merge", ctypes.c_int32), ("storage", ctypes.c_int32), ("dist", ctypes.c_int32),
                ("block_capacity", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("stream", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p)]


class EsdfParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_float), ("d_max", ctypes.c_float), ("reserved", ctypes.c_uint32 * 6)]


class EsdfStats(ctypes.Structure):
    _fields_ = [("updates", ctypes.c_uint64), ("dirty_blocks", ctypes.c_uint32),
                ("raise_rounds", ctypes.c_uint32), ("lower_rounds", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("voxels", ctypes.c_uint64)]


class Frame(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_uint64), ("width", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("pose", ctypes.c_float * 12), ("colors", ctypes.c_void_p)]


class HashStats(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint64), ("blocks", ctypes.c_uint64), ("mean_probe", ctypes.c_double),
                ("max_probe", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("points", "valid", "invalid", "out_of_bounds", "rays", "touches", "voxels",
                 "cells", "new_blocks", "blocks", "calls")]


EXPORTED = ["vbx_default_params", "vbx_map_create", "vbx_map_create_ex", "vbx_map_destroy",
            "vbx_map_set_stream", "vbx_integrate", "vbx_integrate_batch", "vbx_integrate_frames",
            "vbx_integrate_frames_noalloc", "vbx_integrate_projective", "vbx_write_blocks", "vbx_esdf_enable", "vbx_esdf_update",
            "vbx_esdf_export", "vbx_export_colors", "vbx_map_hash_stats",
            "vbx_integrate_multi", "vbx_map_sync", "vbx_map_clear_error", "vbx_map_reserve",
            "vbx_map_num_blocks", "vbx_export_blocks", "vbx_import_blocks", "vbx_last_touches",
            "vbx_map_stats", "vbx_map_interpolate", "vbx_debug_traverse", "vbx_debug_traverse_blocks",
            "vbx_status_string",
            "vbx_map_clear",
            "vbx_map_profile", "vbx_map_profile_read", "vbx_map_profile_stages", "vbx_profile_stage_name",
            "vbx_map_get_tuning", "vbx_map_set_tuning", "vbx_map_autotune",
            "vbx_graph_create", "vbx_graph_launch", "vbx_graph_destroy",
            "vbx_server_clock", "vbx_server_create", "vbx_server_add_map", "vbx_server_submit",
            "vbx_server_wait", "vbx_server_drain", "vbx_server_stats", "vbx_server_reset_stats",
            "vbx_server_map", "vbx_server_destroy"]

TUNING_CANDIDATES = 10
# (update_split, update_columns, update_threads) of each candidate, in vbx_map_autotune's order
TUNING_LIST = [(1, 0, 256), (2, 0, 256), (4, 0, 256), (2, 1, 256), (4, 1, 256), (8, 1, 256),
               (1, 0, 1024), (2, 0, 1024), (4, 0, 1024), (2, 0, 512)]


class ServerParams(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_frames_per_tick", ctypes.c_uint32),
                ("max_points_per_tick", ctypes.c_uint64), ("max_inflight", ctypes.c_int32),
                ("grow", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class ServerSummary(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("ticks", ctypes.c_uint64), ("frames", ctypes.c_uint64),
                ("points", ctypes.c_uint64), ("replays", ctypes.c_uint64), ("maps", ctypes.c_uint32),
                ("rejected_maps", ctypes.c_uint32), ("budget_bytes", ctypes.c_uint64),
                ("used_bytes", ctypes.c_uint64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("points_per_s", ctypes.c_double), ("mean_frames_per_tick", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("update_split", ctypes.c_int32), ("update_threads", ctypes.c_int32),
                ("update_columns", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]

PROFILE_STAGES = 10


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * PROFILE_STAGES), ("launches", ctypes.c_uint64 * PROFILE_STAGES)]

_lib = None


def lib(path: Optional[str] = None):
    """Loads libvbx.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"vbx: {p} is not built; run paper_1611_03631_amd.build.build()")
    L = ctypes.CDLL(p)
    vp, sz, i32, u32, f32p = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p
    L.vbx_default_params.argtypes = [ctypes.POINTER(MapParams)]
    L.vbx_default_params.restype = None
    L.vbx_map_create.argtypes = [ctypes.c_float, ctypes.c_float, i32, ctypes.POINTER(vp)]
    L.vbx_map_create_ex.argtypes = [ctypes.POINTER(MapParams), ctypes.POINTER(vp)]
    L.vbx_map_destroy.argtypes = [vp]
    L.vbx_map_destroy.restype = None
    L.vbx_map_set_stream.argtypes = [vp, vp]
    L.vbx_integrate.argtypes = [vp, f32p, sz, f32p]
    L.vbx_integrate_batch.argtypes = [vp, vp, vp, f32p, i32]
    L.vbx_integrate_frames.argtypes = [vp, ctypes.POINTER(Frame), i32]
    L.vbx_integrate_frames_noalloc.argtypes = [vp, ctypes.POINTER(Frame), i32]
    L.vbx_integrate_projective.argtypes = [vp, ctypes.POINTER(Frame), i32, vp]
    L.vbx_map_interpolate.argtypes = [vp, vp, sz, vp]
    L.vbx_integrate_multi.argtypes = [vp, ctypes.POINTER(Frame), i32]
    L.vbx_map_sync.argtypes = [vp]
    L.vbx_map_clear_error.argtypes = [vp]
    L.vbx_map_reserve.argtypes = [vp, u32]
    L.vbx_map_num_blocks.argtypes = [vp, ctypes.POINTER(sz)]
    L.vbx_export_blocks.argtypes = [vp, vp, vp, sz, ctypes.POINTER(sz)]
    L.vbx_import_blocks.argtypes = [vp, vp, vp, sz]
    L.vbx_write_blocks.argtypes = [vp, vp, vp, sz]
    L.vbx_esdf_enable.argtypes = [vp, ctypes.POINTER(EsdfParams)]
    L.vbx_esdf_update.argtypes = [vp, ctypes.POINTER(EsdfStats)]
    L.vbx_esdf_export.argtypes = [vp, vp, vp, vp, sz, ctypes.POINTER(sz)]
    L.vbx_export_colors.argtypes = [vp, vp, vp, sz, ctypes.POINTER(sz)]
    L.vbx_last_touches.argtypes = [vp, vp, vp, sz, ctypes.POINTER(sz)]
    L.vbx_map_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.vbx_map_hash_stats.argtypes = [vp, ctypes.POINTER(HashStats)]
    L.vbx_debug_traverse.argtypes = [vp, vp, i32, vp, i32, vp]
    L.vbx_debug_traverse_blocks.argtypes = [vp, vp, i32, vp, i32, vp]
    L.vbx_status_string.argtypes = [i32]
    L.vbx_status_string.restype = ctypes.c_char_p
    L.vbx_map_clear.argtypes = [vp]
    L.vbx_map_profile.argtypes = [vp, i32]
    L.vbx_map_profile_stages.argtypes = [vp, u32]
    L.vbx_map_profile_read.argtypes = [vp, ctypes.POINTER(Profile), i32]
    L.vbx_map_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.vbx_map_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.vbx_map_autotune.argtypes = [vp, ctypes.POINTER(Frame), i32, ctypes.POINTER(Tuning), vp]
    L.vbx_profile_stage_name.argtypes = [i32]
    L.vbx_profile_stage_name.restype = ctypes.c_char_p
    L.vbx_graph_create.argtypes = [vp, i32, ctypes.POINTER(Frame), vp, i32, ctypes.POINTER(vp)]
    L.vbx_graph_launch.argtypes = [vp, ctypes.POINTER(Frame), i32]
    L.vbx_graph_destroy.argtypes = [vp]
    L.vbx_graph_destroy.restype = None
    L.vbx_server_clock.argtypes = []
    L.vbx_server_clock.restype = ctypes.c_double
    L.vbx_server_create.argtypes = [ctypes.POINTER(ServerParams), ctypes.POINTER(vp)]
    L.vbx_server_add_map.argtypes = [vp, ctypes.POINTER(MapParams), ctypes.POINTER(i32)]
    L.vbx_server_submit.argtypes = [vp, i32, ctypes.POINTER(Frame), ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_uint64)]
    L.vbx_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.vbx_server_drain.argtypes = [vp]
    L.vbx_server_stats.argtypes = [vp, ctypes.POINTER(ServerSummary)]
    L.vbx_server_reset_stats.argtypes = [vp]
    L.vbx_server_map.argtypes = [vp, i32]
    L.vbx_server_map.restype = vp
    L.vbx_server_destroy.argtypes = [vp]
    L.vbx_server_destroy.restype = None
    for name in EXPORTED:
        if name not in ("vbx_default_params", "vbx_map_destroy", "vbx_status_string",
                        "vbx_profile_stage_name", "vbx_graph_destroy", "vbx_server_clock",
                        "vbx_server_map", "vbx_server_destroy"):
            getattr(L, name).restype = ctypes.c_int
    if path is None:
        _lib = L
    return L


def _check(status: int, what: str):
    if status != 0:
        raise VbxError(status, what)


def _dev_points(points) -> Tuple[int, int]:
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a device (cuda) torch tensor of shape [N, 3]")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
        raise TypeError("points must be float32 [N, 3]")
    if not points.is_contiguous():
        raise TypeError("points must be contiguous")
    return points.data_ptr(), int(points.shape[0])


def _pose12(pose) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(pose, dtype=np.float32).reshape(12))
    return p


_WEIGHTING = {"const": W_CONST, "quad": W_QUAD}
_MERGE = {"simple": MERGE_NONE, "none": MERGE_NONE, "grouped": MERGE_GROUPED}
_STORAGE = {"f32": F32, "f16": F16, "s16": S16}
_DIST = {"eq1": DIST_EQ1, "ray": DIST_ALONG_RAY}


def map_params(voxel_size: float, trunc: float, weighting: str = "const", merge: str = "simple",
               storage: str = "f32", w_max: float = 1e4, max_range: float = 5.0, z_min: float = 0.1,
               dist: str = "eq1", block_capacity: int = 65536, keep_touches: bool = False,
               stream_handle: int = 0, full_ray: bool = False, color: bool = False) -> MapParams:
    p = MapParams()
    lib().vbx_default_params(ctypes.byref(p))
    p.voxel_size, p.trunc, p.w_max = voxel_size, trunc, w_max
    p.max_range, p.z_min = max_range, z_min
    p.weighting, p.merge = _WEIGHTING[weighting], _MERGE[merge]
    p.storage, p.dist = _STORAGE[storage], _DIST[dist]
    p.block_capacity = block_capacity
    p.flags = ((FLAG_KEEP_TOUCHES if keep_touches else 0) | (FLAG_FULL_RAY if full_ray else 0) |
               (FLAG_COLOR if color else 0))
    p.stream = stream_handle
    return p


class Map:
    """A TSDF map on the current HIP device (wraps vbx_map)."""

    def __init__(self, voxel_size: float, trunc: float, weighting: str = "const",
                 merge: str = "simple", storage: str = "f32", w_max: float = 1e4,
                 max_range: float = 5.0, z_min: float = 0.1, dist: str = "eq1",
                 block_capacity: int = 65536, keep_touches: bool = False, stream=None,
                 allocator=None, full_ray: bool = False, color: bool = False):
        """allocator: optional (alloc, free) pair of callables, alloc(nbytes) -> device address
        (0 when it cannot) and free(address), used for the map's hash table, block pool and
        device state instead of hipMalloc / hipFree.  color: the map keeps a colour per voxel
        and raycasting frames carry one per point (the fourth element of a frame tuple)."""
        L = lib()
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        p = map_params(voxel_size, trunc, weighting, merge, storage, w_max, max_range, z_min, dist,
                       block_capacity, keep_touches, s.cuda_stream, full_ray, color)
        self._hooks = None
        if allocator is not None:
            a_py, f_py = allocator
            # the ctypes thunks must outlive the map: kept on the object
            self._hooks = (ALLOC_FN(lambda nbytes, ctx: a_py(int(nbytes)) or None),
                           FREE_FN(lambda ptr, ctx: f_py(int(ptr)) if ptr else None))
            p.alloc, p.free = self._hooks
        h = ctypes.c_void_p()
        _check(L.vbx_map_create_ex(ctypes.byref(p), ctypes.byref(h)), "vbx_map_create_ex")
        self._h = h
        self._owned = True
        self.params = dict(voxel_size=voxel_size, trunc=trunc, weighting=weighting, merge=merge,
                           storage=storage, w_max=w_max, max_range=max_range, z_min=z_min,
                           dist=dist, block_capacity=block_capacity, full_ray=full_ray, color=color)

    @classmethod
    def _borrowed(cls, handle, params: dict, owner):
        """A view of a map another object owns (a server's)."""
        m = cls.__new__(cls)
        m._h = ctypes.c_void_p(handle)
        m._owned = False
        m._owner = owner
        m.params = dict(params)
        m.stream = None
        return m

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                lib().vbx_map_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- integration -------------------------------------------------------
    def integrate(self, points, pose):
        ptr, n = _dev_points(points)
        pz = _pose12(pose)
        _check(lib().vbx_integrate(self._h, ptr, n, pz.ctypes.data), "vbx_integrate")

    def interpolate(self, points):
        """Distances at device points float32 [N, 3] by trilinear interpolation (device float32
        [N], NaN where unknown); stream-ordered on the map's stream."""
        ptr, n = _dev_points(points)
        out = torch.empty(n, dtype=torch.float32, device=points.device)
        _check(lib().vbx_map_interpolate(self._h, ptr, n, out.data_ptr() if n else None),
               "vbx_map_interpolate")
        return out

    def integrate_frames(self, frames: Sequence[Tuple]):
        """frames: sequence of (points tensor [N,3], pose [3,4]), (points, pose, width) or
        (points, pose, width, colors) with colors a device int32 / uint32 tensor [N] of RGBA8
        (red in the low byte)."""
        arr = make_frames(frames)
        _check(lib().vbx_integrate_frames(self._h, arr, len(frames)), "vbx_integrate_frames")

    def integrate_frames_noalloc(self, frames: Sequence[Tuple]):
        """As integrate_frames, with the call's scratch memory taken from the library's fixed
        per-device region (no device allocation; calls overlapping on one device race)."""
        arr = make_frames(frames)
        _check(lib().vbx_integrate_frames_noalloc(self._h, arr, len(frames)),
               "vbx_integrate_frames_noalloc")

    def integrate_projective(self, frames: Sequence[Tuple], intrinsics):
        """Projection mapping (Sec. IV-B) of organised frames [(points, pose, width)] with pinhole
        intrinsics (fx, fy, cx, cy)."""
        arr = make_frames(frames)
        K = np.ascontiguousarray(np.asarray(intrinsics, dtype=np.float32).reshape(4))
        _check(lib().vbx_integrate_projective(self._h, arr, len(frames), K.ctypes.data),
               "vbx_integrate_projective")

    def integrate_batch(self, points_list, poses):
        F = len(points_list)
        ptrs = (ctypes.c_void_p * F)()
        ns = (ctypes.c_size_t * F)()
        for i, pts in enumerate(points_list):
            ptrs[i], ns[i] = _dev_points(pts)
        P = np.ascontiguousarray(np.asarray(poses, dtype=np.float32).reshape(F, 12))
        _check(lib().vbx_integrate_batch(self._h, ptrs, ns, P.ctypes.data, F), "vbx_integrate_batch")

    # -- state ---------------------------------------------------------------
    def sync(self) -> int:
        """Waits for the map's stream; returns the sticky device status (0 = ok)."""
        return int(lib().vbx_map_sync(self._h))

    def clear_error(self):
        _check(lib().vbx_map_clear_error(self._h), "vbx_map_clear_error")

    def reserve(self, block_capacity: int):
        _check(lib().vbx_map_reserve(self._h, block_capacity), "vbx_map_reserve")

    def num_blocks(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().vbx_map_num_blocks(self._h, ctypes.byref(n)), "vbx_map_num_blocks")
        return int(n.value)

    def export(self):
        """(coords int32 [B,3] ascending, dw float32 [B,4096,2] with D in metres and W)."""
        L = lib()
        n = ctypes.c_size_t()
        _check(L.vbx_export_blocks(self._h, None, None, 0, ctypes.byref(n)), "vbx_export_blocks")
        B = int(n.value)
        coords = np.zeros((B, 3), np.int32)
        dw = np.zeros((B, 4096, 2), np.float32)
        _check(L.vbx_export_blocks(self._h, coords.ctypes.data, dw.ctypes.data, B, ctypes.byref(n)),
               "vbx_export_blocks")
        return coords, dw

    def export_colors(self):
        """(coords int32 [B,3] ascending, packed RGB8 uint32 [B,4096]) of a colour map."""
        L = lib()
        n = ctypes.c_size_t()
        _check(L.vbx_export_colors(self._h, None, None, 0, ctypes.byref(n)), "vbx_export_colors")
        B = int(n.value)
        coords = np.zeros((B, 3), np.int32)
        rgb = np.zeros((B, 4096), np.uint32)
        _check(L.vbx_export_colors(self._h, coords.ctypes.data, rgb.ctypes.data, B, ctypes.byref(n)),
               "vbx_export_colors")
        return coords, rgb

    def write_blocks(self, coords: np.ndarray, dw: np.ndarray):
        """Writes TSDF blocks (coords [B,3], dw [B,4096,2], D in metres) in place, allocating the
        missing ones; they count as changed for the next ESDF update."""
        c = np.ascontiguousarray(coords, np.int32).reshape(-1, 3)
        d = np.ascontiguousarray(dw, np.float32).reshape(-1, 4096, 2)
        _check(lib().vbx_write_blocks(self._h, c.ctypes.data, d.ctypes.data, c.shape[0]),
               "vbx_write_blocks")

    # -- ESDF layer (Sec. V-A) ------------------------------------------------
    def esdf_enable(self, gamma: float, d_max: float):
        p = EsdfParams()
        p.gamma, p.d_max = gamma, d_max
        _check(lib().vbx_esdf_enable(self._h, ctypes.byref(p)), "vbx_esdf_enable")

    def esdf_update(self) -> dict:
        st = EsdfStats()
        _check(lib().vbx_esdf_update(self._h, ctypes.byref(st)), "vbx_esdf_update")
        return {n: int(getattr(st, n)) for n, _ in EsdfStats._fields_ if n != "reserved"}

    def esdf_export(self):
        """(coords int32 [B,3] ascending, d float32 [B,4096] signed metres, info uint8 [B,4096]:
        bit 0 observed, bit 1 fixed, bits 2..6 parent neighbour index, bit 7 negative side)."""
        L = lib()
        n = ctypes.c_size_t()
        _check(L.vbx_esdf_export(self._h, None, None, None, 0, ctypes.byref(n)), "vbx_esdf_export")
        B = int(n.value)
        coords = np.zeros((B, 3), np.int32)
        d = np.zeros((B, 4096), np.float32)
        info = np.zeros((B, 4096), np.uint8)
        _check(L.vbx_esdf_export(self._h, coords.ctypes.data, d.ctypes.data, info.ctypes.data, B,
                                 ctypes.byref(n)), "vbx_esdf_export")
        return coords, d, info

    def import_blocks(self, coords: np.ndarray, dw: np.ndarray):
        c = np.ascontiguousarray(coords, np.int32).reshape(-1, 3)
        d = np.ascontiguousarray(dw, np.float32).reshape(-1, 4096, 2)
        _check(lib().vbx_import_blocks(self._h, c.ctypes.data, d.ctypes.data, c.shape[0]),
               "vbx_import_blocks")

    def last_touches(self):
        """Voxels touched by the last call: (coords int32 [T,3], counts uint32 [T]), unordered."""
        L = lib()
        n = ctypes.c_size_t()
        _check(L.vbx_last_touches(self._h, None, None, 0, ctypes.byref(n)), "vbx_last_touches")
        T = int(n.value)
        coords = np.zeros((T, 3), np.int32)
        counts = np.zeros(T, np.uint32)
        _check(L.vbx_last_touches(self._h, coords.ctypes.data, counts.ctypes.data, T,
                                  ctypes.byref(n)), "vbx_last_touches")
        return coords, counts

    def clear(self):
        """Removes every block (stream-ordered)."""
        _check(lib().vbx_map_clear(self._h), "vbx_map_clear")

    def profile(self, enable: bool = True, stages=None):
        """Per-stage event timing of this map's calls: every stage, none, or only the named
        stages (each timed stage costs its calls two event records)."""
        L = lib()
        if stages is None:
            _check(L.vbx_map_profile(self._h, 1 if enable else 0), "vbx_map_profile")
            return
        names = [L.vbx_profile_stage_name(i).decode() for i in range(PROFILE_STAGES)]
        mask = 0
        for st in stages:
            mask |= 1 << names.index(st)
        _check(L.vbx_map_profile_stages(self._h, mask if enable else 0), "vbx_map_profile_stages")

    def profile_read(self, reset: bool = True) -> dict:
        """{stage: (milliseconds, launches)} summed since the last reset (synchronises)."""
        L = lib()
        p = Profile()
        _check(L.vbx_map_profile_read(self._h, ctypes.byref(p), 1 if reset else 0),
               "vbx_map_profile_read")
        return {L.vbx_profile_stage_name(i).decode(): (p.ms[i], int(p.launches[i]))
                for i in range(PROFILE_STAGES)}

    def tuning(self) -> dict:
        t = Tuning()
        _check(lib().vbx_map_get_tuning(self._h, ctypes.byref(t)), "vbx_map_get_tuning")
        return {"update_split": int(t.update_split), "update_threads": int(t.update_threads),
                "update_columns": int(t.update_columns)}

    def set_tuning(self, update_split: int, update_threads: int = 256, update_columns: int = 0):
        t = Tuning()
        t.update_split = update_split
        t.update_threads = update_threads
        t.update_columns = update_columns
        _check(lib().vbx_map_set_tuning(self._h, ctypes.byref(t)), "vbx_map_set_tuning")

    def autotune(self, frames) -> dict:
        """Times every candidate tuning on a scratch map and keeps the fastest.
        Returns {"best": tuning dict, "ms": [per-candidate ms]}."""
        arr = make_frames(frames)
        best = Tuning()
        ms = (ctypes.c_double * TUNING_CANDIDATES)()
        _check(lib().vbx_map_autotune(self._h, arr, len(frames), ctypes.byref(best), ms),
               "vbx_map_autotune")
        return {"best": {"update_split": int(best.update_split), "update_threads": int(best.update_threads),
                         "update_columns": int(best.update_columns)}, "ms": list(ms)}

    def hash_stats(self) -> dict:
        """Block-hash occupancy: slots, blocks, mean and maximum lookup probe length."""
        h = HashStats()
        _check(lib().vbx_map_hash_stats(self._h, ctypes.byref(h)), "vbx_map_hash_stats")
        return {"slots": int(h.slots), "blocks": int(h.blocks), "mean_probe": float(h.mean_probe),
                "max_probe": int(h.max_probe)}

    def stats(self) -> dict:
        s = Stats()
        _check(lib().vbx_map_stats(self._h, ctypes.byref(s)), "vbx_map_stats")
        return {n: int(getattr(s, n)) for n, _ in Stats._fields_}


def make_frames(frames) -> ctypes.Array:
    arr = (Frame * len(frames))()
    for i, f in enumerate(frames):
        pts, pose = f[0], f[1]
        width = int(f[2]) if len(f) > 2 and f[2] is not None else 0
        ptr, n = _dev_points(pts)
        arr[i].points = ptr
        arr[i].n = n
        arr[i].width = width
        if len(f) > 3 and f[3] is not None:
            col = f[3]
            if not (col.is_cuda and col.is_contiguous() and col.element_size() == 4 and col.numel() == n):
                raise ValueError("colors: a contiguous device tensor of 4-byte words, one per point")
            arr[i].colors = col.data_ptr() if n else None
        pz = _pose12(pose)
        for k in range(12):
            arr[i].pose[k] = float(pz[k])
    return arr


def integrate_multi(maps: Sequence[Map], frames: Sequence[Tuple]):
    """frames[i] (points, pose[, width]) into maps[i], one pass on maps[0]'s stream."""
    M = len(maps)
    hs = (ctypes.c_void_p * M)(*[m.handle for m in maps])
    arr = make_frames(frames)
    _check(lib().vbx_integrate_multi(hs, arr, M), "vbx_integrate_multi")


class Graph:
    """One integration call captured into a HIP graph (frames[i] into maps[owner[i]]),
    replayed by `launch`; frames keep their point count and width, pointers and poses may
    change."""

    def __init__(self, maps: Sequence[Map], frames: Sequence[Tuple], owner=None):
        self._maps = list(maps)          # keeps the maps alive while the graph is
        M = len(self._maps)
        hs = (ctypes.c_void_p * M)(*[m.handle for m in self._maps])
        arr = make_frames(frames)
        self._F = len(frames)
        own = None
        if owner is not None:
            own = (ctypes.c_int32 * self._F)(*[int(x) for x in owner])
        h = ctypes.c_void_p()
        _check(lib().vbx_graph_create(hs, M, arr, own, self._F, ctypes.byref(h)), "vbx_graph_create")
        self._h = h
        self._keep = frames

    def launch(self, frames: Optional[Sequence[Tuple]] = None):
        if frames is None:
            _check(lib().vbx_graph_launch(self._h, None, 0), "vbx_graph_launch")
        else:
            arr = make_frames(frames)
            _check(lib().vbx_graph_launch(self._h, arr, len(frames)), "vbx_graph_launch")
            self._keep = frames

    def close(self):
        if self._h:
            lib().vbx_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching map server (wraps vbx_server): frames are submitted one request at
    a time and batched into ticks on the device as they arrive."""

    def __init__(self, budget_bytes: int, max_frames_per_tick: int = 0, max_points_per_tick: int = 0,
                 max_inflight: int = 0, grow: bool = True, stream=None):
        p = ServerParams()
        p.budget_bytes = int(budget_bytes)
        p.max_frames_per_tick = max_frames_per_tick
        p.max_points_per_tick = max_points_per_tick
        p.max_inflight = max_inflight
        p.grow = 1 if grow else 0
        p.stream = stream.cuda_stream if stream is not None else None
        h = ctypes.c_void_p()
        _check(lib().vbx_server_create(ctypes.byref(p), ctypes.byref(h)), "vbx_server_create")
        self._h = h
        self._params = {}
        self._keep = {}        # points of requests not known to be finished
        self._frame = Frame()

    @staticmethod
    def clock() -> float:
        return float(lib().vbx_server_clock())

    def add_map(self, **kw) -> int:
        """Admits a map (keyword arguments as for Map); raises VbxError(OUT_OF_MEMORY) when
        the budget cannot hold it."""
        p = map_params(**kw)
        mid = ctypes.c_int32()
        _check(lib().vbx_server_add_map(self._h, ctypes.byref(p), ctypes.byref(mid)), "vbx_server_add_map")
        self._params[int(mid.value)] = kw
        return int(mid.value)

    def submit(self, map_id: int, points, pose, width: int = 0, t_arrival: float = 0.0) -> int:
        f = self._frame
        ptr, n = _dev_points(points)
        f.points, f.n, f.width = ptr, n, width
        pz = _pose12(pose)
        for k in range(12):
            f.pose[k] = float(pz[k])
        t = ctypes.c_uint64()
        _check(lib().vbx_server_submit(self._h, map_id, ctypes.byref(f), float(t_arrival), ctypes.byref(t)),
               "vbx_server_submit")
        self._keep[int(t.value)] = points
        return int(t.value)

    def wait(self, ticket: int):
        """(status, completion time) of a request; blocks until it completes."""
        st = ctypes.c_int32()
        td = ctypes.c_double()
        _check(lib().vbx_server_wait(self._h, ticket, ctypes.byref(st), ctypes.byref(td)), "vbx_server_wait")
        self._keep.pop(ticket, None)
        return int(st.value), float(td.value)

    def drain(self):
        _check(lib().vbx_server_drain(self._h), "vbx_server_drain")
        self._keep.clear()

    def stats(self) -> dict:
        s = ServerSummary()
        _check(lib().vbx_server_stats(self._h, ctypes.byref(s)), "vbx_server_stats")
        return {name: getattr(s, name) for name, _ in ServerSummary._fields_}

    def reset_stats(self):
        _check(lib().vbx_server_reset_stats(self._h), "vbx_server_reset_stats")
        self._keep.clear()

    def map(self, map_id: int) -> Map:
        h = lib().vbx_server_map(self._h, map_id)
        if not h:
            raise VbxError(ERR_INVALID_ARG, "vbx_server_map")
        return Map._borrowed(h, self._params.get(map_id, {}), self)

    def close(self):
        if getattr(self, "_h", None):
            lib().vbx_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_traverse(A: torch.Tensor, B: torch.Tensor, cap: int = 128):
    """Voxels visited from A[i] to B[i] (voxel units, device float32 [n,3])."""
    n = A.shape[0]
    out = torch.zeros((n, cap, 3), dtype=torch.int32, device=A.device)
    counts = torch.zeros(n, dtype=torch.int32, device=A.device)
    _check(lib().vbx_debug_traverse(A.data_ptr(), B.data_ptr(), n, out.data_ptr(), cap,
                                    counts.data_ptr()), "vbx_debug_traverse")
    return out, counts


def debug_traverse_blocks(A: torch.Tensor, B: torch.Tensor, cap: int = 128):
    """Blocks (voxel index >> 4) passed through from A[i] to B[i] (voxel units, device float32
    [n,3]), found as the integration finds them."""
    n = A.shape[0]
    out = torch.zeros((n, cap, 3), dtype=torch.int32, device=A.device)
    counts = torch.zeros(n, dtype=torch.int32, device=A.device)
    _check(lib().vbx_debug_traverse_blocks(A.data_ptr(), B.data_ptr(), n, out.data_ptr(), cap,
                                           counts.data_ptr()), "vbx_debug_traverse_blocks")
    return out, counts
