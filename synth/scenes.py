"""Seeded synthetic depth and LiDAR workloads.

This module only builds inputs: analytic scenes (axis-aligned boxes, spheres,
vertical cylinders, planes), sensor poses and noisy point clouds in the sensor
frame.  It holds none of the integration arithmetic (no voxels, no distances,
no weights), so both the GPU path and the CPU oracle can draw from it.

Conventions
-----------
* Pinhole cameras: fx = fy = 100 * W / 160 with the principal point at the
  image centre; pixel (i, j) looks along ((i + 0.5 - W/2)/fx, (j + 0.5 - H/2)/fy, 1).
  Camera frame: x right, y down, z forward.  World frame: z up.
* Depth noise is added to the camera-frame depth z and the point is placed on
  its pixel ray at the noisy depth.  LiDAR noise is along the beam.
* Invalid pixels and beams without a return are NaN points.  Points beyond the
  sensor's maximum range are kept (the integrator rejects them).
* Poses are float32 [3, 4] row-major T_world_sensor.
* Intersections are computed in float64 and written as float32.
* Only elementwise numpy arithmetic is used (no BLAS products), so a frame is bit-identical
  however many threads generate frames concurrently.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Tuple

import numpy as np

SEED_BASE = 1611036310


# --------------------------------------------------------------------------
# Workload container
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    params: dict                      # integrator parameters of the workload
    poses: np.ndarray                 # float32 [F, 3, 4]
    frame_fn: Callable[[int], np.ndarray]   # frame index -> float32 [N, 3]
    width: int = 0
    height: int = 0
    description: str = ""

    @property
    def n_frames(self) -> int:
        return int(self.poses.shape[0])

    def frame(self, k: int) -> np.ndarray:
        return self.frame_fn(k)

    def frames(self, lo: int = 0, hi: Optional[int] = None):
        hi = self.n_frames if hi is None else hi
        for k in range(lo, hi):
            yield self.frame_fn(k), self.poses[k]


def _cached(fn):
    cache = {}

    def get(k):
        if k not in cache:
            cache[k] = fn(k)
        return cache[k]
    return get


# --------------------------------------------------------------------------
# Ray casting against analytic primitives (float64)
# --------------------------------------------------------------------------
def _hit_room_inside(o, d, lo, hi):
    """Distance to the exit of an axis-aligned room, ray starting inside."""
    t = np.full(d.shape[0], np.inf)
    for k in range(3):
        dk = d[:, k]
        with np.errstate(divide="ignore", invalid="ignore"):
            tk = np.where(dk > 0, (hi[k] - o[k]) / dk,
                          np.where(dk < 0, (lo[k] - o[k]) / dk, np.inf))
        t = np.minimum(t, tk)
    return t


def _hit_boxes(o, d, boxes):
    """Nearest entry distance into any of the solid boxes [(lo, hi)], origin outside."""
    best = np.full(d.shape[0], np.inf)
    # directions never have an exactly zero component here except by accident;
    # nudge zeros so the slab arithmetic stays finite
    dd = np.where(d == 0.0, 1e-300, d)
    inv = [1.0 / dd[:, k] for k in range(3)]
    for lo, hi in boxes:
        tmin = np.full(d.shape[0], -np.inf)
        tmax = np.full(d.shape[0], np.inf)
        for k in range(3):
            t1 = (lo[k] - o[k]) * inv[k]
            t2 = (hi[k] - o[k]) * inv[k]
            tmin = np.maximum(tmin, np.minimum(t1, t2))
            tmax = np.minimum(tmax, np.maximum(t1, t2))
        ok = (tmax >= tmin) & (tmin > 1e-9) & (tmin < best)
        best = np.where(ok, tmin, best)
    return best


def _dot3(d, v):
    """Row-wise dot product of d [n, 3] with a 3-vector, elementwise (no BLAS)."""
    return (d[:, 0] * v[0] + d[:, 1] * v[1]) + d[:, 2] * v[2]


def _hit_spheres(o, d, spheres):
    best = np.full(d.shape[0], np.inf)
    dd = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    for c, r in spheres:
        oc = o - c
        b = _dot3(d, oc)
        cc = float((oc[0] * oc[0] + oc[1] * oc[1]) + oc[2] * oc[2]) - r * r
        disc = b * b - dd * cc
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t = (-b - sq) / dd
        ok &= t > 1e-9
        best = np.where(ok & (t < best), t, best)
    return best


def _hit_cylinders(o, d, cyls):
    """Vertical solid cylinders (cx, cy, r, h) standing on z = 0; side and top cap."""
    best = np.full(d.shape[0], np.inf)
    a = d[:, 0] ** 2 + d[:, 1] ** 2
    for cx, cy, r, h in cyls:
        ox, oy = o[0] - cx, o[1] - cy
        b = d[:, 0] * ox + d[:, 1] * oy
        c = ox * ox + oy * oy - r * r
        disc = b * b - a * c
        ok = (disc >= 0) & (a > 0)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (-b - np.sqrt(np.where(ok, disc, 0.0))) / a
        z = o[2] + t * d[:, 2]
        ok &= (t > 1e-9) & (z >= 0) & (z <= h)
        best = np.where(ok & (t < best), t, best)
        # top cap
        with np.errstate(divide="ignore", invalid="ignore"):
            tc = (h - o[2]) / d[:, 2]
        xc = o[0] + tc * d[:, 0] - cx
        yc = o[1] + tc * d[:, 1] - cy
        okc = (tc > 1e-9) & (xc * xc + yc * yc <= r * r)
        best = np.where(okc & (tc < best), tc, best)
    return best


def _hit_ground(o, d):
    with np.errstate(divide="ignore", invalid="ignore"):
        t = -o[2] / d[:, 2]
    return np.where((d[:, 2] < 0) & (t > 0), t, np.inf)


# --------------------------------------------------------------------------
# Sensors
# --------------------------------------------------------------------------
def pinhole_dirs(width: int, height: int) -> np.ndarray:
    """Camera-frame pixel directions with unit z, float64 [H*W, 3], row-major pixels."""
    f = 100.0 * width / 160.0
    i = (np.arange(width) + 0.5 - width / 2.0) / f
    j = (np.arange(height) + 0.5 - height / 2.0) / f
    jj, ii = np.meshgrid(j, i, indexing="ij")
    return np.stack([ii.ravel(), jj.ravel(), np.ones(width * height)], axis=1)


def lidar_dirs(n_beams: int = 64, n_az: int = 2048, el_lo: float = -25.0,
               el_hi: float = 3.0) -> np.ndarray:
    """Unit beam directions in the sensor frame (x forward, y left, z up), [beams*az, 3]."""
    el = np.deg2rad(np.linspace(el_lo, el_hi, n_beams))
    az = 2.0 * np.pi * np.arange(n_az) / n_az
    ee, aa = np.meshgrid(el, az, indexing="ij")
    return np.stack([(np.cos(ee) * np.cos(aa)).ravel(), (np.cos(ee) * np.sin(aa)).ravel(),
                     np.sin(ee).ravel()], axis=1)


def camera_rotation(forward, down=(0.0, 0.0, -1.0)) -> np.ndarray:
    """R_world_cam whose columns are the camera x (right), y (down), z (forward) axes."""
    z = np.asarray(forward, float)
    z = z / np.linalg.norm(z)
    y = np.asarray(down, float)
    y = y - z * (y @ z)
    y = y / np.linalg.norm(y)
    x = np.cross(y, z)
    return np.stack([x, y, z], axis=1)


def make_pose(R: np.ndarray, t) -> np.ndarray:
    T = np.zeros((3, 4), np.float64)
    T[:, :3] = R
    T[:, 3] = t
    return T.astype(np.float32)


def _depth_frame(pose32, dirs_cam, hit_fn, sigma_fn, rng, invalid_rate=0.0):
    """Cast pixel rays, add depth noise, return camera-frame float32 points (NaN = invalid)."""
    pose = pose32.astype(np.float64)
    R, t = pose[:, :3], pose[:, 3]
    d_world = np.stack([_dot3(dirs_cam, R[k]) for k in range(3)], axis=1)
    tz = hit_fn(t, d_world)                 # distance along d_world; dirs have unit z
    z = tz.copy()                           # camera-frame depth of the hit
    ok = np.isfinite(z)
    sig = sigma_fn(np.where(ok, z, 1.0))
    zn = z + rng.standard_normal(z.shape[0]) * sig
    ok &= zn > 0
    if invalid_rate > 0:
        ok &= rng.random(z.shape[0]) >= invalid_rate
    pts = dirs_cam * zn[:, None]
    pts[~ok] = np.nan
    return pts.astype(np.float32)


# --------------------------------------------------------------------------
# Scene builders
# --------------------------------------------------------------------------
def _room_scene_c1(rng):
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([4.0, 4.0, 3.0])
    cam = np.array([2.0, 2.0, 1.5])
    spheres = []
    while len(spheres) < 3:
        r = rng.uniform(0.3, 0.6)
        c = rng.uniform(lo + r, hi - r)
        if np.linalg.norm(c - cam) < r + 0.3:
            continue
        spheres.append((c, r))
    return lo, hi, cam, spheres


def config1(seed: int = SEED_BASE + 0) -> Workload:
    """Single 160x120 depth frame of a 4x4x3 m box room with 3 spheres."""
    rng = np.random.default_rng(seed)
    lo, hi, cam, spheres = _room_scene_c1(rng)
    R = camera_rotation([1.0, 0.0, 0.0])
    pose = make_pose(R, cam)
    dirs = pinhole_dirs(160, 120)

    def hit(o, d):
        return np.minimum(_hit_room_inside(o, d, lo, hi), _hit_spheres(o, d, spheres))

    frame_rng = np.random.default_rng(seed + 7919)

    @_cached
    def frame(k):
        return _depth_frame(pose, dirs, hit, lambda z: 0.005 * z * z, frame_rng)

    params = dict(voxel_size=0.10, trunc=0.30, max_range=5.0, weighting="const",
                  merge="simple", storage="f32")
    return Workload("c1_room_160x120", params, pose[None], frame, 160, 120,
                    "single 160x120 frame, 4x4x3 m room, 3 spheres, sigma=0.005 z^2")


def _circle_dist_box(lo, hi, radius=1.5, height=1.5, n=720):
    th = np.linspace(0, 2 * np.pi, n, endpoint=False)
    p = np.stack([radius * np.cos(th), radius * np.sin(th), np.full(n, height)], axis=1)
    q = np.maximum(np.maximum(lo - p, 0.0), p - hi)
    return float(np.min(np.linalg.norm(q, axis=1)))


def _room_scene_c2(rng, clear=0.5):
    lo, hi = np.array([-5.0, -5.0, 0.0]), np.array([5.0, 5.0, 3.0])
    boxes = []
    while len(boxes) < 20:
        fx, fy = rng.uniform(0.2, 1.5, size=2)
        h = rng.uniform(0.2, 2.0)
        cx = rng.uniform(-5 + fx / 2, 5 - fx / 2)
        cy = rng.uniform(-5 + fy / 2, 5 - fy / 2)
        blo = np.array([cx - fx / 2, cy - fy / 2, 0.0])
        bhi = np.array([cx + fx / 2, cy + fy / 2, h])
        if _circle_dist_box(blo, bhi) < clear:
            continue
        boxes.append((blo, bhi))
    spheres = []
    while len(spheres) < 10:
        r = rng.uniform(0.2, 0.6)
        c = rng.uniform(lo + r, hi - r)
        rho = math.hypot(c[0], c[1])
        if math.hypot(rho - 1.5, c[2] - 1.5) - r < clear:
            continue
        spheres.append((c, r))
    return lo, hi, boxes, spheres


def room_sequence(width: int, height: int, n_frames: int, seed: int, phase: float = 0.0,
                  invalid_rate: float = 0.05, noise_scale: float = 1.0):
    """Camera on a 1.5 m circle at 1.5 m height in a 10x10x3 m furnished room,
    optical axis radially outward; returns (poses, frame_fn).  noise_scale multiplies the
    depth noise (0 with invalid_rate 0: the exact surface points of the same scene and poses,
    i.e. ground truth)."""
    rng = np.random.default_rng(seed)
    lo, hi, boxes, spheres = _room_scene_c2(rng)
    poses = []
    for k in range(n_frames):
        th = phase + 2.0 * np.pi * k / 100.0
        c = np.array([1.5 * np.cos(th), 1.5 * np.sin(th), 1.5])
        R = camera_rotation([np.cos(th), np.sin(th), 0.0])
        poses.append(make_pose(R, c))
    poses = np.stack(poses)
    dirs = pinhole_dirs(width, height)

    def hit(o, d):
        t = _hit_room_inside(o, d, lo, hi)
        t = np.minimum(t, _hit_boxes(o, d, boxes))
        return np.minimum(t, _hit_spheres(o, d, spheres))

    def sigma(z):
        return noise_scale * (0.0012 + 0.0019 * (z - 0.4) ** 2)

    def frame(k):
        frng = np.random.default_rng([seed, 104729, k])
        return _depth_frame(poses[k], dirs, hit, sigma, frng, invalid_rate)
    return poses, frame


def config2(n_frames: int = 100, seed: int = SEED_BASE + 1, width: int = 640,
            height: int = 480, cache: bool = True) -> Workload:
    """100-frame 640x480 depth sequence in a 10x10x3 m room with 20 boxes and 10 spheres."""
    poses, frame = room_sequence(width, height, n_frames, seed)
    params = dict(voxel_size=0.05, trunc=0.15, max_range=5.0, weighting="quad",
                  merge="grouped", storage="f32")
    return Workload(f"c2_room_{width}x{height}x{n_frames}", params, poses,
                    _cached(frame) if cache else frame, width, height,
                    "640x480 depth, circular path r=1.5 m, 20 boxes + 10 spheres, 5% invalid")


def _street_scene(rng):
    buildings = []
    for side in (-1.0, 1.0):
        for _ in range(20):
            wx, wy = rng.uniform(8.0, 20.0, size=2)
            h = rng.uniform(5.0, 20.0)
            cx = rng.uniform(-100.0, 100.0)
            near = rng.uniform(8.0, 12.0)
            ylo, yhi = (near, near + wy) if side > 0 else (-near - wy, -near)
            buildings.append((np.array([cx - wx / 2, ylo, 0.0]), np.array([cx + wx / 2, yhi, h])))
    trees = []
    for _ in range(60):
        r = rng.uniform(0.2, 0.5)
        h = rng.uniform(3.0, 8.0)
        y = rng.uniform(5.0, 7.0) * (1.0 if rng.random() < 0.5 else -1.0)
        x = rng.uniform(-100.0, 100.0)
        trees.append((x, y, r, h))
    return buildings, trees


def config3(n_sweeps: int = 50, seed: int = SEED_BASE + 2, n_beams: int = 64,
            n_az: int = 2048, cache: bool = True) -> Workload:
    """50 sweeps of a 64-beam LiDAR driving 1 m per sweep along a synthetic street."""
    rng = np.random.default_rng(seed)
    buildings, trees = _street_scene(rng)
    dirs = lidar_dirs(n_beams, n_az)
    poses = np.stack([make_pose(np.eye(3), [-24.5 + k, 0.0, 1.8]) for k in range(n_sweeps)])

    def frame(k):
        frng = np.random.default_rng([seed, 15485863, k])
        o = poses[k].astype(np.float64)[:, 3]
        t = _hit_ground(o, dirs)
        t = np.minimum(t, _hit_boxes(o, dirs, buildings))
        t = np.minimum(t, _hit_cylinders(o, dirs, trees))
        ok = np.isfinite(t)
        tn = t + frng.standard_normal(t.shape[0]) * 0.02
        ok &= tn > 0
        pts = dirs * np.where(ok, tn, 0.0)[:, None]
        pts[~ok] = np.nan
        return pts.astype(np.float32)

    params = dict(voxel_size=0.20, trunc=0.60, max_range=60.0, weighting="const",
                  merge="simple", storage="f32")
    return Workload(f"c3_street_lidar_{n_beams}x{n_az}x{n_sweeps}", params, poses,
                    _cached(frame) if cache else frame, n_az, n_beams,
                    "64-beam LiDAR, street with 40 buildings and 60 trees, sigma 2 cm")


MULTI_RES = ((160, 120), (320, 240), (640, 480))
MULTI_VOXEL = (0.02, 0.05, 0.10)


def multi_map_class(m: int) -> Tuple[int, int]:
    """Sensor class of map m in the 32-map mix: 8 x 160x120, 16 x 320x240, 8 x 640x480."""
    if m % 4 == 0:
        return MULTI_RES[0]
    if m % 4 == 3:
        return MULTI_RES[2]
    return MULTI_RES[1]


def config4_map(m: int, n_ticks: int = 100, seed: int = SEED_BASE + 3,
                storage: str = "f16") -> Workload:
    """Map m of the 32-map batched mix: its own furnished room, its own trajectory phase."""
    w, h = multi_map_class(m)
    v = MULTI_VOXEL[m % 3]
    poses, frame = room_sequence(w, h, n_ticks, seed + 1000 * (m + 1),
                                 phase=2.0 * np.pi * m / 32.0)
    params = dict(voxel_size=v, trunc=3.0 * v, max_range=5.0, weighting="quad",
                  merge="grouped", storage=storage)
    return Workload(f"c4_map{m}_{w}x{h}", params, poses, _cached(frame), w, h,
                    "one map of the 32-map batched mix")


# --------------------------------------------------------------------------
# The simulated ESDF benchmark: a 10 x 10 x 10 m space with three planes (the ground and two
# walls), a cube and a sphere, seen by a noiseless 320x240 depth sensor (5 m range) from random
# six-degree-of-freedom poses in free space at least 1 m from every obstacle.
# --------------------------------------------------------------------------
def _esdf_scene(rng):
    cube = (np.array([2.0, 5.5, 0.0]) + rng.uniform(-0.5, 0.5, 3) * [1, 1, 0],)
    cube = (cube[0], cube[0] + np.array([2.0, 2.0, 2.0]))
    sphere = (np.array([6.5, 3.5, 2.5]) + rng.uniform(-0.5, 0.5, 3), 1.25)
    return cube, sphere


def esdf_scene_distance(p, cube, sphere) -> np.ndarray:
    """Signed distance (metres) from points p [n,3] to the scene's solids: the ground (z < 0), the
    walls x < 0 and y > 10, the cube and the sphere; positive in free space."""
    p = np.asarray(p, np.float64)
    d = p[:, 2].copy()
    d = np.minimum(d, p[:, 0])
    d = np.minimum(d, 10.0 - p[:, 1])
    lo, hi = cube
    q = np.maximum(lo - p, p - hi)
    outside = np.sqrt((np.maximum(q, 0.0) ** 2).sum(axis=1))
    inside = np.minimum(q.max(axis=1), 0.0)
    d = np.minimum(d, outside + inside)
    c, r = sphere
    d = np.minimum(d, np.sqrt(((p - c) ** 2).sum(axis=1)) - r)
    return d


def _random_rotation(rng) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def esdf_benchmark(n_views: int = 50, width: int = 320, height: int = 240,
                   seed: int = SEED_BASE + 5):
    """Returns (poses [n,3,4] float32, frame_fn, distance_fn): noiseless depth frames of the
    simulated ESDF scene and its ground-truth signed distance at any points."""
    rng = np.random.default_rng(seed)
    cube, sphere = _esdf_scene(rng)
    poses = []
    while len(poses) < n_views:
        t = rng.uniform(1.0, 9.0, 3)
        if esdf_scene_distance(t[None, :], cube, sphere)[0] < 1.0:
            continue
        poses.append(make_pose(_random_rotation(rng), t))
    poses = np.stack(poses)
    dirs = pinhole_dirs(width, height)

    def hit(o, d):
        t = _hit_room_inside(o, d, np.array([0.0, -1e6, 0.0]), np.array([1e6, 10.0, 1e6]))
        t = np.minimum(t, _hit_boxes(o, d, [cube]))
        return np.minimum(t, _hit_spheres(o, d, [sphere]))

    def frame(k):
        frng = np.random.default_rng([seed, 7919, k])
        return _depth_frame(poses[k], dirs, hit, lambda z: 0.0 * z, frng, 0.0)

    return poses, frame, lambda p: esdf_scene_distance(p, cube, sphere)


# --------------------------------------------------------------------------
# Point colours (a textured scene for the colour layer)
# --------------------------------------------------------------------------
def point_colors(points: np.ndarray, pose: np.ndarray, seed: int, k: int = 0,
                 cell: float = 0.3, noise: float = 8.0) -> np.ndarray:
    """RGBA8 colours (red in the low byte, alpha 255) of sensor-frame points seen from `pose`:
    a checker texture of 0.3 m world cells, each cell a seeded palette colour, plus per-point
    sensor noise (normal, sigma `noise` per channel, frame k's own draw), rounded and clipped to
    [0, 255].  Invalid (NaN) points get 0.  Elementwise arithmetic only."""
    p = np.asarray(points, np.float64).reshape(-1, 3)
    T = np.asarray(pose, np.float64).reshape(3, 4)
    w = [T[r, 0] * p[:, 0] + T[r, 1] * p[:, 1] + T[r, 2] * p[:, 2] + T[r, 3] for r in range(3)]
    ok = np.isfinite(w[0]) & np.isfinite(w[1]) & np.isfinite(w[2])
    cx = [np.floor(np.where(ok, x, 0.0) / cell).astype(np.int64) for x in w]
    h = (cx[0] * 73856093) ^ (cx[1] * 19349663) ^ (cx[2] * 83492791) ^ int(seed % (1 << 30))
    h = h & 0xFFFFFF
    base = np.stack([(h >> (8 * c)) & 255 for c in range(3)], axis=1).astype(np.float64)
    rng = np.random.default_rng([seed, 7919, k])
    val = np.clip(np.rint(base + rng.normal(0.0, noise, size=base.shape)), 0, 255).astype(np.uint32)
    out = val[:, 0] | (val[:, 1] << 8) | (val[:, 2] << 16) | np.uint32(255 << 24)
    return np.where(ok, out, np.uint32(0)).astype(np.uint32)
