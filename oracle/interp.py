"""Oracle of the distance query by trilinear interpolation (test infrastructure).

Only the test-suite may import this module; the product library never loads it.  It follows the accuracy evaluation of Sec. VI-A: a ground-truth surface point is
looked up in the distance field by trilinear interpolation over the eight voxels around it,
and the interpolated distance is that point's error.

Readings (stated, since the paper gives no formula):

* voxel (i, j, k) holds the field at its centre ((i, j, k) + 1/2) v;
* a query is known only where all eight voxels around it are allocated and observed (W > 0);
* the corner choice takes u = x * (1/v) - 1/2 per axis in binary32, with the binary32
  reciprocal of v that the map holds, corner floor(u) and fraction u - floor(u) (a binary32
  subtraction, rounded where u lies in (-1/2, 0)), so that CPU and GPU pick the same eight
  voxels with the same fractions; the blend itself is binary64 here.
"""
from __future__ import annotations

import numpy as np

VOX_LIMIT = 1 << 18   # |voxel index| < 2^18


def interpolate(coords: np.ndarray, D: np.ndarray, W: np.ndarray, voxel_size: float,
                points: np.ndarray) -> np.ndarray:
    """Distances (float64 [N], NaN where unknown) at points (float32 [N, 3], world frame).

    coords: int [B, 3] block indices; D, W: [B, 4096] per block, voxel (x, y, z) of a block at
    index x + 16 y + 256 z.
    """
    pts = np.asarray(points, np.float32).reshape(-1, 3)
    index = {tuple(int(c) for c in b): n for n, b in enumerate(np.asarray(coords).reshape(-1, 3))}
    iv = np.float32(1.0) / np.float32(voxel_size)
    out = np.full(pts.shape[0], np.nan)
    for p in range(pts.shape[0]):
        u = pts[p] * iv - np.float32(0.5)          # binary32, one rounding per operation
        if not np.all(np.isfinite(u)):
            continue
        fl = np.floor(u)
        if np.any(fl < -VOX_LIMIT) or np.any(fl >= VOX_LIMIT - 1):
            continue
        base = fl.astype(np.int64)
        f = (u - fl).astype(np.float64)            # rounded as binary32, as the map's query does
        d = np.empty((2, 2, 2))
        known = True
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    g = base + (cx, cy, cz)
                    blk = index.get((int(g[0] >> 4), int(g[1] >> 4), int(g[2] >> 4)))
                    if blk is None:
                        known = False
                        break
                    loc = int(g[0] & 15) + 16 * int(g[1] & 15) + 256 * int(g[2] & 15)
                    if not W[blk, loc] > 0:
                        known = False
                        break
                    d[cz, cy, cx] = D[blk, loc]
                if not known:
                    break
            if not known:
                break
        if not known:
            continue
        # blend along x, then y, then z
        cx0 = d[:, :, 0] * (1.0 - f[0]) + d[:, :, 1] * f[0]     # [z, y]
        cy0 = cx0[:, 0] * (1.0 - f[1]) + cx0[:, 1] * f[1]       # [z]
        out[p] = cy0[0] * (1.0 - f[2]) + cy0[1] * f[2]
    return out


def surface_error(dist: np.ndarray, trunc: float) -> dict:
    """The evaluation's error statistics over the known queries of ground-truth surface points:
    |distance| capped at the truncation distance."""
    known = np.isfinite(dist)
    e = np.minimum(np.abs(dist[known]), trunc)
    return {"known": int(known.sum()), "total": int(dist.size),
            "mean": float(e.mean()) if e.size else float("nan"),
            "rms": float(np.sqrt(np.mean(e * e))) if e.size else float("nan")}
