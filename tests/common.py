"""Helpers shared by the GPU parity tests: run the oracle and the GPU library on the same
seeded inputs and compare them to the parity bar.

Comparison rules
----------------
* Bit-exact: the allocated block set, the touched voxels with their ray counts, and W under
  constant weighting with binary32 storage (W is then an integer count).
* D and W: within the bounds of :func:`compare_export`, which add to the flat tol_d (1e-4 v for
  binary32 storage, 2e-3 v for binary16 storage) only what the binary32 distance error and the
  fixed-point sums can propagate, and report how many voxels needed that addition.
"""
from __future__ import annotations

import sys

import numpy as np

import oracle


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_map(params: dict, **over):
    p = dict(params)
    p.update(over)
    return oracle.OracleMap(p["voxel_size"], p["trunc"], weighting=p.get("weighting", "const"),
                            merge=p.get("merge", "simple"), w_max=p.get("w_max", 1e4),
                            max_range=p.get("max_range", 5.0), z_min=p.get("z_min", 0.1),
                            storage=p.get("storage", "f32"), dist=p.get("dist", "eq1"),
                            full_ray=p.get("full_ray", False), color=p.get("color", False))


def gpu_map(vbx, params: dict, **over):
    p = dict(params)
    p.update(over)
    return vbx.Map(p["voxel_size"], p["trunc"], weighting=p.get("weighting", "const"),
                   merge=p.get("merge", "simple"), storage=p.get("storage", "f32"),
                   w_max=p.get("w_max", 1e4), max_range=p.get("max_range", 5.0),
                   z_min=p.get("z_min", 0.1), dist=p.get("dist", "eq1"),
                   block_capacity=p.get("block_capacity", 4096),
                   keep_touches=p.get("keep_touches", True), full_ray=p.get("full_ray", False),
                   color=p.get("color", False))


def touches_dict(coords, counts):
    return dict(zip(map(tuple, np.asarray(coords).tolist()), np.asarray(counts).tolist()))


def compare_touches(gpu, orc):
    g = touches_dict(*gpu)
    o = touches_dict(*orc)
    if g != o:
        only_g = set(g) - set(o)
        only_o = set(o) - set(g)
        diff = [k for k in set(g) & set(o) if g[k] != o[k]]
        raise AssertionError(f"touch sets differ: {len(only_g)} only on GPU, {len(only_o)} only in "
                             f"oracle, {len(diff)} with different counts (of {len(o)})")
    return len(o)


def _ulp_half(x: np.ndarray) -> np.ndarray:
    """Spacing of binary16 numbers at |x| (2^-24 below the normal range)."""
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    return np.where(ax >= 2.0 ** -14, 2.0 ** (e - 10), 2.0 ** -24)


def distance_error(params: dict) -> float:
    """Bound e on the difference between the kernel's binary32 Eq. (1) distance and the exact one
    from the same ray end point: each offset p_k - (g_k + 1/2) v is formed from the exact centre
    with two roundings (2u relative, u = 2^-24), the squared norm adds three more, the square
    root halves the total and the hardware root (within one ulp) adds two: 5.5u |p - x| in all,
    with |p - x| <= delta + v for a voxel the band visits.  The stated bound rounds that up to 8u."""
    v = float(np.float32(params["voxel_size"]))
    delta = float(np.float32(params["trunc"]))
    if "dist_err" in params:        # a path whose distance error has another bound (stated there)
        return float(params["dist_err"])
    return 8.0 * 2.0 ** -24 * (delta + v)


def weight_fraction_bits(params: dict) -> int:
    """Fractional bits kw of the kernels' fixed-point per-voxel sums: 38 - c with 2^c the smallest
    power of two >= 1 / z_min^2 under quadratic weighting (c = 0 under constant weighting)."""
    if params.get("weighting", "const") == "const":
        return 38
    zf = np.float32(params.get("z_min", 0.1))
    wmax = np.float32(1.0) / (zf * zf)
    c = 0
    while np.float32(2.0 ** c) < wmax:
        c += 1
    return 38 - c


def compare_export(gpu_export, orc_export, params: dict, storage: str = "f32", quiet: bool = False):
    """Compares a GPU export with the oracle's on the same frames.

    D bound per voxel (metres): tol_d + e (1 + 2 delta M / ((delta - eps) W)) + q 2 delta / W, where
    * tol_d = 1e-4 v for binary32 storage.  For the 16-bit storages ("f16", "s16"), compared with
      the oracle's mode that rounds to the same storage after every frame, tol_d = 2^-10 delta plus
      one storage step (2^-11 delta for binary16 D / delta, delta / 32767 for the fixed-point code):
      the kernels' binary32 update and the oracle's binary64 one can round to neighbouring stored
      values where the exact result lies a hair from a midpoint.  A flipped D differs by one step;
      a flipped binary16 W (relative 2^-10 at most) changes the weight of a later frame's update,
      which moves D by at most 2^-10 W s |d - D| / (W + s)^2 <= 2^-11 delta (|d - D| <= 2 delta);
      two such W flips and one D flip make the bound;
    * e is the binary32 distance error bound of :func:`distance_error`; on the Eq. (5) ramp a ray's
      weight moves with its distance (slope 1 / (delta - eps)), so an error e in d moves D by at most
      e (1 + sum over those rays of w |d - D| / ((delta - eps) W)) <= e (1 + 2 delta M / ((delta - eps) W)).
      The rays concerned are those within e of the ramp (a ray just beyond -delta, or just in front
      of -eps, in the oracle can fall on it in binary32), so M, the summed point weight of every ray
      that saw the voxel, bounds their weight; the ramp term is 0 under constant weighting.  Where W
      is close to M (a voxel seen in front of the ramp) the bound is tol_d + 4e;
    * q = n 2^-kw / 2 bounds the rounding of the fixed-point sums of the voxel's n rays, with
      n <= mass / w_min (every ray carries at least one point's weight, 1 or 1/max_range^2).
    Away from the ramp and for any voxel of fair weight the bound is tol_d plus a few 1e-6 v.
    W bound: rtol W + e M / (delta - eps) + q, rtol = 1e-5 (binary32) or 2e-3 (binary16 W, plus
    one binary16 step of W for a flipped rounding).
    For 16-bit storage the result also counts the differences in storage steps (binary16 ulps of
    D / delta, or 1/32767 of delta), since a binary32 result a hair from a rounding midpoint can
    round to the neighbouring step on one side only.
    Constant weighting with binary32 storage: W bit-exact.
    Returns the statistics, including how many voxels needed more than the plain tol_d."""
    coords, dw = gpu_export
    oc, oD, oW, oM = orc_export[:4]
    oR = orc_export[4] if len(orc_export) > 4 else None
    assert np.array_equal(coords, oc), f"block sets differ: {coords.shape[0]} vs {oc.shape[0]}"
    v = float(np.float32(params["voxel_size"]))
    delta = float(np.float32(params["trunc"]))
    quad = params.get("weighting", "const") == "quad"
    if storage == "f32":
        tol_d = 1e-4 * v
    else:
        tol_d = 2.0 ** -10 * delta + (2.0 ** -11 * delta if storage == "f16" else delta / 32767.0)
    rtol = 1e-5 if storage == "f32" else 2e-3
    e = distance_error(params)
    w_min = 1.0 / float(params.get("max_range", 5.0)) ** 2 if quad else 1.0
    D = dw[:, :, 0].astype(np.float64)
    W = dw[:, :, 1].astype(np.float64)
    if not quad and storage == "f32":
        bad = np.count_nonzero(W != oW)
        assert bad == 0, f"constant-weight W differs in {bad} voxels"
    Mq = oM if quad else np.zeros_like(oW)
    q = (oM / w_min) * 2.0 ** -(weight_fraction_bits(params) + 1)
    # 16-bit storage keeps W in binary16: one flipped rounding is one binary16 step of W, which
    # below 2^-14 (the subnormal range) is a fixed 2^-24 rather than a relative 2^-11
    wflip = _ulp_half(oW) if storage != "f32" else 0.0
    werr = np.abs(W - oW) - (rtol * oW + wflip + e * Mq / (delta - v) + q)
    if werr.max(initial=-1) > 0:
        b, l = np.unravel_index(np.argmax(werr), W.shape)
        raise AssertionError(
            f"W out of tolerance ({storage}) in {np.count_nonzero(werr > 0)} voxels; worst at block "
            f"{coords[b].tolist()} voxel {l}: W {W[b, l]!r} vs {oW[b, l]!r} (excess {werr[b, l]:.3g}), "
            f"D {D[b, l]!r} vs {oD[b, l]!r}, ray weight sum {oM[b, l]!r}"
            + (f", on the ramp {oR[b, l]!r}" if oR is not None else ""))
    known = oW > 0
    Wk = np.where(known, oW, 1.0)
    tol_vox = tol_d + e * (1.0 + 2.0 * delta / (delta - v) * Mq / Wk) + q * 2.0 * delta / Wk
    derr = np.where(known, np.abs(D - oD), 0.0)
    ratio = derr / tol_vox
    if ratio.max(initial=0.0) > 1.0:
        b, l = np.unravel_index(np.argmax(ratio), D.shape)
        raise AssertionError(
            f"D out of tolerance in {np.count_nonzero(ratio > 1.0)} voxels; worst at block "
            f"{coords[b].tolist()} voxel {l}: D {D[b, l]!r} vs {oD[b, l]!r} (bound {tol_vox[b, l]!r}), "
            f"W {W[b, l]!r} vs {oW[b, l]!r}, ray weight sum {oM[b, l]!r}"
            + (f", on the ramp {oR[b, l]!r}" if oR is not None else ""))
    above = known & (derr > tol_d)
    res = dict(blocks=int(coords.shape[0]), known=int(known.sum()),
               max_d_err=float(derr.max(initial=0.0)),
               max_d_err_voxels=float(derr.max(initial=0.0)) / v,
               worst_ratio=float(ratio.max(initial=0.0)),
               above_plain_tol=int(above.sum()),
               max_d_err_voxels_above_plain=float(derr[above].max(initial=0.0)) / v,
               tiny_weight=int((known & (oW < 1e-3 * oM)).sum()),
               ramp_seen=int((known & (oR > 0)).sum()) if oR is not None else None)
    if storage != "f32":
        # in storage steps: a binary16 ulp of D / delta, or the fixed-point step 1/32767 of delta
        step = _ulp_half(oD / delta) * delta if storage == "f16" else np.full(oD.shape, delta / 32767.0)
        steps = np.where(known, derr / step, 0.0)
        res["max_steps"] = float(steps.max(initial=0.0))
        res["above_1step"] = int((steps > 1.0).sum())
        res["above_2e-3v"] = int((derr > 2e-3 * v).sum())
        wstep = _ulp_half(oW)
        res["max_w_steps"] = float(np.where(known, np.abs(W - oW) / wstep, 0.0).max(initial=0.0))
    if not quiet:
        log(f"  compare ({storage}): {res}")
    return res
