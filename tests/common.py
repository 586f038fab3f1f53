"""Helpers shared by the GPU parity tests: run the oracle and the GPU library on the same
seeded inputs and compare them to the parity bar.

Comparison rules
----------------
* Bit-exact: the allocated block set, the touched voxels with their ray counts, and W under
  constant weighting with binary32 storage (W is then an integer count).
* D (metres): |D - D_oracle| <= tol_d (1 + 2 delta / (delta - eps) * R / W_oracle) for every voxel
  the oracle knows with a weight that is not vanishingly small; tol_d = 1e-4 v (binary32
  storage) or 2e-3 v (binary16 storage, compared with the oracle's binary16-emulating mode).
  R is the summed weight of the rays that saw the voxel on the Eq. (5) drop-off ramp (0 under
  constant weighting and for voxels seen only in front of the ramp).  On the ramp a ray's
  weight moves with its distance, slope 1/(delta - eps), so a distance rounding error e moves D
  by up to e (1 + sum over ramp rays of w |d - D| / ((delta - eps) W)) <= e (1 + 2 delta R /
  ((delta - eps) W)); the binary32 geometry's error is a few ulps of the world coordinates.
  "Vanishingly small": W_oracle below 1e-3 of the voxel's summed ray weights, i.e. the voxel
  was only seen in the last 1/1000 of the ramp.
* W: |W - W_oracle| <= rtol W_oracle + (tol_d / (delta - eps)) * mass, where mass is the
  voxel's summed ray weights: the second term is the weight change that a distance error of
  tol_d causes through the Eq. (5) ramp.  rtol = 1e-5 (binary32) or 2e-3 (binary16).
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
                            storage=p.get("storage", "f32"), dist=p.get("dist", "eq1"))


def gpu_map(vbx, params: dict, **over):
    p = dict(params)
    p.update(over)
    return vbx.Map(p["voxel_size"], p["trunc"], weighting=p.get("weighting", "const"),
                   merge=p.get("merge", "simple"), storage=p.get("storage", "f32"),
                   w_max=p.get("w_max", 1e4), max_range=p.get("max_range", 5.0),
                   z_min=p.get("z_min", 0.1), dist=p.get("dist", "eq1"),
                   block_capacity=p.get("block_capacity", 4096),
                   keep_touches=p.get("keep_touches", True))


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


def compare_export(gpu_export, orc_export, params: dict, storage: str = "f32"):
    coords, dw = gpu_export
    oc, oD, oW, oM = orc_export[:4]
    oR = orc_export[4] if len(orc_export) > 4 else None
    assert np.array_equal(coords, oc), f"block sets differ: {coords.shape[0]} vs {oc.shape[0]}"
    v = float(np.float32(params["voxel_size"]))
    delta = float(np.float32(params["trunc"]))
    tol_d = (1e-4 if storage == "f32" else 2e-3) * v
    rtol = 1e-5 if storage == "f32" else 2e-3
    D = dw[:, :, 0].astype(np.float64)
    W = dw[:, :, 1].astype(np.float64)
    if params.get("weighting", "const") == "const" and storage == "f32":
        bad = np.count_nonzero(W != oW)
        assert bad == 0, f"constant-weight W differs in {bad} voxels"
    atol_w = tol_d / (delta - v) * oM
    werr = np.abs(W - oW) - (rtol * oW + atol_w)
    assert werr.max(initial=-1) <= 0, f"W out of tolerance in {np.count_nonzero(werr > 0)} voxels"
    known = (oW > 0) & (oW >= 1e-3 * oM)
    tol_vox = np.full(D.shape, tol_d)
    if oR is not None and params.get("weighting", "const") == "quad":
        tol_vox = tol_d * (1.0 + 2.0 * delta / (delta - v) * oR / np.where(oW > 0, oW, 1.0))
    excess = np.where(known, np.abs(D - oD) / tol_vox, 0.0)
    derr = np.abs(D - oD)[known]
    worst = float(derr.max(initial=0.0))
    if excess.max(initial=0.0) > 1.0:
        b, l = np.unravel_index(np.argmax(excess), D.shape)
        raise AssertionError(
            f"D out of tolerance in {np.count_nonzero(excess > 1.0)} voxels; worst at block "
            f"{coords[b].tolist()} voxel {l}: D {D[b, l]!r} vs {oD[b, l]!r} (bound {tol_vox[b, l]!r}), "
            f"W {W[b, l]!r} vs {oW[b, l]!r}, ray weight sum {oM[b, l]!r}, on the ramp {oR[b, l] if oR is not None else None!r}")
    strict = known & (tol_vox <= tol_d)
    return dict(blocks=int(coords.shape[0]), known=int(known.sum()), max_d_err=worst,
                max_d_err_voxels=worst / v,
                max_d_err_voxels_off_ramp=float(np.abs(D - oD)[strict].max(initial=0.0)) / v)
