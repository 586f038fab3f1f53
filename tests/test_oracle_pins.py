"""The CPU oracle against what the paper and plain mathematics fix (no GPU needed)."""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
from tests import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(oracle_lib, pin):
    pin()


# Plausible mistakes planted in a copy of the oracle; each must be caught by a pin.
MUTATIONS = {
    "eq1_sign_flipped": ("double sgn = dot > 0.0f ? 1.0 : (dot < 0.0f ? -1.0 : 0.0);",
                         "double sgn = dot > 0.0f ? -1.0 : (dot < 0.0f ? 1.0 : 0.0);"),
    "tie_to_highest_axis": ("if (axis < 0 || tM[k] < tM[axis]) axis = k;",
                            "if (axis < 0 || tM[k] <= tM[axis]) axis = k;"),
    "dropoff_slope": ("return (d + delta) / (delta - eps);", "return (d + delta) / delta;"),
    "no_weight_cap": ("vx->W = vx->W + sw < wmax ? vx->W + sw : wmax;", "vx->W = vx->W + sw;"),
    "merge_drops_old_weight": ("vx->D = (vx->W * vx->D + swd) / (vx->W + sw);",
                               "vx->D = (vx->D + swd) / (vx->W + sw);"),
    "rotation_transposed": ("q[k] = ((pose[4 * k] * x + pose[4 * k + 1] * y) + pose[4 * k + 2] * z) + pose[4 * k + 3];",
                            "q[k] = ((pose[k] * x + pose[4 + k] * y) + pose[8 + k] * z) + pose[4 * k + 3];"),
    "group_mean_unweighted": ("return wbits > 0 ? (uint64_t)rintf(ldexpf(w, wbits)) : 1u;", "return 1u;"),
    "no_band_behind_surface": ("float t1 = r + delta;", "float t1 = r;"),
    "no_distance_clamp": ("return d < -d64 ? -d64 : (d > d64 ? d64 : d);", "return d;"),
    "corner_not_centre": ("double x = ((double)g[k] + 0.5) * v64;\n                double f = ray->p64[k] - x;",
                          "double x = ((double)g[k]) * v64;\n                double f = ray->p64[k] - x;"),
    "weight_one_over_z": ("w64[nv] = P->weighting == 1 ? 1.0 / ((double)z * (double)z) : 1.0;",
                          "w64[nv] = P->weighting == 1 ? 1.0 / (double)z : 1.0;"),
    "group_weight_dropped": ("rays[nr].wgt = sw;", "rays[nr].wgt = w64[ki[lo].idx];"),
    "half_rounding_truncates": ("double r = nearbyint(ax / ulp) * ulp;", "double r = floor(ax / ulp) * ulp;"),
    # the projective distance along the ray (Sec. I reading)
    "along_ray_sign_flipped": ("dot += (ray->p64[k] - x) * es64[k];", "dot += (x - ray->p64[k]) * es64[k];"),
    "along_ray_binary32_length": ("d = dot / er;", "d = dot / (double)r;"),
    # where binary16 storage rounds: D / delta (not metres), W after the Eq. (4) cap
    "binary16_rounds_metres": (": orc_round_half(vx->D);",
                               ": orc_round_half(vx->D * (double)P->trunc) / (double)P->trunc;"),
    "binary16_rounds_w_before_cap": (
        "vx->W = vx->W + sw < wmax ? vx->W + sw : wmax;\n    if (P->fp16) {\n"
        "        vx->D = P->fp16 == 2 ? orc_round_s16(vx->D) : orc_round_half(vx->D);\n"
        "        vx->W = orc_round_half(vx->W);\n    }",
        "vx->W = P->fp16 ? orc_round_half(vx->W + sw) : vx->W + sw;\n"
        "    if (vx->W > wmax) vx->W = wmax;\n"
        "    if (P->fp16) vx->D = P->fp16 == 2 ? orc_round_s16(vx->D) : orc_round_half(vx->D);"),
    # the 16-bit fixed-point distance: D / delta in steps of 1/32767, to nearest
    "s16_rounds_metres": ("? orc_round_s16(vx->D) :",
                          "? orc_round_s16(vx->D * (double)P->trunc) / (double)P->trunc :"),
    "s16_truncates": ("double i = nearbyint(x * 32767.0);", "double i = trunc(x * 32767.0);"),
    "s16_power_of_two_step": ("return i / 32767.0;", "return i / 32768.0;"),
    "s16_stored_as_binary16": ("? orc_round_s16(vx->D) :", "? orc_round_half(vx->D) :"),
    # the Eq. (5) ramp diagnostic
    "ramp_counts_behind_band": ("if (P->weighting == 1 && d > -d64 && d <= -eps) vx->ramp += ray->wgt;",
                                "if (P->weighting == 1 && d <= -eps) vx->ramp += ray->wgt;"),
    "ramp_counts_dropped_weight": ("vx->ramp += ray->wgt;", "vx->ramp += w;"),
    # the whole-ray update (Sec. IV-B)
    "full_ray_ignored": ("float t0 = whole ? 0.0f : r - delta;", "float t0 = r - delta;"),
    # colour (Sec. IV-B): running mean with the old weight, 8-bit storage, grouped mean colour
    "color_drops_old_weight": ("nearbyint((vx->W * vx->C[k] + swc[k]) / (vx->W + sw))",
                               "nearbyint((vx->C[k] + swc[k]) / (1.0 + sw))"),
    "color_truncates": ("nearbyint((vx->W * vx->C[k] + swc[k]) / (vx->W + sw))",
                        "floor((vx->W * vx->C[k] + swc[k]) / (vx->W + sw))"),
    "group_color_ties_up": ("if (2 * r > (unsigned __int128)den || (2 * r == (unsigned __int128)den && (q & 1))) c = q + 1;",
                            "if (2 * r >= (unsigned __int128)den) c = q + 1;"),
    "group_color_first_point": ("for (int k = 0; k < 3; ++k) rays[nr].col[k] = group_color_channel(cs[k], cso);",
                                "for (int k = 0; k < 3; ++k) rays[nr].col[k] = (double)(((colors ? colors[valid[ki[lo].idx]] : 0u) >> (8 * k)) & 255u);"),
    # projection mapping (Sec. IV-B)
    "projective_pixel_rounded": ("const size_t pix = (size_t)floorf(uf) + (size_t)width * (size_t)floorf(vf);",
                                 "const size_t pix = (size_t)rintf(uf) + (size_t)width * (size_t)rintf(vf);"),
    "projective_distance_sign": ("const double d = (double)zm - z;", "const double d = z - (double)zm;"),
    "projective_rotation_not_transposed": (
        "cam[k] = (pose[k] * e[0] + pose[4 + k] * e[1]) + pose[8 + k] * e[2];",
        "cam[k] = (pose[4 * k] * e[0] + pose[4 * k + 1] * e[1]) + pose[4 * k + 2] * e[2];"),
    "projective_band_too_wide": ("if (!(zm - cam[2] > -delta)) continue;", "if (!(zm - cam[2] > -2.0f * delta)) continue;"),
    "full_ray_stops_at_point": ("float t1 = r + delta;\n    for (int k = 0; k < 3; ++k) {\n        float u = e[k] / r;",
                                "float t1 = whole ? r : r + delta;\n    for (int k = 0; k < 3; ++k) {\n        float u = e[k] / r;"),
}

FAST_FIRST = [pins.pin_head_on_plane, pins.pin_full_ray_head_on, pins.pin_projective_plane, pins.pin_dropoff_values,
              pins.pin_running_average, pins.pin_color_sequence, pins.pin_color_group_mean,
              pins.pin_along_ray_off_axis, pins.pin_binary16_sequence, pins.pin_s16_sequence,
              pins.pin_ramp_diagnostic,
              pins.pin_validity, pins.pin_identical_points, pins.pin_merged_singletons,
              pins.pin_group_mean, pins.pin_round_half, pins.pin_weight_sums,
              pins.pin_permutation, pins.pin_dda_dyadic, pins.pin_dda_random]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(oracle_lib, name):
    old, new = MUTATIONS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    tmp = tempfile.mkdtemp(prefix="orc_mut_")
    try:
        path = os.path.join(tmp, "vbx_oracle.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = os.path.join(tmp, "liboracle_mut.so")
        subprocess.run(["gcc", *oracle.CFLAGS, path, "-o", lib, "-lm"], check=True)
        caught = []
        for pin in FAST_FIRST:
            try:
                pin(lib)
            except AssertionError:
                caught.append(pin.__name__)
                break
        assert caught, f"planted mistake '{name}' passed every pin"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
