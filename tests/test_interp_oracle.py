"""Pins of the interpolation oracle against closed forms (CPU only).

Trilinear interpolation reproduces a field that is linear in x, y and z exactly, so a linear
field with distinct slopes per axis fails for a swapped axis, a wrong corner, a wrong fraction
or a wrong block/voxel index.  Queries at voxel centres return that voxel's value exactly, and
a missing or unobserved corner makes the query unknown.
"""
import numpy as np
import pytest

from oracle import interp


def linear_blocks(block_range, v, slope, offset):
    """Blocks covering block_range (per axis, inclusive lo..hi) with D linear in the voxel
    centre position, W = 1."""
    (x0, x1), (y0, y1), (z0, z1) = block_range
    coords, D = [], []
    l = np.arange(4096)
    lx, ly, lz = l & 15, (l >> 4) & 15, l >> 8
    for bx in range(x0, x1 + 1):
        for by in range(y0, y1 + 1):
            for bz in range(z0, z1 + 1):
                cx = (16 * bx + lx + 0.5) * v
                cy = (16 * by + ly + 0.5) * v
                cz = (16 * bz + lz + 0.5) * v
                coords.append((bx, by, bz))
                D.append(slope[0] * cx + slope[1] * cy + slope[2] * cz + offset)
    coords = np.array(coords, np.int32)
    D = np.array(D)
    return coords, D, np.ones_like(D)


def effective_point(q, v):
    """The point the binary32 corner choice actually interpolates at, in the units of the voxel
    centres (i + 1/2) v: (floor(u) + f + 1/2) v with u = q * (1/v) - 1/2 and f = u - floor(u),
    each rounded as binary32."""
    iv = np.float32(1.0) / np.float32(v)
    u = np.asarray(q, np.float32) * iv - np.float32(0.5)
    fl = np.floor(u)
    f = u - fl
    return (fl.astype(np.float64) + f.astype(np.float64) + 0.5) * v


@pytest.mark.parametrize("v", [0.05, 0.2])
def test_linear_field_is_reproduced_across_blocks_and_signs(v):
    slope, offset = (0.7, -1.3, 2.9), 0.25
    coords, D, W = linear_blocks(((-2, 1), (-1, 1), (-2, 0)), v, slope, offset)
    rng = np.random.default_rng(7)
    lo = np.array([-2 * 16, -1 * 16, -2 * 16]) * v + v       # keep all eight corners inside
    hi = np.array([2 * 16, 2 * 16, 1 * 16]) * v - v
    q = rng.uniform(lo, hi, size=(400, 3)).astype(np.float32)
    # points on block boundaries (corners in two to eight blocks)
    q[:8] = np.array([[0.0, 0.0, 0.0], [16 * v, 0, 0], [0, 16 * v, 0], [0, 0, -16 * v],
                      [16 * v, 16 * v, -16 * v], [-16 * v, 0.001, 0.002], [0.003, 16 * v, 0],
                      [-16 * v, -0.5 * v, -16 * v]], np.float32)
    d = interp.interpolate(coords, D, W, v, q)
    assert np.all(np.isfinite(d))
    qe = effective_point(q, v)
    expect = qe @ np.array(slope) + offset
    # the corner values are fp64 evaluations of the field: agreement to fp64 rounding
    assert np.max(np.abs(d - expect)) < 1e-12


def test_voxel_centres_return_the_voxel_value():
    v = 0.25   # centres (i + 1/2) / 4 are exact in binary32, so u is an exact integer
    rng = np.random.default_rng(3)
    coords = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [0, 0, 1], [1, 0, 1], [0, 1, 1],
                       [1, 1, 1]], np.int32)
    D = rng.normal(size=(8, 4096))
    W = np.ones_like(D)
    g = rng.integers(0, 31, size=(200, 3))
    q = ((g + 0.5) * v).astype(np.float32)
    d = interp.interpolate(coords, D, W, v, q)
    for k in range(g.shape[0]):
        b = tuple(int(x) for x in g[k] >> 4)
        blk = [tuple(c) for c in coords.tolist()].index(b)
        loc = int(g[k][0] & 15) + 16 * int(g[k][1] & 15) + 256 * int(g[k][2] & 15)
        assert d[k] == D[blk, loc]


def test_missing_or_unobserved_corner_is_unknown():
    v = 0.1
    coords, D, W = linear_blocks(((0, 1), (0, 0), (0, 0)), v, (1.0, 2.0, 3.0), 0.0)
    q = np.array([[0.5, 0.5, 0.5],                 # inside block (0, 0, 0)
                  [1.6, 0.5, 0.5],                 # corners in blocks 0 and 1 (both present)
                  [3.2, 0.5, 0.5],                 # block (2, 0, 0) missing
                  [0.5, 1.56, 0.5],                # y corner in block (0, 1, 0): missing
                  [np.nan, 0.5, 0.5],
                  [0.5, 0.5, -0.01]], np.float32)  # z corner in block (0, 0, -1): missing
    d = interp.interpolate(coords, D, W, v, q)
    assert np.isfinite(d[:2]).all() and np.isnan(d[2:]).all()
    # one unobserved corner voxel of the first query: voxel (4, 4, 4) of block (0, 0, 0)
    W2 = W.copy()
    W2[0, 4 + 16 * 4 + 256 * 4] = 0.0
    assert np.isnan(interp.interpolate(coords, D, W2, v, q[:1]))[0]


def test_surface_error_caps_at_truncation():
    s = interp.surface_error(np.array([0.01, -0.02, np.nan, 5.0]), 0.1)
    assert s["known"] == 3 and s["total"] == 4
    assert abs(s["mean"] - (0.01 + 0.02 + 0.1) / 3) < 1e-15


# ---------------------------------------------------------------------------
# Planted mistakes: each altered copy of the oracle must fail at least one pin above.
# ---------------------------------------------------------------------------
MISTAKES = [
    ("transposed voxel index", "16 * int(g[1] & 15) + 256 * int(g[2] & 15)",
     "256 * int(g[1] & 15) + 16 * int(g[2] & 15)"),
    ("swapped lerp weights", "cx0 = d[:, :, 0] * (1.0 - f[0]) + d[:, :, 1] * f[0]",
     "cx0 = d[:, :, 0] * f[0] + d[:, :, 1] * (1.0 - f[0])"),
    ("fraction of the wrong axis", "cy0 = cx0[:, 0] * (1.0 - f[1]) + cx0[:, 1] * f[1]",
     "cy0 = cx0[:, 0] * (1.0 - f[2]) + cx0[:, 1] * f[2]"),
    ("no half-voxel shift", "u = pts[p] * iv - np.float32(0.5)", "u = pts[p] * iv"),
    ("round instead of floor", "fl = np.floor(u)", "fl = np.round(u)"),
    ("every corner in the base corner's block",
     "blk = index.get((int(g[0] >> 4), int(g[1] >> 4), int(g[2] >> 4)))",
     "blk = index.get((int(base[0] >> 4), int(base[1] >> 4), int(base[2] >> 4)))"),
    ("unobserved corners accepted", "if not W[blk, loc] > 0:", "if False:"),
    ("error not capped", "e = np.minimum(np.abs(dist[known]), trunc)", "e = np.abs(dist[known])"),
]


def _altered(old, new):
    import oracle.interp as mod
    src = open(mod.__file__).read()
    assert src.count(old) == 1, old
    ns = {"__name__": "altered_interp"}
    exec(compile(src.replace(old, new), "altered_interp", "exec"), ns)

    class M:
        pass
    m = M()
    m.interpolate, m.surface_error = ns["interpolate"], ns["surface_error"]
    return m


def _pins_pass(mod):
    global interp
    saved = interp
    interp = mod
    try:
        for check in (lambda: test_linear_field_is_reproduced_across_blocks_and_signs(0.05),
                      lambda: test_linear_field_is_reproduced_across_blocks_and_signs(0.2),
                      test_voxel_centres_return_the_voxel_value,
                      test_missing_or_unobserved_corner_is_unknown,
                      test_surface_error_caps_at_truncation):
            try:
                check()
            except AssertionError:
                return False
        return True
    finally:
        interp = saved


def test_pins_pass_on_the_oracle_itself():
    import oracle.interp as mod
    assert _pins_pass(mod)


@pytest.mark.parametrize("name,old,new", MISTAKES, ids=[m[0] for m in MISTAKES])
def test_planted_mistake_is_caught(name, old, new):
    assert not _pins_pass(_altered(old, new)), f"no pin catches: {name}"
