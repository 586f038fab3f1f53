"""Pins of the CPU oracle: checks against what the paper and plain mathematics fix.

Each ``pin_*`` function takes the path of an oracle build and raises
AssertionError when the oracle disagrees with the independent expectation.
They are run against the real oracle (tests/test_oracle_pins.py) and against
copies of the oracle with planted mistakes, each of which must fail at least one
pin.

None of these checks calls back into the oracle's own arithmetic to produce
the expected value: traversals are enumerated with exact rational arithmetic,
distances and weights come from closed forms of the head-on geometry, and
binary16 rounding is compared with numpy's conversion.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction as Fr

import numpy as np

import oracle


# --------------------------------------------------------------------------
# exact segment / voxel enumeration
# --------------------------------------------------------------------------
def exact_voxel_sets(A, B):
    """Voxels met by the closed segment A->B (voxel units): (open-cube hits, closed-cube hits)."""
    A = [Fr(float(a)) for a in A]
    B = [Fr(float(b)) for b in B]
    D = [B[k] - A[k] for k in range(3)]
    lo = [math.floor(min(A[k], B[k])) - 1 for k in range(3)]
    hi = [math.floor(max(A[k], B[k])) + 1 for k in range(3)]
    opened, closed = set(), set()
    for g in itertools.product(*[range(lo[k], hi[k] + 1) for k in range(3)]):
        c_ok, o_ok = True, True
        Lc, Hc = Fr(0), Fr(1)
        Lo, Ho = None, None
        for k in range(3):
            if D[k] == 0:
                if not (g[k] <= A[k] <= g[k] + 1):
                    c_ok = False
                if not (g[k] < A[k] < g[k] + 1):
                    o_ok = False
            else:
                t1 = (g[k] - A[k]) / D[k]
                t2 = (g[k] + 1 - A[k]) / D[k]
                tl, th = min(t1, t2), max(t1, t2)
                Lc, Hc = max(Lc, tl), min(Hc, th)
                Lo = tl if Lo is None else max(Lo, tl)
                Ho = th if Ho is None else min(Ho, th)
        if c_ok and Lc <= Hc:
            closed.add(g)
        if o_ok and (Lo is None or (Lo < Ho and Lo < 1 and Ho > 0)):
            opened.add(g)
    return opened, closed


def check_path_shape(path, A, B):
    """Length, end points and 6-connectivity of a traversal."""
    ga = tuple(int(math.floor(float(a))) for a in A)
    gb = tuple(int(math.floor(float(b))) for b in B)
    assert len(path) == sum(abs(gb[k] - ga[k]) for k in range(3)) + 1, "traversal length"
    assert tuple(path[0]) == ga and tuple(path[-1]) == gb, "traversal end points"
    for i in range(1, len(path)):
        diff = np.abs(np.asarray(path[i]) - np.asarray(path[i - 1]))
        assert diff.sum() == 1, "traversal is not 6-connected"


def crossing_params(path, A, B):
    """Exact segment parameter at which each step of the path crosses a voxel face."""
    A = [Fr(float(a)) for a in A]
    B = [Fr(float(b)) for b in B]
    out = []
    for i in range(1, len(path)):
        k = int(np.nonzero(np.asarray(path[i]) - np.asarray(path[i - 1]))[0][0])
        step = int(path[i][k] - path[i - 1][k])
        face = path[i - 1][k] + (1 if step > 0 else 0)
        out.append(((face - A[k]) / (B[k] - A[k]), k))
    return out


def pin_dda_dyadic(lib_path=None, n=400, seed=11):
    """On inputs where binary32 arithmetic is exact, the traversal is exactly the set of
    voxels the segment passes through, steps in order of the face-crossing parameter,
    and on exact ties steps the lowest axis first."""
    rng = np.random.default_rng(seed)
    ties = 0
    for it in range(n):
        A = rng.integers(-48, 48, size=3).astype(np.float64) / 16.0
        D = np.array([rng.choice([-1, 1]) * 2.0 ** rng.integers(-1, 3) if rng.random() < 0.85 else 0.0
                      for _ in range(3)])
        if it % 5 == 0:                      # force corner and edge hits
            A = np.floor(A) + 0.5
            D = np.array([2.0, 2.0, 2.0 if it % 10 == 0 else 0.0]) * rng.choice([-1, 1], size=3)
        B = A + D
        path = [tuple(map(int, g)) for g in oracle.dda(A, B, lib_path)]
        check_path_shape(path, A, B)
        opened, closed = exact_voxel_sets(A, B)
        assert set(path) <= closed, f"visited a voxel the segment misses: {A} {B}"
        assert opened <= set(path), f"skipped a voxel the segment crosses: {A} {B}"
        cp = crossing_params(path, A, B)
        for (t0, k0), (t1, k1) in zip(cp, cp[1:]):
            assert t0 <= t1, "steps out of crossing order"
            if t0 == t1:
                ties += 1
                assert k0 < k1, "tie not broken to the lowest axis"
    assert ties > 20


def pin_dda_random(lib_path=None, n=1500, seed=12):
    """On random binary32 segments the traversal covers every voxel the segment passes
    through the interior of and visits only voxels the segment touches, except where two
    face crossings are closer than binary32 can resolve."""
    rng = np.random.default_rng(seed)
    exceptions = 0
    for _ in range(n):
        A = rng.uniform(-3, 3, size=3).astype(np.float32)
        B = (A + rng.uniform(-4, 4, size=3)).astype(np.float32)
        path = [tuple(map(int, g)) for g in oracle.dda(A, B, lib_path)]
        check_path_shape(path, A, B)
        opened, closed = exact_voxel_sets(A, B)
        if set(path) <= closed and opened <= set(path):
            continue
        exceptions += 1
        # an exception must come from two nearly equal crossing parameters
        ts = sorted(float(t) for t, _ in crossing_params(path, A, B))
        gaps = [b - a for a, b in zip(ts, ts[1:])]
        assert gaps and min(gaps) < 1e-5, f"traversal error not explained by a near tie: {A} {B}"
    assert exceptions <= n // 100


# --------------------------------------------------------------------------
# head-on plane (closed forms)
# --------------------------------------------------------------------------
V = 0.125          # powers of two keep every binary32 operation exact
DELTA = 3 * V


def _axis_pose(axis, sign):
    """Pose whose sensor z axis points along world axis `axis` with `sign`; sensor origin at a
    voxel centre.  Entries are 0/+-1 so the transform is exact."""
    R = np.zeros((3, 3))
    z = np.zeros(3)
    z[axis] = sign
    other = [(axis + 1) % 3, (axis + 2) % 3]
    x = np.zeros(3)
    x[other[0]] = 1.0
    y = np.cross(z, x)
    R[:, 0], R[:, 1], R[:, 2] = x, y, z
    T = np.zeros((3, 4), np.float32)
    T[:, :3] = R
    T[:, 3] = [0.0625 + 0.25, 0.0625 - 0.5, 0.0625 + 0.125]   # voxel centres at v = 0.125
    return T


def head_on_expectation(Z, axis, sign, weighting, frames, pose, full_ray=False):
    """Touched voxels, D and W after `frames` identical frames of one ray along the sensor
    z axis hitting a plane at depth Z (Eqs. 1-5 evaluated on the axis).  full_ray: the ray
    updates every voxel from the sensor on, not only the truncation band."""
    s = pose[:, 3].astype(np.float64)
    p = s.copy()
    p[axis] += sign * Z
    lo_t, hi_t = (0.0 if full_ray else max(Z - DELTA, 0.0)), Z + DELTA
    a, b = s[axis] + sign * lo_t, s[axis] + sign * hi_t
    ga, gb = math.floor(a / V), math.floor(b / V)
    cols = range(min(ga, gb), max(ga, gb) + 1)
    out = {}
    base = [math.floor(s[k] / V) for k in range(3)]
    for g in cols:
        vox = list(base)
        vox[axis] = g
        xc = (g + 0.5) * V
        d = sign * (p[axis] - xc)              # on the axis |p - x| = |d| and the sign is the dot
        if weighting == "const":
            w = 1.0
        else:
            f = 1.0 if d > -V else ((d + DELTA) / (DELTA - V) if d > -DELTA else 0.0)
            w = f / (Z * Z)
        dc = max(-DELTA, min(DELTA, d))
        out[tuple(vox)] = (dc, frames * w)
    return out


def _export_dict(m):
    coords, D, W = m.export()[:3]
    res = {}
    for b in range(coords.shape[0]):
        for l in np.nonzero(W[b] > 0)[0]:
            g = (16 * coords[b, 0] + (l & 15), 16 * coords[b, 1] + ((l >> 4) & 15),
                 16 * coords[b, 2] + (l >> 8))
            res[tuple(int(x) for x in g)] = (D[b, l], W[b, l])
    return res, coords


def pin_head_on_plane(lib_path=None):
    """One ray along each of the six axis directions to a plane at dyadic depth, repeated
    over several frames: touched column, D = clamped signed distance, W = frames x weight."""
    for axis, sign, weighting, Z, frames in [
            (0, 1, "const", 1.3125, 3), (0, -1, "const", 0.9375, 2), (1, 1, "quad", 2.0625, 3),
            (1, -1, "quad", 1.5, 1), (2, 1, "quad", 1.25, 4), (2, -1, "const", 3.0, 2),
            (2, 1, "const", 0.25, 1)]:
        pose = _axis_pose(axis, sign)
        m = oracle.OracleMap(V, DELTA, weighting=weighting, merge="simple", w_max=1e30,
                             max_range=10.0, z_min=0.1, lib_path=lib_path)
        pt = np.array([[0.0, 0.0, Z]], np.float32)
        for _ in range(frames):
            st = m.integrate(pt, pose)
        exp = head_on_expectation(Z, axis, sign, weighting, frames, pose)
        tc, tn = m.last_touches()
        assert {tuple(map(int, c)) for c in tc} == set(exp), "touched column"
        assert np.all(tn == 1)
        assert st["touches"] == len(exp)
        got, coords = _export_dict(m)
        for g, (dc, W) in exp.items():
            if W == 0:
                assert g not in got
                continue
            assert abs(got[g][0] - dc) <= 1e-12, f"D at {g}: {got[g][0]} vs {dc}"
            assert abs(got[g][1] - W) <= 1e-12 * max(1.0, W), f"W at {g}: {got[g][1]} vs {W}"
        blocks = {tuple(int(x) // 16 if int(x) >= 0 else -((-int(x) + 15) // 16) for x in g) for g in exp}
        assert {tuple(map(int, c)) for c in coords} == blocks, "allocated blocks"
        m.close()


def pin_full_ray_head_on(lib_path=None):
    """Raycasting over the whole ray (Sec. IV-B: every voxel from the sensor to delta behind the
    point): on the head-on axis the touched column runs from the sensor's voxel to delta behind
    the plane; the free space in front of the band holds D = +delta (the clamped distance) and
    the full weight of every frame."""
    for axis, sign, weighting, Z, frames in [(0, 1, "const", 1.3125, 2), (2, -1, "quad", 2.0625, 3),
                                             (1, 1, "quad", 0.25, 1)]:
        pose = _axis_pose(axis, sign)
        m = oracle.OracleMap(V, DELTA, weighting=weighting, merge="simple", w_max=1e30,
                             max_range=10.0, z_min=0.1, full_ray=True, lib_path=lib_path)
        pt = np.array([[0.0, 0.0, Z]], np.float32)
        for _ in range(frames):
            st = m.integrate(pt, pose)
        exp = head_on_expectation(Z, axis, sign, weighting, frames, pose, full_ray=True)
        band = head_on_expectation(Z, axis, sign, weighting, frames, pose)
        assert len(exp) > len(band) or Z <= DELTA
        tc, tn = m.last_touches()
        assert {tuple(map(int, c)) for c in tc} == set(exp), "touched column"
        assert np.all(tn == 1) and st["touches"] == len(exp)
        got, _ = _export_dict(m)
        free = 0
        for g, (dc, W) in exp.items():
            if W == 0:
                assert g not in got
                continue
            assert abs(got[g][0] - dc) <= 1e-12 and abs(got[g][1] - W) <= 1e-12 * max(1.0, W), g
            free += dc == DELTA
        assert free >= int((Z - DELTA) / V) - 1, "free space in front of the band"
        m.close()


def _stair_frame(Z, W=16, H=16, f=8.0):
    """An organised frame whose pixel (i, j) sees depth z_ij = Z + ((i + 2 j) mod 5) / 32 along
    ((i + 1/2 - W/2) / f, (j + 1/2 - H/2) / f, 1) (exact in binary32 for dyadic Z): a depth that
    changes from pixel to pixel, so that the pixel a voxel projects to matters."""
    i, j = np.meshgrid(np.arange(W), np.arange(H))
    z = Z + ((i.ravel() + 2 * j.ravel()) % 5) / 32.0
    d = np.stack([(i.ravel() + 0.5 - W / 2) / f, (j.ravel() + 0.5 - H / 2) / f, np.ones(W * H)], axis=1)
    return (d * z[:, None]).astype(np.float32), (f, f, W / 2, H / 2)


def pin_projective_plane(lib_path=None):
    """Projection mapping (Sec. IV-B) of a depth image seen head-on, worked in exact arithmetic:
    the blocks are the ones raycasting allocates for the same frame; every voxel of them that
    projects into the image (camera point c = R^T (x - t), pixel (floor(f c_x / c_z + W/2),
    floor(f c_y / c_z + H/2))) with a depth difference z_pixel - c_z above -delta takes
    D = clamp(z_pixel - c_z, +-delta) and the frame's weight (1, or 1/z_pixel^2 with the Eq. (5)
    drop-off); the rest is untouched.  Two frames: W doubles, D stays."""
    for axis, sign, weighting, Z, frames in [(0, 1, "const", 1.0, 2), (2, 1, "quad", 1.25, 1),
                                             (1, -1, "const", 0.75, 1)]:
        pose = _axis_pose(axis, sign)
        pts, intr = _stair_frame(Z)
        zpix = [Fr(float(z)) for z in pts[:, 2]]
        m = oracle.OracleMap(V, DELTA, weighting=weighting, merge="simple", w_max=1e30,
                             max_range=10.0, z_min=0.1, lib_path=lib_path)
        ray = oracle.OracleMap(V, DELTA, weighting=weighting, merge="simple", w_max=1e30,
                               max_range=10.0, z_min=0.1, lib_path=lib_path)
        for _ in range(frames):
            st = m.integrate_projective(pts, pose, 16, intr)
        ray.integrate(pts, pose)
        coords = m.export()[0]
        assert np.array_equal(coords, ray.export()[0]), "blocks: the ones raycasting allocates"
        R = [[Fr(float(pose[r, c])) for c in range(3)] for r in range(3)]
        t = [Fr(float(pose[r, 3])) for r in range(3)]
        got, _ = _export_dict(m)
        seen = 0
        for b in coords.tolist():
            for l in range(4096):
                g = (16 * b[0] + (l & 15), 16 * b[1] + ((l >> 4) & 15), 16 * b[2] + (l >> 8))
                e = [(Fr(g[k]) + Fr(1, 2)) * Fr(V) - t[k] for k in range(3)]
                c = [sum(R[r][k] * e[r] for r in range(3)) for k in range(3)]
                hit = c[2] > 0
                if hit:
                    u = Fr(intr[0]) * c[0] / c[2] + Fr(intr[2])
                    vv = Fr(intr[1]) * c[1] / c[2] + Fr(intr[3])
                    hit = 0 <= u < 16 and 0 <= vv < 16
                if hit:
                    zp = zpix[math.floor(u) + 16 * math.floor(vv)]
                    hit = zp - c[2] > -Fr(DELTA)
                if not hit:
                    assert g not in got, f"{g} updated outside the image or behind the band"
                    continue
                d = zp - c[2]
                dc = max(-Fr(DELTA), min(Fr(DELTA), d))
                w = Fr(1)
                if weighting == "quad":
                    fd = 1 if d > -Fr(V) else ((d + Fr(DELTA)) / (Fr(DELTA) - Fr(V)) if d > -Fr(DELTA) else 0)
                    w = Fr(1) / (zp * zp) * fd
                if w == 0:
                    assert g not in got
                    continue
                seen += 1
                assert g in got, f"{g} not updated"
                assert abs(got[g][0] - float(dc)) <= 1e-12, f"D at {g}: {got[g][0]} vs {float(dc)}"
                assert abs(got[g][1] - float(frames * w)) <= 1e-12 * float(frames * w), f"W at {g}"
        assert seen == len(got) and seen > 100
        assert st["touches"] >= seen
        m.close(); ray.close()


def _rgb(r, g, b):
    return np.uint32(r | (g << 8) | (b << 16))


def _round_half_even(x: Fr) -> int:
    return round(x)          # Python rounds fractions half to even


def pin_color_sequence(lib_path=None):
    """Colour (Sec. IV-B): each voxel keeps the running mean of its rays' colours with the
    weights of Eq. (3), blended with the weight it held before the frame and stored as 8-bit
    channels (nearest, ties to even).  One ray per frame on the head-on axis, the same depth
    every frame (so each voxel's weight is the same every frame and cancels): C_1 = c_1,
    C_(k+1) = round((k C_k + c_(k+1)) / (k + 1)); 15.5 rounds to 16 and 16.5 to 16."""
    cols = [(10, 200, 7), (21, 100, 8), (23, 0, 255), (2, 33, 254)]
    for weighting in ("const", "quad"):
        pose = _axis_pose(2, 1)
        m = oracle.OracleMap(V, DELTA, weighting=weighting, merge="simple", w_max=1e30,
                             max_range=10.0, color=True, lib_path=lib_path)
        C = None
        for k, c in enumerate(cols):
            m.integrate(np.array([[0.0, 0.0, 1.3125]], np.float32), pose, colors=np.array([_rgb(*c)]))
            C = list(c) if C is None else [_round_half_even((k * Fr(C[i]) + c[i]) / (k + 1)) for i in range(3)]
            if k == 1:
                assert C[0] == 16, "15.5 rounds to the even 16"
            if k == 2:
                assert C[0] == 18
        exp = head_on_expectation(1.3125, 2, 1, weighting, len(cols), pose)
        coords = m.export()[0]
        rgb = m.export_colors()
        got = {}
        for b in range(coords.shape[0]):
            for l in range(4096):
                g = (16 * coords[b, 0] + (l & 15), 16 * coords[b, 1] + ((l >> 4) & 15), 16 * coords[b, 2] + (l >> 8))
                got[g] = int(rgb[b, l])
        want = int(_rgb(*C))
        for g, (_, W) in exp.items():
            assert got[g] == (want if W > 0 else 0), f"colour at {g}: {got[g]:06x} vs {want:06x}"
        m.close()


def pin_color_group_mean(lib_path=None):
    """Grouped raycasting takes the weighted mean of the points' colours in a voxel (Sec. IV-B),
    rounded to 8 bits (nearest, ties to even): points at one depth (equal weights) in one voxel;
    every voxel the group's ray updates first takes exactly that colour."""
    pose = _axis_pose(2, 1)
    xs = np.array([-0.0625, -0.03125, 0.0, 0.03125], np.float32)   # one voxel (v = 0.125)
    for weighting, cols, mean in [("const", [(10, 0, 1), (23, 4, 1)], (16, 2, 1)),
                                  ("quad", [(10, 9, 0), (23, 9, 0), (12, 9, 255), (100, 9, 255)], (36, 9, 128)),
                                  ("const", [(1, 2, 3)], (1, 2, 3))]:
        m = oracle.OracleMap(V, DELTA, weighting=weighting, merge="grouped", w_max=1e30,
                             max_range=10.0, color=True, lib_path=lib_path)
        n = len(cols)
        pts = np.stack([xs[:n], np.zeros(n, np.float32), np.full(n, 1.3125, np.float32)], axis=1)
        st = m.integrate(pts, pose, colors=np.array([_rgb(*c) for c in cols]))
        assert st["rays"] == 1
        rgb = m.export_colors()
        W = m.export()[2]
        assert np.all(rgb[W > 0] == _rgb(*mean)) and np.all(rgb[W == 0] == 0)
        m.close()


def pin_dropoff_values(lib_path=None):
    """Eq. (5) at the distances where it changes form: d > -eps full weight, d = -(eps+delta)/2
    half weight, d <= -delta zero weight (W stays 0 while the block is still allocated)."""
    pose = _axis_pose(2, 1)
    Z = 1.0                                 # end point at a voxel centre: d in multiples of v
    m = oracle.OracleMap(V, DELTA, weighting="quad", merge="simple", w_max=1e30,
                         max_range=10.0, lib_path=lib_path)
    m.integrate(np.array([[0.0, 0.0, Z]], np.float32), pose)
    got, _ = _export_dict(m)
    s = pose[:, 3].astype(np.float64)
    ix, iy = math.floor(s[0] / V), math.floor(s[1] / V)
    pz = s[2] + Z
    om = 1.0 / (Z * Z)
    for dv, f in [(2, 1.0), (1, 1.0), (0, 1.0), (-1, 1.0), (-2, 0.5), (-3, 0.0)]:
        g = (ix, iy, math.floor((pz - dv * V) / V))
        if f == 0.0:
            assert g not in got, "weight behind -delta must be 0"
        else:
            assert abs(got[g][1] - om * f) <= 1e-12, f"Eq. 5 at d={dv}v"
            assert abs(got[g][0] - dv * V) <= 1e-12



def _identity_pose():
    T = np.zeros((3, 4), np.float32)
    T[:, :3] = np.eye(3)
    T[:, 3] = [0.0625 + 0.25, 0.0625 - 0.5, 0.0625 + 0.125]   # a voxel centre at v = 0.125
    return T


def _exact_dist(p, s, g, mode):
    """Eq. (1) (mode "eq1") or the projective distance along the ray (mode "ray") of voxel g's
    centre, from exact rational p, s; returns (d as float, exact dot product)."""
    x = [(Fr(int(gk)) + Fr(1, 2)) * Fr(V) for gk in g]
    f = [p[k] - x[k] for k in range(3)]
    e = [p[k] - s[k] for k in range(3)]
    dot = sum(f[k] * e[k] for k in range(3))
    if mode == "ray":
        return float(dot) / math.sqrt(float(sum(ek * ek for ek in e))), dot
    mag = math.sqrt(float(sum(fk * fk for fk in f)))
    return (mag if dot > 0 else (-mag if dot < 0 else 0.0)), dot


def pin_along_ray_off_axis(lib_path=None):
    """Oblique rays whose band passes beside voxel centres: under the projective reading (Sec. I,
    the distance along the sensor ray) d = (p - x).(p - s) / |p - s|, under Eq. (1)
    d = |p - x| sign((p - x).(p - s)); after one frame D = clamp(d, +-delta) and W = f(d) / z^2.
    The inputs are dyadic, so p and s are exact and the ray length is irrational; the two
    readings differ by a large fraction of a voxel on most of the band's voxels."""
    pose = _identity_pose()
    s = [Fr(float(c)) for c in pose[:, 3]]
    differ = 0
    for q in ([0.75, 0.5, 1.3125], [-0.625, 0.375, 1.0625], [0.3125, -0.8125, 0.875]):
        q32 = np.array([q], np.float32)
        p = [s[k] + Fr(q[k]) for k in range(3)]       # identity rotation: exact in binary32
        om = 1.0 / (q[2] * q[2])
        for mode in ("ray", "eq1"):
            for weighting in ("const", "quad"):
                m = oracle.OracleMap(V, DELTA, weighting=weighting, merge="simple", w_max=1e30,
                                     max_range=10.0, dist=mode, lib_path=lib_path)
                m.integrate(q32, pose)
                tc, _ = m.last_touches()
                got, _ = _export_dict(m)
                checked = 0
                for g in map(tuple, tc.tolist()):
                    d, dot = _exact_dist(p, s, g, mode)
                    if mode == "eq1" and abs(dot) < 1e-9:
                        continue              # the sign is decided in binary32 there
                    if weighting == "const" and mode == "ray":
                        d1, _ = _exact_dist(p, s, g, "eq1")
                        differ += abs(d1 - d) > 0.05 * V
                    f = 1.0 if (weighting == "const" or d > -V) else (
                        (d + DELTA) / (DELTA - V) if d > -DELTA else 0.0)
                    w = f * (1.0 if weighting == "const" else om)
                    if w == 0.0:
                        assert g not in got, f"{mode}: weight behind -delta must be 0 at {g}"
                        continue
                    dc = max(-DELTA, min(DELTA, d))
                    assert abs(got[g][0] - dc) <= 1e-12, f"{mode} D at {g}: {got[g][0]} vs {dc}"
                    assert abs(got[g][1] - w) <= 1e-12 * w, f"{mode} W at {g}: {got[g][1]} vs {w}"
                    checked += 1
                assert checked >= 5
                m.close()
    assert differ >= 6, "geometry does not separate the two distance readings"


def _f16(x):
    """Binary16 rounding by numpy's conversion (round to nearest even)."""
    return float(np.float16(x))


def pin_binary16_sequence(lib_path=None):
    """Binary16 storage: after every frame D / delta and W are rounded to binary16, W after the
    Eq. (4) cap.  A head-on sequence worked in exact arithmetic with numpy's float16 rounding:
    frames of repeated points (constant weighting, so each frame's sums are exact), W stalling at
    2048 (2049 is not a binary16 number and rounds to even), D stalling where a frame moves it by
    less than half a binary16 step, and W_max = 2999 (not a binary16 number) reached inside a frame,
    where the cap comes first and the rounding then gives 3000."""
    pose = _axis_pose(2, 1)
    sz = Fr(float(pose[2, 3]))
    wmax = 2999.0
    m = oracle.OracleMap(V, DELTA, weighting="const", merge="simple", w_max=wmax,
                         max_range=10.0, storage="f16", lib_path=lib_path)
    frames = [(3, 1.3125), (1, 1.34375), (2, 1.28125), (2041, 1.3125), (1, 1.3125),
              (1, 1.375), (1000, 1.25), (1, 1.3125)]
    state = {}                    # voxel z index -> (D / delta, W) as stored (binary16 values)
    ix, iy = math.floor(float(pose[0, 3]) / V), math.floor(float(pose[1, 3]) / V)
    stalled_d = 0
    for f, (n, Z) in enumerate(frames):
        pz = sz + Fr(Z)
        lo, hi = math.floor((pz - Fr(DELTA)) / Fr(V)), math.floor((pz + Fr(DELTA)) / Fr(V))
        m.integrate(np.repeat(np.array([[0.0, 0.0, Z]], np.float32), n, axis=0), pose)
        for gz in range(lo, hi + 1):
            d = pz - (Fr(gz) + Fr(1, 2)) * Fr(V)
            dc = max(Fr(-DELTA), min(Fr(DELTA), d))
            D0, W0 = state.get(gz, (0.0, 0.0))
            exact = (Fr(W0) * Fr(D0) + n * dc / Fr(DELTA)) / (Fr(W0) + n)
            D1 = _f16(float(exact))
            W1 = _f16(min(W0 + n, wmax))
            if f == 5 and D1 == D0 and exact != Fr(D0):
                stalled_d += 1
            state[gz] = (D1, W1)
        centre = state[math.floor(pz / Fr(V))]
        if f == 5:
            assert centre[1] == 2048.0, "W must stall at 2048 (2049 rounds to even)"
        if f >= 6:
            assert centre[1] == 3000.0, "W capped at 2999, then rounded to binary16"
    assert stalled_d >= 1, "sequence does not exercise a stalled D"
    got, _ = _export_dict(m)
    for gz, (Dq, Wq) in state.items():
        g = (ix, iy, gz)
        assert got[g][1] == Wq, f"W at {g}: {got[g][1]} vs {Wq}"
        assert got[g][0] == Dq * DELTA, f"D at {g}: {got[g][0] / DELTA} vs {Dq} (units of delta)"
    m.close()

    # 1/z^2 weights (not binary16 numbers) on the Eq. (5) ramp, one ray per frame
    m = oracle.OracleMap(V, DELTA, weighting="quad", merge="simple", w_max=1e4,
                         max_range=10.0, storage="f16", lib_path=lib_path)
    state = {}
    for Z in (1.25, 1.1875, 1.3125, 1.25, 1.21875):
        pz = float(sz) + Z
        m.integrate(np.array([[0.0, 0.0, Z]], np.float32), pose)
        om = 1.0 / (Z * Z)
        for gz in range(math.floor((pz - DELTA) / V), math.floor((pz + DELTA) / V) + 1):
            d = pz - (gz + 0.5) * V
            fd = 1.0 if d > -V else ((d + DELTA) / (DELTA - V) if d > -DELTA else 0.0)
            w = om * fd
            if w == 0.0:
                continue
            D0, W0 = state.get(gz, (0.0, 0.0))
            dc = max(-DELTA, min(DELTA, d))
            state[gz] = (_f16((W0 * D0 + w * (dc / DELTA)) / (W0 + w)), _f16(min(W0 + w, 1e4)))
    got, _ = _export_dict(m)
    for gz, (Dq, Wq) in state.items():
        g = (ix, iy, gz)
        assert got[g][1] == Wq and got[g][0] == Dq * DELTA, f"quad binary16 at {g}"
    m.close()


def _s16(x):
    """Nearest multiple of 1/32767 in [-1, 1], ties to even (Python's round is half-even on
    fractions), as an exact fraction."""
    i = round(Fr(x) * 32767)
    return Fr(max(-32767, min(32767, i)), 32767)


def pin_s16_sequence(lib_path=None):
    """16-bit fixed-point distance storage: after every frame D / delta is rounded to the nearest
    multiple of 1/32767 (ties to even) and W to binary16, W after the Eq. (4) cap.  The head-on
    sequence of the binary16 pin, worked in exact rational arithmetic: W stalls at 2048 as in
    binary16, D keeps moving where binary16 stalls (its step is 1/32767 of delta everywhere, where
    binary16's is 2^-11 of delta near |D| = delta), D stalls where a frame moves it by less than
    half a step, the clamped D = +-delta is exact, and W_max = 2999 is capped before rounding."""
    pose = _axis_pose(2, 1)
    sz = Fr(float(pose[2, 3]))
    wmax = 2999.0
    m = oracle.OracleMap(V, DELTA, weighting="const", merge="simple", w_max=wmax,
                         max_range=10.0, storage="s16", lib_path=lib_path)
    frames = [(3, 1.3125), (1, 1.34375), (2, 1.28125), (2041, 1.3125), (1, 1.3125),
              (1, 1.375), (1, 1.34375), (1000, 1.25), (1, 1.3125)]
    state = {}                 # voxel z index -> (D / delta exact fraction, W float) as stored
    ix, iy = math.floor(float(pose[0, 3]) / V), math.floor(float(pose[1, 3]) / V)
    moved_where_f16_stalls = stalled = 0
    for f, (n, Z) in enumerate(frames):
        pz = sz + Fr(Z)
        lo, hi = math.floor((pz - Fr(DELTA)) / Fr(V)), math.floor((pz + Fr(DELTA)) / Fr(V))
        m.integrate(np.repeat(np.array([[0.0, 0.0, Z]], np.float32), n, axis=0), pose)
        for gz in range(lo, hi + 1):
            d = pz - (Fr(gz) + Fr(1, 2)) * Fr(V)
            dc = max(Fr(-DELTA), min(Fr(DELTA), d))
            D0, W0 = state.get(gz, (Fr(0), 0.0))
            exact = (Fr(W0) * D0 + n * dc / Fr(DELTA)) / (Fr(W0) + n)
            D1 = _s16(exact)
            W1 = _f16(min(W0 + n, wmax))
            if f >= 5 and D1 != D0 and _f16(float(exact)) == _f16(float(D0)):
                moved_where_f16_stalls += 1
            if f >= 4 and D1 == D0 and exact != D0:
                stalled += 1
            state[gz] = (D1, W1)
        centre = state[math.floor(pz / Fr(V))]
        if f == 5:
            assert centre[1] == 2048.0, "W must stall at 2048 (2049 rounds to even)"
        if f >= 7:
            assert centre[1] == 3000.0, "W capped at 2999, then rounded to binary16"
    assert moved_where_f16_stalls >= 1, "sequence does not separate the two 16-bit forms"
    assert stalled >= 1, "sequence does not exercise a stalled D"
    assert any(Dq == 1 for Dq, _ in state.values()), "sequence has no clamped voxel"
    got, _ = _export_dict(m)
    for gz, (Dq, Wq) in state.items():
        g = (ix, iy, gz)
        assert got[g][1] == Wq, f"W at {g}: {got[g][1]} vs {Wq}"
        expect = (int(Dq * 32767) / 32767.0) * DELTA     # the binary64 the oracle exports
        assert got[g][0] == expect, f"D at {g}: {got[g][0] / DELTA} vs {Dq} (units of delta)"
    m.close()
    # rounding ties go to the even code, and the code saturates at +-32767
    for i in (0, 1, 2, 32765, -7):
        assert oracle.round_s16((i + 0.5) / 32767.0, lib_path) == (i + (i & 1)) / 32767.0, i
    assert oracle.round_s16(1.00001, lib_path) == 1.0 and oracle.round_s16(-1.5, lib_path) == -1.0


def pin_ramp_diagnostic(lib_path=None):
    """The ramp diagnostic of the oracle's export: per voxel, the summed point weight 1/z^2 of the
    rays that saw it on the Eq. (5) drop-off ramp, -delta < d <= -eps (on the head-on axis d is
    the signed distance to the plane).  It takes no part in D or W."""
    pose = _axis_pose(2, 1)
    sz = float(pose[2, 3])
    ix, iy = math.floor(float(pose[0, 3]) / V), math.floor(float(pose[1, 3]) / V)
    m = oracle.OracleMap(V, DELTA, weighting="quad", merge="simple", w_max=1e30,
                         max_range=10.0, lib_path=lib_path)
    expect = {}
    # end points at voxel centres (d = -eps and d = -delta exactly on the band) and between them
    for n, Z in ((1, 1.0), (2, 1.0625), (1, 1.5), (3, 0.96875)):
        m.integrate(np.repeat(np.array([[0.0, 0.0, Z]], np.float32), n, axis=0), pose)
        pz = sz + Z
        for gz in range(math.floor((pz - DELTA) / V), math.floor((pz + DELTA) / V) + 1):
            d = pz - (gz + 0.5) * V
            expect.setdefault(gz, 0.0)
            if -DELTA < d <= -V:
                expect[gz] += n / (Z * Z)
    coords, D, W, mass, ramp = m.export()
    seen = 0
    for b in range(coords.shape[0]):
        for l in range(4096):
            g = (16 * coords[b, 0] + (l & 15), 16 * coords[b, 1] + ((l >> 4) & 15),
                 16 * coords[b, 2] + (l >> 8))
            r = expect.get(int(g[2]), 0.0) if (g[0], g[1]) == (ix, iy) else 0.0
            assert abs(ramp[b, l] - r) <= 1e-12 * max(1.0, r), f"ramp weight at {g}: {ramp[b, l]} vs {r}"
            seen += r > 0
    assert seen >= 3
    m.close()

# --------------------------------------------------------------------------
# accumulation: weight sums, counts and D against exact enumeration
# --------------------------------------------------------------------------
def _rand_rays(rng, n, spread=0.6):
    pts = rng.uniform(-spread, spread, size=(n, 3))
    pts[:, 2] = rng.uniform(0.9, 1.6, size=n)
    return pts.astype(np.float32)


def world_point32(pose, q):
    """Binary32 world point ((R0 x + R1 y) + R2 z) + t of a sensor point, every operation rounded
    to binary32 (numpy float32 scalars), in the order the geometry tier fixes."""
    T = np.asarray(pose, np.float32).reshape(3, 4)
    x, y, z = (np.float32(c) for c in np.asarray(q, np.float32).reshape(3))
    out = np.zeros(3, np.float32)
    for k in range(3):
        out[k] = ((T[k, 0] * x + T[k, 1] * y) + T[k, 2] * z) + T[k, 3]
    return out


def pin_weight_sums(lib_path=None, seed=5):
    """W = sum of per-observation weights, D = weighted mean of clamped distances and the
    per-voxel ray counts, with the visited voxels enumerated exactly per ray."""
    rng = np.random.default_rng(seed)
    # map parameters are binary32; the expectation uses their exact values
    v, delta = float(np.float32(0.1)), float(np.float32(0.3))
    pose = np.zeros((3, 4), np.float32)
    pose[:, :3] = [[0, 0, 1], [-1, 0, 0], [0, -1, 0]]     # camera looking along +x
    pose[:, 3] = [0.013, 0.021, 0.037]
    for weighting in ("const", "quad"):
        pts = _rand_rays(rng, 60)
        m = oracle.OracleMap(v, delta, weighting=weighting, merge="simple", w_max=1e30,
                             max_range=5.0, z_min=0.1, lib_path=lib_path)
        m.integrate(pts, pose)
        s = pose[:, 3].astype(np.float64)
        acc = {}
        skipped = 0
        for q32 in pts:
            # the world point is the binary32 transform (fixed order, no fused multiply-add);
            # Eq. (1) is then evaluated exactly from it
            p = world_point32(pose, q32).astype(np.float64)
            q = q32.astype(np.float64)
            e = p - s
            r = np.linalg.norm(e)
            u = e / r
            a = (s + u * max(r - delta, 0.0)) / v
            b = (s + u * (r + delta)) / v
            opened, closed = exact_voxel_sets(a, b)
            if opened != closed or any(abs(x - round(x)) < 1e-4 for x in list(a) + list(b)):
                skipped += 1
                continue
            om = 1.0 if weighting == "const" else 1.0 / (q[2] * q[2])
            for g in closed:
                x = (np.asarray(g) + 0.5) * v
                d = np.linalg.norm(p - x) * np.sign(np.dot(p - x, p - s))
                f = 1.0 if (weighting == "const" or d > -v) else (
                    (d + delta) / (delta - v) if d > -delta else 0.0)
                sw, swd, n = acc.get(g, (0.0, 0.0, 0))
                acc[g] = (sw + om * f, swd + om * f * max(-delta, min(delta, d)), n + 1)
        assert skipped < 10
        tc, tn = m.last_touches()
        touches = {tuple(map(int, c)): int(k) for c, k in zip(tc, tn)}
        got, _ = _export_dict(m)
        checked = 0
        for g, (sw, swd, n) in acc.items():
            # voxels that a skipped ray also touched carry extra weight; compare the rest
            if touches.get(g) != n:
                continue
            checked += 1
            if sw == 0:
                assert g not in got
                continue
            assert abs(got[g][1] - sw) <= 1e-9 * sw, f"W {got[g][1]} vs {sw}"
            assert abs(got[g][0] - swd / sw) <= 1e-9, f"D {got[g][0]} vs {swd / sw}"
        assert checked > 0.8 * len(acc)
        m.close()


# --------------------------------------------------------------------------
# grouped raycasting
# --------------------------------------------------------------------------
def pin_group_mean(lib_path=None, seed=3):
    """The group's ray end point is the weighted mean of its points, to within the 2^-20 voxel
    fixed-point grid and binary32 rounding; a single point is kept exactly."""
    rng = np.random.default_rng(seed)
    v = np.float32(0.05)
    for weighting in ("const", "quad"):
        wbits = oracle.weight_bits(weighting, 0.1)
        for _ in range(200):
            n = int(rng.integers(1, 40))
            key = rng.integers(-200, 200, size=3)
            p = ((key + rng.uniform(0.01, 0.99, size=(n, 3))) * float(v)).astype(np.float32)
            keys = np.floor(p * (np.float32(1) / v)).astype(np.int64)
            p = p[np.all(keys == keys[0], axis=1)]
            if p.shape[0] == 0:
                continue
            z = rng.uniform(0.3, 5.0, size=p.shape[0]).astype(np.float32)
            w = np.ones_like(z) if weighting == "const" else (np.float32(1) / (z * z)).astype(np.float32)
            got = oracle.group_mean(p, w, float(v), wbits, lib_path)
            if p.shape[0] == 1:
                assert np.array_equal(got, p[0]), "single point must be kept exactly"
                continue
            W = sum(Fr(float(x)) for x in w)
            for k in range(3):
                exact = sum(Fr(float(wi)) * Fr(float(pi)) for wi, pi in zip(w, p[:, k])) / W
                err = abs(float(got[k]) - float(exact))
                tol = (2.0 ** -19 + 2.0 ** -20) * float(v) + 2 * np.spacing(np.float32(abs(exact)))
                assert err <= tol, f"group mean off by {err} (tol {tol})"


def pin_merged_singletons(lib_path=None, seed=8):
    """When every point is alone in its voxel, grouped raycasting equals per-point raycasting."""
    rng = np.random.default_rng(seed)
    pose = np.zeros((3, 4), np.float32)
    pose[:, :3] = np.eye(3)
    pose[:, 3] = [0.1, -0.2, 0.05]
    # points on a sparse lattice: at most one per 0.1 m voxel
    ij = np.stack(np.meshgrid(np.arange(-6, 7), np.arange(-5, 6), indexing="ij"), -1).reshape(-1, 2)
    pts = np.zeros((ij.shape[0], 3), np.float32)
    pts[:, 0] = ij[:, 0] * 0.31 + rng.uniform(-0.02, 0.02, ij.shape[0])
    pts[:, 1] = ij[:, 1] * 0.29 + rng.uniform(-0.02, 0.02, ij.shape[0])
    pts[:, 2] = rng.uniform(1.5, 2.5, ij.shape[0])
    for weighting in ("const", "quad"):
        a = oracle.OracleMap(0.1, 0.3, weighting=weighting, merge="simple", lib_path=lib_path)
        b = oracle.OracleMap(0.1, 0.3, weighting=weighting, merge="grouped", lib_path=lib_path)
        sa = a.integrate(pts, pose)
        sb = b.integrate(pts, pose)
        assert sa["rays"] == sb["rays"] == pts.shape[0]
        ca, Da, Wa = a.export()[:3]
        cb, Db, Wb = b.export()[:3]
        assert np.array_equal(ca, cb) and np.array_equal(Wa, Wb) and np.array_equal(Da, Db)
        a.close(); b.close()


def pin_identical_points(lib_path=None):
    """n identical points form one group whose ray carries n times the point weight."""
    pose = _axis_pose(2, 1)
    Z = 1.0 + 0.0625
    for weighting, n in (("const", 7), ("quad", 5)):
        one = oracle.OracleMap(V, DELTA, weighting=weighting, merge="simple", w_max=1e30,
                               max_range=10.0, lib_path=lib_path)
        grp = oracle.OracleMap(V, DELTA, weighting=weighting, merge="grouped", w_max=1e30,
                               max_range=10.0, lib_path=lib_path)
        pt = np.array([[0.0, 0.0, Z]], np.float32)
        one.integrate(pt, pose)
        st = grp.integrate(np.repeat(pt, n, axis=0), pose)
        assert st["rays"] == 1
        go, _ = _export_dict(one)
        gg, _ = _export_dict(grp)
        assert set(go) == set(gg)
        for g in go:
            assert abs(gg[g][1] - n * go[g][1]) <= 1e-12 * n * go[g][1]
            # the grouped end point sits on the 2^-20 voxel grid
            assert abs(gg[g][0] - go[g][0]) <= 2.0 ** -18 * V
        one.close(); grp.close()


# --------------------------------------------------------------------------
# merging over frames, limits and storage rounding
# --------------------------------------------------------------------------
def pin_running_average(lib_path=None):
    """Eq. (3)-(4) over frames: with a head-on ray at two depths the distance is the
    weight-averaged distance and the weight is capped at W_max."""
    pose = _axis_pose(2, 1)
    m = oracle.OracleMap(V, DELTA, weighting="const", merge="simple", w_max=5.0,
                         max_range=10.0, lib_path=lib_path)
    z1, z2 = 1.0625, 1.125            # second surface one half voxel further
    for _ in range(3):
        m.integrate(np.array([[0.0, 0.0, z1]], np.float32), pose)
    m.integrate(np.array([[0.0, 0.0, z2]], np.float32), pose)
    got, _ = _export_dict(m)
    s = pose[:, 3].astype(np.float64)
    g = (math.floor(s[0] / V), math.floor(s[1] / V), math.floor((s[2] + z1) / V))
    xc = (g[2] + 0.5) * V
    d1, d2 = (s[2] + z1) - xc, (s[2] + z2) - xc
    assert abs(got[g][0] - (3 * d1 + d2) / 4) <= 1e-12
    assert got[g][1] == 4.0
    for _ in range(3):
        m.integrate(np.array([[0.0, 0.0, z1]], np.float32), pose)
    got, _ = _export_dict(m)
    assert got[g][1] == 5.0, "weight must saturate at W_max"
    m.close()


def pin_validity(lib_path=None):
    """Invalid points (NaN, zero range, beyond maximum range, behind the camera under 1/z^2)
    produce no ray."""
    pose = _axis_pose(2, 1)
    pts = np.array([[np.nan, 0, 1], [0, 0, 0], [0, 0, 5.5], [0, 3, 4.5], [0.1, 0.1, -1.0],
                    [0, 0, 1.0]], np.float32)
    m = oracle.OracleMap(0.1, 0.3, weighting="const", merge="simple", max_range=5.0,
                         lib_path=lib_path)
    st = m.integrate(pts, pose)
    assert st["valid"] == 2 and st["invalid"] == 4      # the -z point is valid for const weighting
    mq = oracle.OracleMap(0.1, 0.3, weighting="quad", merge="simple", max_range=5.0,
                          lib_path=lib_path)
    st = mq.integrate(pts, pose)
    assert st["valid"] == 1 and st["rays"] == 1
    m.close(); mq.close()


def pin_round_half(lib_path=None, seed=4):
    """Binary16 storage rounding agrees with numpy's float16 conversion (saturating at 65504)."""
    rng = np.random.default_rng(seed)
    xs = np.concatenate([rng.uniform(-1, 1, 3000), rng.uniform(0, 70000, 2000),
                         rng.uniform(-1e-4, 1e-4, 1000), [65504.0, 65519.0, 2049.0, 2051.0, 1e-8]])
    for x in xs:
        expect = float(np.float16(x)) if abs(x) < 65504 else math.copysign(65504.0, x)
        if math.isinf(expect):
            expect = math.copysign(65504.0, x)
        assert oracle.round_half(float(x), lib_path) == expect, x


def pin_permutation(lib_path=None, seed=9):
    """Shuffling the points of a frame does not change the integrated map."""
    import synth
    w = synth.config1()
    pts = w.frame(0)[::3]
    perm = np.random.default_rng(seed).permutation(pts.shape[0])
    for merge in ("simple", "grouped"):
        a = oracle.OracleMap(0.1, 0.3, weighting="quad", merge=merge, lib_path=lib_path)
        b = oracle.OracleMap(0.1, 0.3, weighting="quad", merge=merge, lib_path=lib_path)
        a.integrate(pts, w.poses[0])
        b.integrate(pts[perm], w.poses[0])
        ca, Da, Wa = a.export()[:3]
        cb, Db, Wb = b.export()[:3]
        assert np.array_equal(ca, cb)
        assert np.array_equal(Wa > 0, Wb > 0)
        ta, tb = a.last_touches(), b.last_touches()
        assert sorted(zip(map(tuple, ta[0]), ta[1])) == sorted(zip(map(tuple, tb[0]), tb[1]))
        # binary64 sums depend on the summation order in their last bits only
        assert np.allclose(Da, Db, rtol=0, atol=1e-12) and np.allclose(Wa, Wb, rtol=1e-10, atol=0)
        a.close(); b.close()


ALL_PINS = [pin_dda_dyadic, pin_dda_random, pin_head_on_plane, pin_full_ray_head_on, pin_projective_plane,
            pin_color_sequence, pin_color_group_mean, pin_dropoff_values,
            pin_along_ray_off_axis, pin_binary16_sequence, pin_s16_sequence, pin_ramp_diagnostic,
            pin_weight_sums, pin_group_mean, pin_merged_singletons, pin_identical_points,
            pin_running_average, pin_validity, pin_round_half, pin_permutation]
