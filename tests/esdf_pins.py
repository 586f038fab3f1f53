"""Pins of the ESDF oracle (Sec. V-A, Algorithm 1): each checks it against something other
than itself -- the closed-form quasi-Euclidean (26-neighbour chamfer) distance, a brute-force
multi-source field, the quasi-Euclidean error bound of Sec. V-B, and the invariants the paper
states (incremental updates reach the field a batch build reaches; FIFO and priority queues
reach the same field; unknown voxels neither take nor pass on distances)."""
from __future__ import annotations

import math

import numpy as np

from oracle import esdf

V = 0.125            # powers of two: sums of v, sqrt(2) v, sqrt(3) v stay close to exact
GAMMA = V            # one-voxel fixed band
DMAX = 4.0
TOL = 1e-12


def _grid(shape, origin=(0, 0, 0)):
    ax = [np.arange(o, o + s) for o, s in zip(origin, shape)]
    g = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.int32)


def _as_dict(exp):
    c, d, info = exp
    return {tuple(x): (dv, int(i)) for x, dv, i in zip(c.tolist(), d.tolist(), info.tolist())}


def _check_parents(field, v=V):
    """Every non-fixed voxel with a parent: the parent is an observed neighbour one step away and
    the voxel's distance is the parent's plus that step (same sign class)."""
    for g, (d, info) in field.items():
        p = (info >> 2) & 31
        fixed = bool(info & 2)
        neg = bool(info & 128)
        if fixed or p == esdf.NO_PARENT:
            continue
        o = esdf.OFFSETS[p]
        q = (g[0] + int(o[0]), g[1] + int(o[1]), g[2] + int(o[2]))
        assert q in field, f"parent of {g} is not an observed voxel"
        step = v * math.sqrt(int((o * o).sum()))
        dq = field[q][0]
        expect = min(dq - step, 0.0) if neg else max(dq + step, 0.0)
        assert abs(d - expect) <= TOL, f"{g}: {d} is not its parent's {dq} + step {step}"


def pin_point_source(lib_path=None):
    """One fixed voxel in a block of observed free space: every voxel's distance is the fixed
    value plus the closed-form 26-neighbour path length to it, capped at d_max."""
    d0 = 0.25 * V
    g = _grid((21, 21, 21), (-10, -10, -10))
    dT = np.where((g == 0).all(axis=1), d0, 3.0 * V)
    exp_d = np.minimum(d0 + esdf.chamfer(g, V), DMAX)
    exp_d[(g == 0).all(axis=1)] = d0
    for queue in ("fifo", "priority"):
        E = esdf.OracleESDF(V, GAMMA, DMAX, queue, lib_path=lib_path)
        E.update(g, dT, np.ones(len(g)))
        c, d, info = E.export()
        assert len(c) == len(g)
        order = np.lexsort((g[:, 2], g[:, 1], g[:, 0]))
        assert np.array_equal(c, g[order])
        assert np.abs(d - exp_d[order]).max() <= TOL, queue
        assert int(((info & 2) > 0).sum()) == 1
        _check_parents(_as_dict((c, d, info)))
        E.close()


def pin_quasi_euclidean_bound(lib_path=None):
    """Sec. V-B: quasi-Euclidean distance exceeds the Euclidean one by at most 1/sin(3 pi / 8) - 1
    = 8.24 % in a plane, the worst case at 22.5 degrees from an axis.  A point source in a
    one-voxel-thick slab: no voxel exceeds the bound, and the voxel (70, 29) (22.5 degrees to
    0.01 degrees) comes within 0.1 % of it."""
    g = _grid((75, 35, 1))
    src = (g == 0).all(axis=1)
    dT = np.where(src, 0.0, 3.0 * V)
    E = esdf.OracleESDF(V, GAMMA, 100.0, "priority", lib_path=lib_path)
    E.update(g, dT, np.ones(len(g)))
    c, d, _ = E.export()
    eu = V * np.sqrt((c.astype(np.float64) ** 2).sum(axis=1))
    far = eu >= 10 * V
    ratio = d[far] / eu[far]
    bound = 1.0 / math.sin(3.0 * math.pi / 8.0)
    assert ratio.max() <= bound + 1e-12
    assert ratio.min() >= 1.0 - 1e-12           # never shorter than the straight line
    k = np.nonzero((c == [70, 29, 0]).all(axis=1))[0][0]
    assert d[k] / eu[k] >= bound * (1 - 1e-3)
    E.close()


def pin_multi_source_brute_force(lib_path=None, seed=3):
    """Random fixed voxels, all with the same value c, in observed free space: the field is c
    plus the path length to the nearest of them (brute force over every voxel and source); with
    a shell of fixed voxels around a solid, the inside is the mirror image, -(c + path length)."""
    rng = np.random.default_rng(seed)
    g = _grid((14, 14, 14))
    c0 = 0.375 * V
    src = rng.random(len(g)) < 0.01
    src[0] = True
    dT = np.where(src, c0, 2.0 * V)
    exp = c0 + np.min(np.stack([esdf.chamfer(g - s, V) for s in g[src]], axis=1), axis=1)
    exp = np.minimum(exp, DMAX)
    exp[src] = c0
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0]))
    for queue in ("fifo", "priority"):
        E = esdf.OracleESDF(V, GAMMA, DMAX, queue, lib_path=lib_path)
        E.update(g, dT, np.ones(len(g)))
        _, d, info = E.export()
        assert np.abs(d - exp[order]).max() <= TOL, queue
        _check_parents(_as_dict(E.export()))
        E.close()
    # solid: the shell (boundary voxels of the grid) is fixed at -c0, the rest negative
    shell = (g == 0).any(axis=1) | (g == 13).any(axis=1)
    dT = np.where(shell, -c0, -2.0 * V)
    exp = -(c0 + np.min(np.stack([esdf.chamfer(g - s, V) for s in g[shell]], axis=1), axis=1))
    exp = np.maximum(exp, -DMAX)
    exp[shell] = -c0
    E = esdf.OracleESDF(V, GAMMA, DMAX, "fifo", lib_path=lib_path)
    E.update(g, dT, np.ones(len(g)))
    _, d, _ = E.export()
    assert np.abs(d - exp[order]).max() <= TOL
    E.close()


def pin_unknown_voxels_block(lib_path=None):
    """Unknown voxels (weight 0) take no distance and pass none on: a region sealed off from the
    fixed voxels by a wall of unknown voxels keeps d_max; a band gamma <= |d| is not fixed."""
    g = _grid((12, 12, 12))
    wall = g[:, 0] == 6
    dT = np.where((g == 0).all(axis=1), 0.0, 3.0 * V)
    dT[(g == [11, 11, 11]).all(axis=1)] = GAMMA          # exactly gamma: not fixed
    w = np.where(wall, 0.0, 1.0)
    E = esdf.OracleESDF(V, GAMMA, DMAX, "fifo", lib_path=lib_path)
    E.update(g, dT, w)
    c, d, info = E.export()
    assert len(c) == int((~wall).sum())
    beyond = c[:, 0] > 6
    assert np.all(d[beyond] == DMAX)
    near = c[:, 0] < 6
    assert np.all(d[near] < DMAX)
    assert int(((info & 2) > 0).sum()) == 1
    E.close()


def _random_field(rng, shape, p_fixed=0.06):
    g = _grid(shape)
    fixed = rng.random(len(g)) < p_fixed
    dT = np.where(fixed, rng.uniform(-0.9, 0.9, len(g)) * GAMMA, 0.0)
    # free space positive, a solid region negative
    solid = (g[:, 2] < 4)
    dT = np.where(fixed, dT, np.where(solid, -2.0 * V, 2.0 * V))
    return g, dT


def pin_incremental_equals_batch(lib_path=None, seed=5):
    """Algorithm 1 applied call by call reaches the field a single batch build of the final TSDF
    reaches: voxels arrive in two calls (new free voxels next to fixed ones seen before), then
    fixed voxels move (up, down, across zero) or leave the band, free voxels enter it, and free
    voxels change side."""
    rng = np.random.default_rng(seed)
    g, dT = _random_field(rng, (12, 12, 12))
    first = rng.random(len(g)) < 0.5
    dT2 = dT.copy()
    fixed = np.abs(dT) < GAMMA
    move = fixed & (rng.random(len(g)) < 0.4)
    dT2[move] = rng.uniform(-0.9, 0.9, int(move.sum())) * GAMMA
    leave = fixed & ~move & (rng.random(len(g)) < 0.3)
    dT2[leave] = np.where(g[leave, 2] < 4, -2.0 * V, 2.0 * V)
    enter = ~fixed & (rng.random(len(g)) < 0.03)
    dT2[enter] = rng.uniform(-0.9, 0.9, int(enter.sum())) * GAMMA
    flip = ~fixed & ~enter & (rng.random(len(g)) < 0.03)       # change side outside the band
    dT2[flip] = -dT[flip]
    ones = np.ones(len(g))
    for queue in ("fifo", "priority"):
        inc = esdf.OracleESDF(V, GAMMA, DMAX, queue, lib_path=lib_path)
        inc.update(g[first], dT[first], ones[first])
        inc.update(g[~first], dT[~first], ones[~first])
        bat = esdf.OracleESDF(V, GAMMA, DMAX, queue, lib_path=lib_path)
        bat.update(g, dT, ones)
        a, b = inc.export(), bat.export()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2] & 3, b[2] & 3)
        assert np.abs(a[1] - b[1]).max() <= TOL, f"{queue}: two calls differ from one"
        changed = move | leave | enter | flip
        inc.update(g[changed], dT2[changed], ones[changed])
        bat2 = esdf.OracleESDF(V, GAMMA, DMAX, queue, lib_path=lib_path)
        bat2.update(g, dT2, ones)
        a, b = inc.export(), bat2.export()
        assert np.array_equal(a[2] & 3, b[2] & 3)
        assert np.abs(a[1] - b[1]).max() <= TOL, f"{queue}: changed fixed voxels"
        _check_parents(_as_dict(a))
        for x in (inc, bat, bat2):
            x.close()


def pin_fifo_equals_priority(lib_path=None, seed=6):
    """The two queue orders the paper compares reach the same field on a random TSDF."""
    rng = np.random.default_rng(seed)
    g, dT = _random_field(rng, (16, 16, 10), p_fixed=0.04)
    out = []
    for queue in ("fifo", "priority"):
        E = esdf.OracleESDF(V, GAMMA, DMAX, queue, lib_path=lib_path)
        E.update(g, dT, np.ones(len(g)))
        out.append(E.export())
        E.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.abs(out[0][1] - out[1][1]).max() <= TOL


ALL_PINS = [pin_point_source, pin_quasi_euclidean_bound, pin_multi_source_brute_force,
            pin_unknown_voxels_block, pin_incremental_equals_batch, pin_fifo_equals_priority]
