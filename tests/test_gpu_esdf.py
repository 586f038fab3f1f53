"""The ESDF layer on the GPU (Sec. V-A, Algorithm 1) against the ESDF oracle.

Both sides read the same TSDF: the TSDF oracle integrates the frames, and its blocks (rounded to
binary32) are written into the GPU map and handed to the ESDF oracle.  The GPU runs the waves
level by level, the oracle with a FIFO and with a bucketed priority queue; they must agree on
which voxels are observed and fixed and on each voxel's side of the surface (bit-exact), on
the distances within the binary32 rounding of a path sum, and every GPU parent must be a valid
one (the distance is the parent's plus the step).

Distance bound: a distance is a band value plus at most n = d_max / v + 1 steps, each a binary32
addition rounded to 2^-24 of at most d_max + sqrt(3) v, with the step itself rounded to 2^-24 of
it: |d_GPU - d_oracle| <= 2 (n + 1) 2^-24 (d_max + 2 v)."""
import numpy as np
import pytest

from tests.common import log, oracle_map

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_03631_amd as vbx
    vbx.lib()
    return vbx


def tolerance(v, d_max):
    n = d_max / v + 1.0
    return 2.0 * (n + 1.0) * 2.0 ** -24 * (d_max + 2.0 * v)


def to_blocks(coords_blocks, c, d, info):
    """Oracle voxel lists -> per-block arrays in the GPU export's layout."""
    index = {tuple(b): i for i, b in enumerate(coords_blocks.tolist())}
    B = coords_blocks.shape[0]
    D = np.zeros((B, 4096))
    I = np.zeros((B, 4096), np.uint8)
    blk = np.floor_divide(c, 16)
    loc = c - 16 * blk
    l = loc[:, 0] + 16 * loc[:, 1] + 256 * loc[:, 2]
    rows = np.array([index[tuple(b)] for b in blk.tolist()], np.int64) if len(c) else np.zeros(0, np.int64)
    D[rows, l] = d
    I[rows, l] = info
    return D, I


def compare_esdf(gpu, orc, v, d_max, what=""):
    from oracle import esdf
    gc, gd, gi = gpu
    oD, oI = to_blocks(gc, *orc)
    obs_g, obs_o = (gi & 1) > 0, (oI & 1) > 0
    assert np.array_equal(obs_g, obs_o), f"{what}: observed sets differ ({obs_g.sum()} vs {obs_o.sum()})"
    assert np.array_equal(gi & 2, oI & 2), f"{what}: fixed bands differ"
    assert np.array_equal(gi & 128, oI & 128), f"{what}: sides differ"
    tol = tolerance(v, d_max)
    err = np.abs(gd.astype(np.float64) - oD)[obs_g]
    worst = float(err.max(initial=0.0))
    assert worst <= tol, f"{what}: |d_GPU - d_oracle| = {worst:.3g} m above {tol:.3g} m"
    # every GPU parent is a valid one
    B = gc.shape[0]
    index = {tuple(b): i for i, b in enumerate(gc.tolist())}
    par = (gi >> 2) & 31
    sel = obs_g & ((gi & 2) == 0) & (par != esdf.NO_PARENT)
    bb, ll = np.nonzero(sel)
    g = 16 * gc[bb] + np.stack([ll & 15, (ll >> 4) & 15, ll >> 8], axis=1)
    off = esdf.OFFSETS[par[bb, ll]]
    q = g + off
    qb = np.floor_divide(q, 16)
    ql = q - 16 * qb
    qrow = np.array([index.get(tuple(x), -1) for x in qb.tolist()], np.int64)
    assert np.all(qrow >= 0), f"{what}: a parent lies in an unallocated block"
    qidx = ql[:, 0] + 16 * ql[:, 1] + 256 * ql[:, 2]
    assert np.all((gi[qrow, qidx] & 1) > 0), f"{what}: a parent is unobserved"
    step = v * np.sqrt((off * off).sum(axis=1))
    dp = gd[qrow, qidx].astype(np.float64)
    neg = (gi[bb, ll] & 128) > 0
    expect = np.where(neg, np.minimum(dp - step, 0.0), np.maximum(dp + step, 0.0))
    perr = np.abs(gd[bb, ll] - expect)
    assert perr.max(initial=0.0) <= 2.0 ** -21 * (d_max + 2 * v), f"{what}: a parent does not give the distance"
    # voxels without a parent outside the band hold d_max (nothing reached them)
    lone = obs_g & ((gi & 2) == 0) & (par == esdf.NO_PARENT)
    assert np.all(np.abs(gd[lone]) == np.float32(d_max)), f"{what}: a voxel without a parent below d_max"
    return {"voxels": int(obs_g.sum()), "fixed": int(((gi & 2) > 0).sum()), "max_err_m": worst,
            "bound_m": tol, "at_d_max": int((np.abs(gd[obs_g]) == np.float32(d_max)).sum())}


def oracle_tsdf(P, frames):
    o = oracle_map(P)
    for p, pose in frames:
        o.integrate(p, pose)
    return o


def f32_blocks(o):
    c, D, W = o.export()[:3]
    return c, D.astype(np.float32), W.astype(np.float32)


def gpu_map_f32(vbx, P, cap=8192):
    return vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"],
                   storage="f32", max_range=P["max_range"], block_capacity=cap)


@pytest.mark.parametrize("gamma_voxels", [1.0, 1.5])   # one-voxel band; half the truncation (3v)
def test_esdf_batch_matches_oracle(vbx, gamma_voxels):
    import synth
    from oracle import esdf
    poses, frame = synth.room_sequence(320, 240, 4, seed=synth.SEED_BASE + 800)
    P = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", max_range=5.0)
    v, d_max = np.float32(0.05), 1.0
    gamma = float(np.float32(gamma_voxels * 0.05))
    o = oracle_tsdf(P, [(frame(k), poses[k]) for k in range(4)])
    c, D, W = f32_blocks(o)
    g = gpu_map_f32(vbx, P)
    g.write_blocks(c, np.stack([D, W], axis=-1))
    g.esdf_enable(gamma, d_max)
    st = g.esdf_update()
    ge = g.esdf_export()
    assert np.array_equal(ge[0], c)
    for queue in ("fifo", "priority"):
        E = esdf.OracleESDF(float(v), gamma, d_max, queue)
        E.update_from_blocks(c, D.astype(np.float64), W.astype(np.float64))
        res = compare_esdf(ge, E.export(), float(v), d_max, f"batch gamma={gamma_voxels}v {queue}")
        log(f"esdf batch gamma={gamma_voxels}v {queue}: {res}; gpu {st}; oracle {E.counts()}")
        E.close()


def test_esdf_incremental_matches_oracle(vbx):
    """Frame by frame: the TSDF oracle integrates a frame, the blocks it touched go to the GPU map
    and to the ESDF oracle, and both ESDFs update incrementally (band voxels appear, move, and
    leave the band as the fused TSDF changes)."""
    import synth
    from oracle import esdf
    poses, frame = synth.room_sequence(320, 240, 6, seed=synth.SEED_BASE + 801)
    P = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", max_range=5.0)
    v, gamma, d_max = 0.05, float(np.float32(0.05)), 0.8
    o = oracle_map(P)
    g = gpu_map_f32(vbx, P)
    g.esdf_enable(gamma, d_max)
    E = esdf.OracleESDF(float(np.float32(v)), gamma, d_max, "priority")
    for k in range(6):
        o.integrate(frame(k), poses[k])
        tc, _ = o.last_touches()
        touched = {tuple(x) for x in np.floor_divide(tc, 16).tolist()}
        c, D, W = f32_blocks(o)
        rows = np.array([i for i, b in enumerate(c.tolist()) if tuple(b) in touched], np.int64)
        g.write_blocks(c[rows], np.stack([D[rows], W[rows]], axis=-1))
        st = g.esdf_update()
        E.update_from_blocks(c[rows], D[rows].astype(np.float64), W[rows].astype(np.float64))
        res = compare_esdf(g.esdf_export(), E.export(), float(np.float32(v)), d_max, f"frame {k}")
        log(f"esdf incremental frame {k}: {len(rows)} blocks written; {res}; gpu {st}")
    E.close()


def test_esdf_point_source_across_blocks(vbx):
    """One band voxel inside 3 x 3 x 3 blocks of observed free space: the GPU field is the band
    value plus the closed-form 26-neighbour path length (binary32), across block borders."""
    from oracle import esdf
    v, gamma, d_max = 0.125, 0.125, 3.0
    P = dict(voxel_size=v, trunc=3 * v, weighting="const", merge="simple", max_range=5.0)
    bc = np.array([[x, y, z] for x in (-1, 0, 1) for y in (-1, 0, 1) for z in (-1, 0, 1)], np.int32)
    dw = np.zeros((27, 4096, 2), np.float32)
    dw[:, :, 0] = 3 * v
    dw[:, :, 1] = 1.0
    src_block = int(np.nonzero((bc == 0).all(axis=1))[0][0])
    d0 = np.float32(0.25 * v)
    dw[src_block, 5 + 16 * 7 + 256 * 9, 0] = d0
    g = gpu_map_f32(vbx, P, cap=64)
    g.write_blocks(bc, dw)
    g.esdf_enable(gamma, d_max)
    g.esdf_update()
    gc, gd, gi = g.esdf_export()
    vox = esdf.voxel_coords(gc)
    exp = np.minimum(float(d0) + esdf.chamfer(vox - np.array([5, 7, 9]), v), d_max).reshape(gd.shape)
    assert int(((gi & 2) > 0).sum()) == 1
    err = np.abs(gd - exp).max()
    assert err <= tolerance(v, d_max), err
    log(f"point source: max |d - closed form| = {err:.3g} m over {gd.size} voxels")


def test_esdf_follows_integration_incrementally(vbx):
    """The ESDF updated after every GPU integration call (blocks flagged by the update kernel)
    equals one ESDF built from scratch on the final TSDF, distances and flags bit for bit."""
    import synth
    poses, frame = synth.room_sequence(320, 240, 5, seed=synth.SEED_BASE + 802)
    P = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", max_range=5.0)
    gamma, d_max = float(np.float32(0.05)), 1.0
    g = gpu_map_f32(vbx, P)
    g.esdf_enable(gamma, d_max)
    for k in range(5):
        g.integrate_frames([(torch.from_numpy(frame(k)).cuda(), poses[k], 320)])
        st = g.esdf_update()
        assert st["dirty_blocks"] > 0
    inc = g.esdf_export()
    c, dw = g.export()
    fresh = gpu_map_f32(vbx, P)
    fresh.write_blocks(c, dw)
    fresh.esdf_enable(gamma, d_max)
    fresh.esdf_update()
    bat = fresh.esdf_export()
    assert np.array_equal(inc[0], bat[0])
    assert np.array_equal(inc[2] & 131, bat[2] & 131)
    assert np.array_equal(inc[1], bat[1])
    # parents too: the lower wave keeps, among the neighbours that give the smallest distance,
    # the one with the smallest index, whatever the order of the rounds
    assert np.array_equal(inc[2], bat[2])
    nothing = g.esdf_update()
    assert nothing["dirty_blocks"] == 0 and nothing["raise_rounds"] == 0
    assert np.array_equal(g.esdf_export()[1], inc[1])
