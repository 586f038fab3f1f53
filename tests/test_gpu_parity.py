"""GPU path (through the C ABI) against the CPU oracle on the same seeded inputs."""
import numpy as np
import pytest

from tests.common import (compare_export, compare_touches, gpu_map, log, oracle_map)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_03631_amd as vbx
    vbx.lib()
    return vbx


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def run_both(vbx, params, frames, batch=False, **over):
    """Integrate frames [(points, pose[, width])] on the GPU and in the oracle."""
    g = gpu_map(vbx, params, **over)
    o = oracle_map(params, **over)
    if batch:
        g.integrate_frames([(dev(f[0]), f[1]) + tuple(f[2:]) for f in frames])
    for f in frames:
        if not batch:
            g.integrate(dev(f[0]), f[1])
        o.integrate(f[0], f[1])
    assert g.sync() == 0
    return g, o


# ---------------------------------------------------------------------------
# traversal primitive
# ---------------------------------------------------------------------------
def test_traversal_bit_exact(vbx):
    import oracle
    rng = np.random.default_rng(21)
    A = rng.uniform(-40, 40, size=(4000, 3)).astype(np.float32)
    B = (A + rng.uniform(-9, 9, size=(4000, 3))).astype(np.float32)
    # dyadic segments with exact face and edge ties
    Ad = (rng.integers(-64, 64, size=(1000, 3)) / 16.0).astype(np.float32)
    Bd = (Ad + rng.choice([-2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.0, 4.0], size=(1000, 3))).astype(np.float32)
    Ac = np.floor(Ad) + np.float32(0.5)
    Bc = (Ac + rng.choice([-2.0, 2.0], size=(1000, 3))).astype(np.float32)
    A = np.concatenate([A, Ad, Ac.astype(np.float32)])
    B = np.concatenate([B, Bd, Bc])
    log(f"traversal: {A.shape[0]} segments")
    out, counts = vbx.debug_traverse(dev(A), dev(B), cap=64)
    out, counts = out.cpu().numpy(), counts.cpu().numpy()
    for i in range(A.shape[0]):
        ref = oracle.dda(A[i], B[i])
        assert counts[i] == ref.shape[0], i
        assert np.array_equal(out[i, :counts[i]], ref), i


def test_traversal_blocks_bit_exact(vbx):
    """The blocks the crossing kernel's block walk finds (from the block-changing steps alone)
    are the distinct blocks of the oracle's voxel traversal, in order: random band-length and
    long segments, and dyadic ones with exact ties at block faces, edges and corners."""
    import oracle
    rng = np.random.default_rng(22)
    A = rng.uniform(-200, 200, size=(3000, 3)).astype(np.float32)
    B = (A + rng.uniform(-40, 40, size=(3000, 3))).astype(np.float32)
    Al = rng.uniform(-200, 200, size=(300, 3)).astype(np.float32)
    Bl = (Al + rng.uniform(-300, 300, size=(300, 3))).astype(np.float32)
    Ad = (16.0 * rng.integers(-4, 4, size=(3000, 3)) + rng.integers(-8, 8, size=(3000, 3)) / 4.0).astype(np.float32)
    Bd = (Ad + rng.integers(-48, 48, size=(3000, 3)) / 2.0).astype(np.float32)
    C = (16.0 * rng.integers(-4, 4, size=(1000, 3))).astype(np.float32)
    D = (rng.integers(-48, 48, size=(1000, 3)) / 8.0).astype(np.float32)
    A = np.concatenate([A, Al, Ad, C - D])
    B = np.concatenate([B, Bl, Bd, C + D])
    log(f"traversal blocks: {A.shape[0]} segments")
    out, counts = vbx.debug_traverse_blocks(dev(A), dev(B), cap=128)
    out, counts = out.cpu().numpy(), counts.cpu().numpy()
    multi = 0
    for i in range(A.shape[0]):
        vox = oracle.dda(A[i], B[i])
        blk = vox >> 4
        keep = np.ones(blk.shape[0], bool)
        keep[1:] = np.any(blk[1:] != blk[:-1], axis=1)
        ref = blk[keep]
        multi += ref.shape[0] > 1
        assert counts[i] == ref.shape[0], i
        assert np.array_equal(out[i, :counts[i]], ref), i
    log(f"  ok: {multi} segments cross blocks")


# ---------------------------------------------------------------------------
# single frames, every mode
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("weighting,merge,dist", [("const", "simple", "eq1"), ("quad", "simple", "eq1"),
                                                  ("const", "grouped", "eq1"), ("quad", "grouped", "eq1"),
                                                  ("quad", "grouped", "ray")])
def test_c1_room_frame(vbx, weighting, merge, dist):
    import synth
    w = synth.config1()
    params = dict(w.params, weighting=weighting, merge=merge, dist=dist)
    log(f"c1 160x120 {weighting} {merge} {dist}")
    g, o = run_both(vbx, params, [(w.frame(0), w.poses[0])])
    n = compare_touches(g.last_touches(), o.last_touches())
    res = compare_export(g.export(), o.export(), params)
    st = g.stats()
    assert st["touches"] == sum(o.last_touches()[1]) and st["voxels"] == n
    log(f"  ok: {res}")


def test_c1_stats_match_oracle(vbx):
    import synth
    w = synth.config1()
    params = dict(w.params)
    pts = w.frame(0).copy()
    pts[::17] = np.nan                       # invalid points
    pts[5::23] *= 3.0                        # beyond max range
    g = gpu_map(vbx, params)
    o = oracle_map(params)
    g.integrate(dev(pts), w.poses[0])
    ost = o.integrate(pts, w.poses[0])
    assert g.sync() == 0
    st = g.stats()
    for k_g, k_o in [("points", "points"), ("valid", "valid"), ("invalid", "invalid"),
                     ("out_of_bounds", "out_of_bounds"), ("rays", "rays"), ("touches", "touches"),
                     ("voxels", "voxels"), ("new_blocks", "new_blocks")]:
        assert st[k_g] == ost[k_o], (k_g, st[k_g], ost[k_o])


@pytest.mark.parametrize("storage", ["f32", "f16", "s16"])
def test_room_sequence_grouped(vbx, storage):
    """Several 320x240 frames of the furnished room (grouped, 1/z^2), frame by frame."""
    import synth
    poses, frame = synth.room_sequence(320, 240, 6, seed=synth.SEED_BASE + 11)
    params = dict(voxel_size=0.05, trunc=0.15, max_range=5.0, weighting="quad", merge="grouped",
                  storage=storage)
    frames = [(frame(k), poses[k]) for k in range(6)]
    log(f"room 320x240 x6 grouped {storage}")
    g, o = run_both(vbx, params, frames)
    compare_touches(g.last_touches(), o.last_touches())
    res = compare_export(g.export(), o.export(), params, storage=storage)
    log(f"  ok: {res}")


def test_lidar_sweeps_simple(vbx):
    import synth
    w = synth.config3(n_sweeps=3, n_az=512)
    params = dict(w.params)
    frames = [(w.frame(k), w.poses[k]) for k in range(3)]
    log("lidar 64x512 x3 simple const")
    g, o = run_both(vbx, params, frames)
    compare_touches(g.last_touches(), o.last_touches())
    res = compare_export(g.export(), o.export(), params)
    log(f"  ok: {res}")


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("width", [0, 64])
def test_grouped_tiles_with_more_voxels_than_their_table(vbx, width):
    """Points scattered so that a 512-point tile spans more distinct voxels than the tile's
    voxel table holds: the runs that find it full become partial groups of their own, which
    the cross-tile merge must combine exactly (some identical neighbours make runs of two)."""
    rng = np.random.default_rng(1611036310 + 77 + width)
    n = 4096
    pts = np.empty((n, 3), np.float32)
    pts[:, :2] = rng.uniform(-2.0, 2.0, size=(n, 2))
    pts[:, 2] = rng.uniform(1.0, 5.0, size=n)
    pts[1::4] = pts[0::4]            # 384 distinct voxels per 512-point tile (table: 256)
    pose = np.eye(3, 4, dtype=np.float32)
    params = dict(voxel_size=0.02, trunc=0.06, weighting="quad", merge="grouped", max_range=10.0,
                  block_capacity=65536)
    frames = [(pts, pose, width)]
    g, o = run_both(vbx, params, frames, batch=True)
    compare_touches(g.last_touches(), o.last_touches())
    res = compare_export(g.export(), o.export(), params)
    st = g.stats()
    log(f"scattered tiles (width {width}): rays {st['rays']}, {res}")
    # identity pose: world = sensor coordinates; one group (ray) per distinct binary32 voxel key
    iv = np.float32(1.0) / np.float32(0.02)
    keys = np.floor(pts * iv).astype(np.int64)
    assert st["rays"] == np.unique(keys, axis=0).shape[0]
    if width == 0:   # every 512-point tile overflowed its 256-slot table
        assert all(np.unique(keys[s:s + 512], axis=0).shape[0] > 256 for s in range(0, n, 512))



def test_grouped_large_bins_merge_in_one_dense_pass(vbx):
    """Every 512-point tile holds the same 256 voxels of one two-voxel z-slab of one block (two
    points each), so that slab's sort bin gets 16 x 256 partial groups: far more than one LDS
    hash batch, merged over the dense table of its 512 voxels.  A second frame, shifted by half
    a voxel, makes each tile span two blocks and two slabs."""
    rng = np.random.default_rng(1611036310 + 91)
    v = 0.05
    ij = np.stack(np.meshgrid(np.arange(16), np.arange(16), indexing="ij"), -1).reshape(-1, 2)
    pts = np.empty((8192, 3), np.float32)
    for t in range(16):                        # tile t: each of the 256 voxels twice
        blk = np.concatenate([ij, ij])[rng.permutation(512)]
        jit = rng.uniform(0.1, 0.9, size=(512, 3))
        pts[512 * t:512 * (t + 1), 0] = (blk[:, 0] + jit[:, 0]) * v
        pts[512 * t:512 * (t + 1), 1] = (blk[:, 1] + jit[:, 1]) * v
        pts[512 * t:512 * (t + 1), 2] = (20 + jit[:, 2]) * v          # voxel z 20: block 1, local z 4
    pose = np.eye(3, 4, dtype=np.float32)
    pose2 = pose.copy()
    pose2[:, 3] = [0.5 * v, 0.5 * v, 0.5 * v]
    params = dict(voxel_size=v, trunc=3 * v, weighting="quad", merge="grouped", max_range=10.0)
    frames = [(pts, pose), (pts, pose2)]      # one call each: touches compare the second frame
    g, o = run_both(vbx, params, frames)
    compare_touches(g.last_touches(), o.last_touches())
    res = compare_export(g.export(), o.export(), params)
    st = g.stats()
    log(f"large bins: rays {st['rays']}, {res}")
    # one ray per distinct binary32 voxel key of each frame (identity rotation: the world point
    # is the sensor point plus the translation, in binary32 as on the device)
    iv = np.float32(1.0) / np.float32(v)
    groups = [np.unique(np.floor((pts + q[:, 3]).astype(np.float32) * iv), axis=0).shape[0]
              for q in (pose, pose2)]
    assert groups[0] == 256
    assert st["rays"] == sum(groups)


def test_empty_and_invalid_frames(vbx):
    params = dict(voxel_size=0.1, trunc=0.3, weighting="quad", merge="grouped")
    g = gpu_map(vbx, params)
    pose = np.eye(3, 4, dtype=np.float32)
    g.integrate(dev(np.zeros((0, 3))), pose)
    g.integrate(dev(np.full((1000, 3), np.nan)), pose)
    assert g.sync() == 0
    assert g.num_blocks() == 0
    st = g.stats()
    assert st["invalid"] == 1000 and st["rays"] == 0


@pytest.mark.parametrize("n", [1, 2, 511, 513, 1023, 1025, 4097])
@pytest.mark.parametrize("merge", ["simple", "grouped"])
def test_ragged_sizes(vbx, n, merge):
    rng = np.random.default_rng(n)
    pts = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(0.5, 3, n)], 1)
    pose = np.eye(3, 4, dtype=np.float32)
    pose[:, 3] = [0.01, 0.02, 0.03]
    params = dict(voxel_size=0.1, trunc=0.3, weighting="quad", merge=merge)
    g, o = run_both(vbx, params, [(pts.astype(np.float32), pose)])
    compare_touches(g.last_touches(), o.last_touches())
    compare_export(g.export(), o.export(), params)


@pytest.mark.parametrize("merge", ["simple", "grouped"])
def test_scattered_points_many_blocks_per_batch(vbx, merge):
    """420 000 points scattered through a 25 m cube (about 4 000 blocks of 1.6 m): consecutive
    rays end in different blocks, so each batch of 256 rays in the crossing kernel brings a few
    hundred blocks to its workgroup's LDS block set, and with more batches than workgroups the
    set fills and is emptied between batches.  Block set, touches and values against the
    oracle."""
    rng = np.random.default_rng(31)
    n = 420000
    pts = np.empty((n, 3), np.float32)
    pts[:, 0] = rng.uniform(-12.5, 12.5, n)
    pts[:, 1] = rng.uniform(-12.5, 12.5, n)
    pts[:, 2] = rng.uniform(0.5, 25.5, n)
    pose = np.eye(3, 4, dtype=np.float32)
    pose[:, 3] = [0.05, -0.02, 0.01]
    params = dict(voxel_size=0.1, trunc=0.3, weighting="quad", merge=merge, max_range=40.0,
                  block_capacity=16384, keep_touches=True)
    log(f"scattered points: {n}, {merge}")
    g, o = run_both(vbx, params, [(pts, pose)])
    nt = compare_touches(g.last_touches(), o.last_touches())
    res = compare_export(g.export(), o.export(), params, quiet=True)
    assert g.num_blocks() > 3000
    log(f"  ok: {g.num_blocks()} blocks, {nt} touched voxels, {res}")


def test_organised_hint_does_not_change_result(vbx):
    import synth
    poses, frame = synth.room_sequence(160, 120, 2, seed=synth.SEED_BASE + 12)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped")
    a = gpu_map(vbx, params)
    b = gpu_map(vbx, params)
    a.integrate_frames([(dev(frame(k)), poses[k], 160) for k in range(2)])
    b.integrate_frames([(dev(frame(k)), poses[k], 0) for k in range(2)])
    assert a.sync() == 0 and b.sync() == 0
    ca, da = a.export()
    cb, db = b.export()
    assert np.array_equal(ca, cb) and np.array_equal(da, db)


def test_permutation_bit_identical(vbx):
    import synth
    w = synth.config1()
    pts = w.frame(0)
    perm = np.random.default_rng(3).permutation(pts.shape[0])
    for merge in ("simple", "grouped"):
        params = dict(w.params, weighting="quad", merge=merge)
        a = gpu_map(vbx, params)
        b = gpu_map(vbx, params)
        a.integrate(dev(pts), w.poses[0])
        b.integrate(dev(pts[perm]), w.poses[0])
        assert a.sync() == 0 and b.sync() == 0
        ca, da = a.export()
        cb, db = b.export()
        assert np.array_equal(ca, cb) and np.array_equal(da, db), merge


def test_repeat_runs_bit_identical(vbx):
    import synth
    poses, frame = synth.room_sequence(320, 240, 3, seed=synth.SEED_BASE + 13)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped")
    outs = []
    for _ in range(2):
        g = gpu_map(vbx, params)
        g.integrate_frames([(dev(frame(k)), poses[k], 320) for k in range(3)])
        assert g.sync() == 0
        outs.append(g.export())
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


# ---------------------------------------------------------------------------
# raycasting over the whole ray (Sec. IV-B): every voxel from the sensor to delta behind
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("weighting,merge", [("const", "simple"), ("quad", "grouped")])
def test_full_ray_room(vbx, weighting, merge):
    """The whole ray: rays cross up to 22 blocks (voxel 0.05 m, range 5 m), the free space in
    front of every surface is carved; touches bit-exact, the map within the parity bar."""
    import synth
    poses, frame = synth.room_sequence(320, 240, 3, seed=synth.SEED_BASE + 900)
    params = dict(voxel_size=0.05, trunc=0.15, max_range=5.0, weighting=weighting, merge=merge,
                  full_ray=True, block_capacity=16384)
    frames = [(frame(k), poses[k], 320) for k in range(3)]
    log(f"full ray 320x240 x3 {weighting} {merge}")
    g, o = run_both(vbx, params, frames)      # frame by frame: the last touches are the last frame's
    compare_touches(g.last_touches(), o.last_touches())
    res = compare_export(g.export(), o.export(), params)
    band = gpu_map(vbx, dict(params, full_ray=False))
    band.integrate_frames([(dev(f[0]), f[1], f[2]) for f in frames])
    assert band.sync() == 0
    nb_band, nb_full = band.export()[0].shape[0], res["blocks"]
    assert nb_full > nb_band, "the whole ray allocates the free space's blocks too"
    log(f"  ok: {res}; blocks {nb_full} (band only: {nb_band})")


def test_full_ray_lidar(vbx):
    """LiDAR sweeps over the whole ray: walks of up to 303 voxels (range 60 m, voxel 0.2 m)."""
    import synth
    w = synth.config3(n_sweeps=2, n_az=512)
    params = dict(w.params, full_ray=True, block_capacity=16384)
    frames = [(w.frame(k), w.poses[k]) for k in range(2)]
    log("full ray lidar 64x512 x2")
    g, o = run_both(vbx, params, frames)
    compare_touches(g.last_touches(), o.last_touches())
    res = compare_export(g.export(), o.export(), params)
    log(f"  ok: {res}")


def test_full_ray_limit(vbx):
    """A whole-ray walk longer than 1024 voxels is refused when the map is made."""
    with pytest.raises(vbx.VbxError) as e:
        gpu_map(vbx, dict(voxel_size=0.02, trunc=0.06, max_range=30.0, full_ray=True))
    assert e.value.status == -6
