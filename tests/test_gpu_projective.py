"""Projection mapping (Sec. IV-B) on the GPU against the oracle: every voxel of the blocks the
frames' truncation bands cross, projected into the depth image.

The pixel choice and the update decisions are binary32 on both sides (the same operations in
the same order), so the touched voxels are bit-exact.  The distance is the pixel's depth minus
the voxel centre's depth: the kernel forms the centre's camera depth in binary32 from world
coordinates, so its error is a few units in the last place of the world coordinates and of the
centre-to-sensor offset, bounded here by 8 * 2^-24 (world extent + max_range) for the parity
bound's distance term."""
import numpy as np
import pytest

from tests.common import compare_export, compare_touches, gpu_map, log, oracle_map

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


def intrinsics(width, height):
    f = 100.0 * width / 160.0           # the synthetic pinhole's focal length (pixels)
    return (f, f, width / 2.0, height / 2.0)


@pytest.mark.parametrize("weighting,storage", [("const", "f32"), ("quad", "f32"), ("quad", "s16")])
def test_projective_room_sequence(vbx, weighting, storage):
    import synth
    W, H = 320, 240
    poses, frame = synth.room_sequence(W, H, 4, seed=synth.SEED_BASE + 950)
    K = intrinsics(W, H)
    params = dict(voxel_size=0.05, trunc=0.15, max_range=5.0, weighting=weighting, merge="simple",
                  storage=storage, block_capacity=8192)
    g = gpu_map(vbx, params)
    o = oracle_map(params)
    log(f"projective 320x240 x4 {weighting} {storage}")
    for k in range(4):
        p = frame(k)
        g.integrate_projective([(dev(p), poses[k], W)], K)
        o.integrate_projective(p, poses[k], W, K)
        assert g.sync() == 0
        n = compare_touches(g.last_touches(), o.last_touches())
    coords = o.export()[0]
    extent = float((np.abs(coords).max() + 1) * 16 * 0.05)
    res = compare_export(g.export(), o.export(), dict(params, dist_err=8 * 2.0 ** -24 * (extent + 5.0)),
                         storage=storage)
    st = g.stats()
    assert st["touches"] > 0
    log(f"  ok: {n} voxels in the last frame; {res}")


def test_projective_blocks_batch_and_merge_mode(vbx):
    """The blocks are the ones raycasting allocates; several frames in one call equal the same
    frames one call each, bit for bit; a map configured for grouped raycasting integrates the
    same way (the merge mode does not apply)."""
    import synth
    W, H = 320, 240
    poses, frame = synth.room_sequence(W, H, 3, seed=synth.SEED_BASE + 951)
    K = intrinsics(W, H)
    params = dict(voxel_size=0.05, trunc=0.15, max_range=5.0, weighting="quad", merge="simple",
                  block_capacity=8192, keep_touches=False)
    frames = [(dev(frame(k)), poses[k], W) for k in range(3)]
    seq = gpu_map(vbx, params)
    for f in frames:
        seq.integrate_projective([f], K)
    bat = gpu_map(vbx, params)
    bat.integrate_projective(frames, K)
    grp = gpu_map(vbx, dict(params, merge="grouped"))
    grp.integrate_projective(frames, K)
    ray = gpu_map(vbx, params)
    ray.integrate_frames(frames)
    for m in (seq, bat, grp, ray):
        assert m.sync() == 0
    a, b, c = seq.export(), bat.export(), grp.export()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    assert np.array_equal(a[0], ray.export()[0])


def test_projective_refuses_unorganised_frames(vbx):
    import synth
    poses, frame = synth.room_sequence(160, 120, 1, seed=synth.SEED_BASE + 952)
    g = gpu_map(vbx, dict(voxel_size=0.1, trunc=0.3))
    with pytest.raises(vbx.VbxError) as e:
        g.integrate_projective([(dev(frame(0)), poses[0], 0)], intrinsics(160, 120))
    assert e.value.status == vbx.ERR_INVALID_ARG
    with pytest.raises(vbx.VbxError):
        g.integrate_projective([(dev(frame(0)), poses[0], 160)], (0.0, 100.0, 80.0, 60.0))
