"""The distance query by trilinear interpolation, on the GPU through the C ABI, against the oracle.

The oracle interpolates the GPU map's own export, so this checks the query alone.  Which
queries are known is a binary32 decision on both sides and must match exactly.  The distances
are blended in binary32 on the GPU and in binary64 in the oracle: eight corners of magnitude at
most delta, three lerp levels of two products and a sum each, so the difference stays below
about 8 * 2^-24 * delta; the test allows 1e-5 v (delta = 3 v here, so about 8 times that bound).
"""
import numpy as np
import pytest

from tests.common import gpu_map, log

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


def world_points(frames):
    out = []
    for p, pose in frames:
        P = np.asarray(p, np.float64)
        P = P[np.all(np.isfinite(P), axis=1)]
        T = np.asarray(pose, np.float64).reshape(3, 4)
        out.append(P @ T[:, :3].T + T[:, 3])
    return np.concatenate(out)


def queries(frames, v, seed):
    rng = np.random.default_rng(seed)
    surf = world_points(frames)
    surf = surf[rng.choice(surf.shape[0], size=min(20000, surf.shape[0]), replace=False)]
    near = surf[:5000] + rng.normal(scale=1.5 * v, size=(5000, 3))
    lo, hi = surf.min(axis=0) - 1.0, surf.max(axis=0) + 1.0
    box = rng.uniform(lo, hi, size=(5000, 3))
    centres = (np.floor(surf[:2000] / v) + 0.5) * v
    odd = np.array([[np.nan, 0.0, 0.0], [0.0, np.inf, 0.0], [1e9, 0.0, 0.0], [-1e9, 1.0, 2.0]])
    return np.concatenate([surf, near, box, centres, odd]).astype(np.float32)


@pytest.mark.parametrize("storage,weighting,merge", [("f32", "quad", "grouped"),
                                                     ("f16", "const", "simple"),
                                                     ("s16", "quad", "grouped")])
def test_interpolation_matches_oracle_on_gpu_map(vbx, storage, weighting, merge):
    import synth
    from oracle import interp
    poses, frame = synth.room_sequence(160, 120, 4, seed=synth.SEED_BASE + 61)
    frames = [(frame(k), poses[k]) for k in range(4)]
    v = 0.05
    P = dict(voxel_size=v, trunc=3 * v, weighting=weighting, merge=merge, storage=storage,
             keep_touches=False)
    g = gpu_map(vbx, P)
    g.integrate_frames([(dev(p), pose, 160) for p, pose in frames])
    assert g.sync() == 0
    q = queries(frames, v, 5)
    got = g.interpolate(dev(q))
    assert g.sync() == 0
    got = got.cpu().numpy().astype(np.float64)
    coords, dw = g.export()
    ref = interp.interpolate(coords, dw[:, :, 0].astype(np.float64), dw[:, :, 1].astype(np.float64),
                             v, q)
    known = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), known)
    assert known.sum() > 10000 and (~known).sum() > 1000
    err = np.max(np.abs(got[known] - ref[known]))
    log(f"{storage} {weighting} {merge}: {int(known.sum())} of {q.shape[0]} known, max |dD| = {err:.3g} m")
    assert err <= 1e-5 * v


def test_interpolation_of_an_empty_map_and_zero_queries(vbx):
    g = gpu_map(vbx, dict(voxel_size=0.1, trunc=0.3))
    out = g.interpolate(dev(np.array([[0.1, 0.2, 0.3], [0.0, 0.0, 0.0]])))
    assert g.sync() == 0
    assert np.isnan(out.cpu().numpy()).all()
    assert g.interpolate(dev(np.zeros((0, 3)))).numel() == 0
