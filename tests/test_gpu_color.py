"""The colour layer on the GPU (Sec. IV-B: a grouped ray carries the mean colour of its points,
and voxel colours are fused with the same weights as the distances) against the oracle.

Bars.  With constant weighting every quantity the colour depends on is an exact small integer on
both sides (ray weights, their sums, W and the channel sums), and both divide once correctly
rounded and round to the nearest integer, ties to even: the colours are bit-identical.  With the
quadratic weighting the GPU sums fixed-point weights (2^-kw) where the oracle sums binary64
ones, so a quotient next to a half-integer may round the other way: each channel may differ by
one unit.  A difference does not grow: the next frame scales it by W / (W + sum w) < 1, and the
binary16 W of the 16-bit storages moves the quotient by at most
(sum w / (W + sum w)) (W / (W + sum w)) 255 / 2048, which keeps the sum of the two below 1.
Voxels are compared where both sides hold W > 0 (a weight below 2^-kw is observed by the oracle
alone)."""
import numpy as np
import pytest

from tests.common import compare_export, gpu_map, log, oracle_map

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_03631_amd as vbx
    vbx.lib()
    return vbx


def _frames(n, w=160, h=120, seed_off=900):
    import synth
    seed = synth.SEED_BASE + seed_off
    poses, frame = synth.room_sequence(w, h, n, seed=seed)
    out = []
    for k in range(n):
        p = frame(k)
        out.append((p, poses[k], w, synth.point_colors(p, poses[k], seed, k)))
    return out


def _dev(frames):
    return [(torch.from_numpy(p).cuda(), pose, w, torch.from_numpy(c.view(np.int32)).cuda())
            for p, pose, w, c in frames]


def compare_colors(g, o, exact, what=""):
    gc, gdw = g.export()
    oc, oD, oW = o.export()[:3]
    assert np.array_equal(gc, oc), f"{what}: block sets differ"
    gcc, grgb = g.export_colors()
    assert np.array_equal(gcc, gc)
    orgb = o.export_colors()
    both = (gdw[..., 1] > 0) & (oW > 0)
    diff = np.zeros(grgb.shape, np.int64)
    for k in range(3):
        a = (grgb.astype(np.int64) >> (8 * k)) & 255
        b = (orgb.astype(np.int64) >> (8 * k)) & 255
        diff = np.maximum(diff, np.abs(a - b))
    worst = int(diff[both].max(initial=0))
    n_off = int((diff[both] > 0).sum())
    # voxels that neither side has observed stay black on both
    assert np.all(grgb[gdw[..., 1] == 0] == 0), f"{what}: an unobserved GPU voxel has a colour"
    if exact:
        assert worst == 0, f"{what}: {n_off} voxels differ (max {worst} units)"
    else:
        assert worst <= 1, f"{what}: colour differs by {worst} units"
    assert np.all(grgb >> 24 == 0)
    return {"voxels": int(both.sum()), "off_by_one": n_off, "max": worst}


@pytest.mark.parametrize("merge", ["simple", "grouped"])
@pytest.mark.parametrize("weighting,storage", [("const", "f32"), ("const", "s16"), ("quad", "f32"),
                                               ("quad", "f16"), ("quad", "s16")])
def test_color_matches_oracle(vbx, merge, weighting, storage):
    """Four frames in one call (the colour kernel folds them in order) and two more one at a time,
    against the oracle integrating frame by frame; D and W stay at their own bars."""
    P = dict(voxel_size=0.05, trunc=0.15, weighting=weighting, merge=merge, storage=storage,
             max_range=5.0, color=True, keep_touches=False)
    fr = _frames(6)
    o = oracle_map(P)
    for p, pose, w, c in fr:
        o.integrate(p, pose, colors=c)
    g = gpu_map(vbx, P)
    dev = _dev(fr)
    g.integrate_frames(dev[:4])
    for f in dev[4:]:
        g.integrate_frames([f])
    res = compare_colors(g, o, exact=weighting == "const", what=f"{merge} {weighting} {storage}")
    compare_export(g.export(), o.export(), P, storage, quiet=True)
    log(f"colour {merge} {weighting} {storage}: {res}")


def test_color_uniform_points(vbx):
    """Every point of every frame has one colour: every observed voxel holds exactly that colour
    (any weights, any rounding), while D and W are those of a map without colour."""
    import synth
    P = dict(voxel_size=0.04, trunc=0.12, weighting="quad", merge="grouped", storage="f16",
             max_range=5.0, keep_touches=False)
    poses, frame = synth.room_sequence(320, 240, 3, seed=synth.SEED_BASE + 901)
    rgb = 17 | (200 << 8) | (93 << 16)
    g = gpu_map(vbx, P, color=True)
    plain = gpu_map(vbx, P)
    for k in range(3):
        p = torch.from_numpy(frame(k)).cuda()
        col = torch.full((p.shape[0],), rgb, dtype=torch.int32, device="cuda")
        g.integrate_frames([(p, poses[k], 320, col)])
        plain.integrate_frames([(p, poses[k], 320)])
    gc, gdw = g.export()
    pc, pdw = plain.export()
    assert np.array_equal(gc, pc) and np.array_equal(gdw, pdw)
    _, col = g.export_colors()
    seen = gdw[..., 1] > 0
    assert np.all(col[seen] == rgb) and np.all(col[~seen] == 0)
    log(f"uniform colour: {int(seen.sum())} voxels")


def test_color_multi_map_and_reserve(vbx):
    """A colour map and a map without colour in one multi-map call: the plain map is unchanged by
    the other's colours; growing the colour map's pool keeps its colours."""
    import paper_1611_03631_amd as V
    P = dict(voxel_size=0.05, trunc=0.15, weighting="const", merge="grouped", storage="f32",
             max_range=5.0, keep_touches=False)
    fr = _frames(3, seed_off=902)
    dev = _dev(fr)
    gcol = gpu_map(vbx, P, color=True, block_capacity=1024)
    gplain = gpu_map(vbx, P, block_capacity=1024)
    ref = gpu_map(vbx, P, block_capacity=1024)
    o = oracle_map(P, color=True)
    for (p, pose, w, c), f in zip(fr, dev):
        V.integrate_multi([gcol, gplain], [f, f[:3]])
        ref.integrate_frames([f[:3]])
        o.integrate(p, pose, colors=c)
    a, b = gplain.export(), ref.export()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    before = compare_colors(gcol, o, exact=True, what="multi")
    _, rgb0 = gcol.export_colors()
    gcol.reserve(4096)
    c1, rgb1 = gcol.export_colors()
    assert np.array_equal(rgb0, rgb1)
    log(f"multi-map colour: {before}")


def test_color_requires_point_colours(vbx):
    P = dict(voxel_size=0.05, trunc=0.15, max_range=5.0, keep_touches=False)
    g = gpu_map(vbx, P, color=True)
    fr = _frames(1, w=64, h=48, seed_off=903)
    p = torch.from_numpy(fr[0][0]).cuda()
    with pytest.raises(vbx.VbxError) as e:
        g.integrate_frames([(p, fr[0][1], 64)])
    assert e.value.status == vbx.ERR_INVALID_ARG
    plain = gpu_map(vbx, P)
    with pytest.raises(vbx.VbxError):
        plain.export_colors()


@pytest.mark.parametrize("tuning", [(2, 256, 0), (2, 512, 0)])
def test_color_update_candidates_agree(vbx, tuning):
    """The colour update's launch candidates (half or quarter blocks) give the same map and
    colours as the default one."""
    P = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", storage="f32",
             max_range=5.0, color=True, keep_touches=False)
    dev = _dev(_frames(5, seed_off=904))
    a = gpu_map(vbx, P)
    a.integrate_frames(dev)
    b = gpu_map(vbx, P)
    b.set_tuning(*tuning)
    b.integrate_frames(dev)
    assert a.sync() == 0 and b.sync() == 0
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea[0], eb[0]) and np.array_equal(ea[1], eb[1])
    assert np.array_equal(a.export_colors()[1], b.export_colors()[1])
