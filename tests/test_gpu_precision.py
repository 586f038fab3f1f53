"""16-bit voxel storage (4 bytes per voxel; every sum and update in binary32, the stored values
rounded once per frame): parity with the oracle's mode that rounds to the same storage, and the
storage error itself against the binary64 oracle over a 100-frame sequence, per voxel-size
class of the 32-map batched mix.

Two 16-bit forms share the layout (D / delta in the low half, binary16 W in the high half):
"f16" stores D / delta as binary16, "s16" as a fixed-point number in steps of 1/32767.  A
binary16 D / delta near +-1 has 11 significant bits, so every frame may move D by up to
2^-12 delta = 7.3e-4 v (delta = 3v) and the rounding errors of a long sequence add up like a
random walk; the fixed-point step is 32767 times finer than delta everywhere in the band."""
import numpy as np
import pytest

from tests.common import compare_export, gpu_map, log, oracle_map

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

T = 100                     # frames per map
CHECKPOINTS = (10, 50, 100)  # frames after which the storage error is measured
BAR = 2e-3                  # |D - D_64| / v for 16-bit storage
# binary16 D / delta misses the bar: after 100 frames its largest error over the three classes
# is 4.2e-3 to 4.7e-3 v (rms 4.5e-4 to 7.3e-4 v); this limit keeps a regression from passing
F16_LIMIT = 6e-3


@pytest.fixture(scope="module")
def vbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_03631_amd as vbx
    vbx.lib()
    return vbx


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def storage_error(gpu_export, e64, emul, v):
    """max and rms |D - D_64| / v over the voxels the storage keeps as observed (the emulating
    oracle's W > 0); also how many binary64-observed voxels the storage lost to W underflow."""
    coords, dw = gpu_export
    assert np.array_equal(coords, e64[0])
    sel = emul[2] > 0
    err = np.abs(dw[:, :, 0].astype(np.float64) - e64[1])[sel] / v
    lost = int(((e64[2] > 0) & ~sel).sum())
    return float(err.max(initial=0.0)), float(np.sqrt(np.mean(err ** 2))), int(sel.sum()), lost


@pytest.mark.parametrize("m", [0, 1, 2])      # voxel 0.02 / 0.05 / 0.10 m (map m of the mix)
def test_16bit_storage_error_per_class(vbx, m):
    import synth
    w = synth.config4_map(m, n_ticks=T)
    P = dict(w.params, block_capacity=8192)
    v = float(np.float32(P["voxel_size"]))
    forms = ("f16", "s16", "f32")
    g = {s: gpu_map(vbx, dict(P, storage=s, keep_touches=False)) for s in forms}
    o = {s: oracle_map(P, storage=s) for s in forms}
    worst = {"f16": 0.0, "s16": 0.0}
    for k in range(T):
        p, pose = w.frame(k), w.poses[k]
        d = dev(p)
        for s in forms:
            g[s].integrate_frames([(d, pose, w.width)])
            o[s].integrate(p, pose)
        if k + 1 in CHECKPOINTS:
            for s in forms:
                assert g[s].sync() == 0
            ex = {s: o[s].export() for s in forms}
            gx = {s: g[s].export() for s in forms}
            # parity: each GPU storage against the oracle rounding to the same storage
            for s in forms:
                compare_export(gx[s], ex[s], P, storage=s)
            # the storage error itself, against the binary64 oracle
            line = []
            for s in forms:
                mx, rms, n, lost = storage_error(gx[s], ex["f32"], ex[s], v)
                if s != "f32":
                    worst[s] = max(worst[s], mx)
                line.append(f"{s} max {mx:.3e} rms {rms:.3e} (lost {lost})")
            log(f"map {m} {w.width}x{w.height} v={v:g} frame {k + 1}: {n} voxels; |D - D64|/v: "
                + "; ".join(line))
            assert worst["s16"] <= BAR, f"fixed-point 16-bit storage misses {BAR} v: {worst['s16']:.3e}"
            assert worst["f16"] <= F16_LIMIT
