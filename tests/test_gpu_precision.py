"""Binary16 storage (D/delta and W stored as binary16, every sum and update in binary32):
parity with the binary16-emulating oracle, and the storage error itself against the binary64
oracle, per voxel-size class of the 32-map batched mix (10 ticks per map)."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def d_error(gpu_export, orc_export, v):
    """max and rms |D - D_oracle| / v over the voxels the parity bar compares: W_o > 0 and W_o at
    least 1e-3 of the voxel's summed ray weights (outside the last 1/1000 of the drop-off ramp,
    where a 1e-7 m change of the binary32 distance moves the weight by a large relative amount)."""
    coords, dw = gpu_export
    oc, oD, oW, oM = orc_export[:4]
    assert np.array_equal(coords, oc)
    sel = (oW > 0) & (oW >= 1e-3 * oM)
    err = np.abs(dw[:, :, 0].astype(np.float64) - oD)[sel] / v
    return float(err.max()), float(np.sqrt(np.mean(err ** 2))), int(sel.sum())


@pytest.mark.parametrize("m", [0, 1, 2])      # voxel 0.02 / 0.05 / 0.10 m (map m of the mix)
def test_f16_storage_error_per_class(vbx, m):
    import synth
    T = 10
    w = synth.config4_map(m, n_ticks=T)
    P = dict(w.params, block_capacity=8192)
    v = float(np.float32(P["voxel_size"]))
    frames = [(w.frame(k), w.poses[k]) for k in range(T)]
    g16 = gpu_map(vbx, dict(P, storage="f16", keep_touches=False))
    g32 = gpu_map(vbx, dict(P, storage="f32", keep_touches=False))
    for p, pose in frames:
        d = dev(p)
        g16.integrate_frames([(d, pose, w.width)])
        g32.integrate_frames([(d, pose, w.width)])
    assert g16.sync() == 0 and g32.sync() == 0
    o16 = oracle_map(P, storage="f16")
    o64 = oracle_map(P, storage="f32")
    for p, pose in frames:
        o16.integrate(p, pose)
        o64.integrate(p, pose)
    e16 = o16.export()
    e64 = o64.export()
    # parity: binary16 GPU against the binary16-emulating oracle, binary32 GPU against binary64
    compare_export(g16.export(), e16, P, storage="f16")
    compare_export(g32.export(), e64, P, storage="f32")
    # the storage error itself: binary16 against the binary64 oracle
    mx16, rms16, n = d_error(g16.export(), e64, v)
    mx32, rms32, _ = d_error(g32.export(), e64, v)
    log(f"map {m} {w.width}x{w.height} v={v:g}: {n} weighted voxels; |D16 - D64|/v max {mx16:.3e} "
        f"rms {rms16:.3e}; |D32 - D64|/v max {mx32:.3e} rms {rms32:.3e}")
    # binary16 keeps D/delta (|D/delta| <= 1) with an 11-bit significand: one rounding per frame
    # is at most 2^-12 delta = 3 * 2^-12 v; ten frames of rounding stay well inside 10x that
    assert mx16 <= 10 * 3 * 2.0 ** -12
    assert mx32 <= 1e-4
