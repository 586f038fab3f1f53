"""Full-size workloads in the launch configuration the benchmark times, against the oracle:
the 50-sweep LiDAR street in one call (and at 0.05 m voxels, grown past 10^4 blocks), and the
32-map tick replayed from a captured graph.
Also the size limits of a call, which must be refused before anything runs."""
from concurrent.futures import ThreadPoolExecutor

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


def test_lidar_street_50_sweeps_one_call(vbx):
    import synth
    w = synth.config3(n_sweeps=50, cache=False)
    with ThreadPoolExecutor(max_workers=16) as ex:
        frames = list(ex.map(w.frame, range(50)))
    P = dict(w.params)
    log("c3 50 x 64x2048 simple const f32: GPU, one call")
    d = dev(np.stack(frames))
    g = gpu_map(vbx, dict(P, block_capacity=4096, keep_touches=False))
    g.integrate_frames([(d[k], w.poses[k], 2048) for k in range(50)])
    assert g.sync() == 0
    log("c3: oracle")
    o = oracle_map(P)
    for k in range(50):
        o.integrate(frames[k], w.poses[k])
    res = compare_export(g.export(), o.export(), P)
    log(f"  ok: {res}")
    st = g.stats()
    assert st["points"] == 50 * 64 * 2048 and st["blocks"] == res["blocks"]


def test_lidar_street_fine_voxels_grown_past_ten_thousand_blocks(vbx):
    """The street at 0.05 m voxels: the map grows past 10^4 blocks, sweep by sweep from a pool of
    256 blocks that the host doubles whenever a sweep finds it full (the sweep is then integrated
    again into the grown pool), and the final map equals the oracle's (block set bit-exact,
    constant weights bit-exact, D within the bar).  The block hash stays shallow."""
    import synth
    w = synth.config3(n_sweeps=50, cache=False)
    with ThreadPoolExecutor(max_workers=16) as ex:
        frames = list(ex.map(w.frame, range(50)))
    P = dict(w.params, voxel_size=0.05, trunc=0.15)
    d = dev(np.stack(frames))
    g = gpu_map(vbx, dict(P, block_capacity=256, keep_touches=False))
    cap, grown = 256, 0
    for k in range(50):
        g.integrate_frames([(d[k], w.poses[k], 2048)])
        while g.sync() == vbx.ERR_POOL_FULL:      # the map is as it was before the sweep
            cap *= 2
            g.reserve(cap)
            grown += 1
            g.integrate_frames([(d[k], w.poses[k], 2048)])
    h = g.hash_stats()
    log(f"c3 at 0.05 m: {h}, pool grown {grown} times to {cap} blocks")
    assert h["blocks"] > 10000 and h["blocks"] == g.num_blocks() and h["slots"] >= 2 * cap
    assert 1.0 <= h["mean_probe"] < 2.0 and h["max_probe"] < 64
    o = oracle_map(P)
    for k in range(50):
        o.integrate(frames[k], w.poses[k])
    res = compare_export(g.export(), o.export(), P)
    log(f"  ok: {res}")


def test_lidar_street_grouped(vbx):
    import synth
    w = synth.config3(n_sweeps=10, cache=False)
    frames = [w.frame(k) for k in range(10)]
    P = dict(w.params, merge="grouped")
    d = dev(np.stack(frames))
    g = gpu_map(vbx, dict(P, block_capacity=4096))
    g.integrate_frames([(d[k], w.poses[k], 2048) for k in range(10)])
    assert g.sync() == 0
    o = oracle_map(P)
    for k in range(10):
        o.integrate(frames[k], w.poses[k])
    res = compare_export(g.export(), o.export(), P)
    log(f"c3 grouped x10 ok: {res}")


@pytest.mark.parametrize("storage", ["f16", "s16", "f32"])
def test_32_map_tick_graph_replay_vs_oracle(vbx, storage):
    """Two ticks of the 32-map mix (8 x 160x120, 16 x 320x240, 8 x 640x480; voxel 0.02 / 0.05
    / 0.10 m), each tick one graph launch, every map against the oracle."""
    import synth
    T, M = 2, 32
    ws = [synth.config4_map(m, n_ticks=T, storage=storage) for m in range(M)]
    frames = [[ws[m].frame(k) for k in range(T)] for m in range(M)]
    maps = [gpu_map(vbx, dict(ws[m].params, block_capacity=4096, keep_touches=False)) for m in range(M)]
    devf = [[dev(frames[m][k]) for k in range(T)] for m in range(M)]
    tick = [[(devf[m][k], ws[m].poses[k], ws[m].width) for m in range(M)] for k in range(T)]
    g = vbx.Graph(maps, tick[0])
    for k in range(T):
        g.launch(tick[k])
    g.close()
    for m in range(M):
        assert maps[m].sync() == 0
    log(f"32-map tick {storage}: oracle")
    worst = 0.0
    for m in range(M):
        P = ws[m].params
        o = oracle_map(P)
        for k in range(T):
            o.integrate(frames[m][k], ws[m].poses[k])
        res = compare_export(maps[m].export(), o.export(), P, storage=storage)
        worst = max(worst, res["max_d_err_voxels"])
    log(f"  ok: 32 maps, worst |dD| = {worst:.2e} voxel")


def test_call_limits_are_refused_before_launch(vbx):
    params = dict(voxel_size=0.1, trunc=0.3, weighting="const", merge="simple")
    g = gpu_map(vbx, params)
    pose = np.eye(3, 4, dtype=np.float32)
    # one point more than a frame may hold (a real buffer of that size: nothing reads past it)
    big = torch.full(((1 << 24) + 1, 3), float("nan"), device="cuda")
    with pytest.raises(vbx.VbxError) as e:
        g.integrate(big, pose)
    assert e.value.status == -6
    del big
    # one frame more than a call may hold
    small = dev(np.full((4, 3), np.nan))
    with pytest.raises(vbx.VbxError) as e:
        g.integrate_frames([(small, pose)] * 4097)
    assert e.value.status == -6
    # a width that does not divide the point count
    with pytest.raises(vbx.VbxError) as e:
        g.integrate_frames([(small, pose, 3)])
    assert e.value.status == -1
    # a non-finite pose
    bad = pose.copy()
    bad[0, 3] = np.inf
    with pytest.raises(vbx.VbxError) as e:
        g.integrate(small, bad)
    assert e.value.status == -1
    # nothing ran, and the map still works
    assert g.sync() == 0 and g.num_blocks() == 0 and g.stats()["calls"] == 0
    g.integrate_frames([(small, pose)] * 4096)
    assert g.sync() == 0 and g.stats()["calls"] == 1 and g.stats()["invalid"] == 4 * 4096
