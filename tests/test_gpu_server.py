"""The map server on the GPU: a map served in a mix of maps ends bit-identical to the same
frames integrated into it alone, in submission order, and matches the oracle integrating those
frames in that order; full pools grow and replay; admission respects the budget."""
import time

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


def same_export(a, b):
    ca, da = a.export()
    cb, db = b.export()
    return np.array_equal(ca, cb) and np.array_equal(da, db)


ROBOTS = [(160, 120, 0.02), (320, 240, 0.05), (640, 480, 0.10), (320, 240, 0.02), (160, 120, 0.05),
          (640, 480, 0.05)]


def robot_frames(n, seed, host=None):
    """Device frames per robot; host (a list, if given) receives the same frames on the host."""
    import synth
    out = []
    for i, (w, h, v) in enumerate(ROBOTS):
        poses, frame = synth.room_sequence(w, h, n, seed=synth.SEED_BASE + seed + i, phase=0.7 * i)
        out.append([(dev(frame(k)), poses[k], w) for k in range(n)])
        if host is not None:
            host.append([(frame(k), poses[k]) for k in range(n)])
    return out


def params_of(v, storage="f16", cap=4096):
    return dict(voxel_size=v, trunc=3 * v, weighting="quad", merge="grouped", storage=storage,
                block_capacity=cap)


@pytest.mark.parametrize("storage", ["f16", "s16", "f32"])
def test_mix_equals_alone(vbx, storage):
    n = 4
    host = []
    frames = robot_frames(n, 400, host)
    torch.cuda.synchronize()
    srv = vbx.Server(budget_bytes=64 << 30)
    ids = [srv.add_map(**params_of(v, storage)) for (_, _, v) in ROBOTS]
    rng = np.random.default_rng(5)
    order = [(i, k) for k in range(n) for i in range(len(ROBOTS))]
    # shuffle across robots but keep each robot's frames in order
    nxt = [0] * len(ROBOTS)
    seq = []
    while len(seq) < len(order):
        i = int(rng.integers(len(ROBOTS)))
        if nxt[i] < n:
            seq.append((i, nxt[i]))
            nxt[i] += 1
    tickets = []
    for j, (i, k) in enumerate(seq):
        p, pose, w = frames[i][k]
        tickets.append(srv.submit(ids[i], p, pose, w, t_arrival=vbx.Server.clock()))
        if j % 5 == 4:
            time.sleep(0.002)      # let several ticks form
    for t in tickets:
        st, td = srv.wait(t)
        assert st == 0
    srv.drain()
    s = srv.stats()
    log(f"server {storage}: {s['ticks']} ticks, {s['mean_frames_per_tick']:.2f} frames/tick, "
        f"p50 {s['p50_ms']:.3f} ms, p99 {s['p99_ms']:.3f} ms")
    assert s["completed"] == len(seq) and s["failed"] == 0 and s["ticks"] >= 1
    assert 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    for i, (_, _, v) in enumerate(ROBOTS):
        alone = gpu_map(vbx, params_of(v, storage))
        for k in range(n):
            alone.integrate_frames([frames[i][k]])
        assert alone.sync() == 0
        assert same_export(alone, srv.map(ids[i])), f"robot {i}"
        # the served map against the oracle, its frames in submission order (the oracle rounds
        # to the same storage after every frame)
        P = params_of(v, storage)
        o = oracle_map(P)
        for p, pose in host[i]:
            o.integrate(p, pose)
        compare_export(srv.map(ids[i]).export(), o.export(), P, storage=storage)
    srv.close()


def test_full_pool_grows_and_replays(vbx):
    frames = robot_frames(3, 410)
    torch.cuda.synchronize()
    srv = vbx.Server(budget_bytes=64 << 30, grow=True)
    ids = [srv.add_map(**params_of(v, "f16", cap=8)) for (_, _, v) in ROBOTS[:3]]
    tickets = [srv.submit(ids[i], *frames[i][k]) for k in range(3) for i in range(3)]
    for t in tickets:
        assert srv.wait(t)[0] == 0
    s = srv.stats()
    assert s["replays"] > 0 and s["failed"] == 0
    for i in range(3):
        alone = gpu_map(vbx, params_of(ROBOTS[i][2], "f16", cap=8192))
        for k in range(3):
            alone.integrate_frames([frames[i][k]])
        assert alone.sync() == 0
        assert same_export(alone, srv.map(ids[i])), f"robot {i}"
    srv.close()


def test_full_pool_without_growth_fails_requests_cleanly(vbx):
    frames = robot_frames(3, 420)
    torch.cuda.synchronize()
    srv = vbx.Server(budget_bytes=64 << 30, grow=False)
    mid = srv.add_map(**params_of(0.05, "f16", cap=40))
    # one small frame fits; the large frames overflow the pool and fail without effect
    small = (frames[0][0][0][:300], frames[0][0][1], 0)
    sub = [small, frames[1][0], small, frames[1][1], small]
    tickets = [srv.submit(mid, *f) for f in sub]
    status = [srv.wait(t)[0] for t in tickets]
    log(f"statuses {status}")
    assert status[1] == vbx.ERR_POOL_FULL and status[3] == vbx.ERR_POOL_FULL
    assert status[0] == 0 and status[2] == 0 and status[4] == 0
    alone = gpu_map(vbx, params_of(0.05, "f16", cap=40))
    for f, st in zip(sub, status):
        if st == 0:
            alone.integrate_frames([f])
    assert alone.sync() == 0
    assert same_export(alone, srv.map(mid))
    assert srv.stats()["failed"] == 2
    srv.close()


def test_admission_under_budget(vbx):
    import paper_1611_03631_amd as v
    srv = v.Server(budget_bytes=100 << 20)
    a = srv.add_map(**params_of(0.05, "f16", cap=4096))          # ~64 MiB pool
    with pytest.raises(v.VbxError) as e:
        srv.add_map(**params_of(0.05, "f16", cap=4096))          # would pass 100 MiB
    assert e.value.status == v.ERR_OUT_OF_MEMORY
    b = srv.add_map(**params_of(0.05, "f16", cap=512))
    s = srv.stats()
    assert (a, b) == (0, 1) and s["maps"] == 2 and s["rejected_maps"] == 1
    assert s["used_bytes"] <= s["budget_bytes"] == 100 << 20
    srv.close()
