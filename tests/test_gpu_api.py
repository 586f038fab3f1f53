"""API-level guarantees of the GPU library, checked on the GPU through the C ABI."""
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


def same_export(a, b):
    ca, da = a.export()
    cb, db = b.export()
    return np.array_equal(ca, cb) and np.array_equal(da, db)


def room(w, h, n, seed):
    import synth
    poses, frame = synth.room_sequence(w, h, n, seed=synth.SEED_BASE + seed)
    return [(frame(k), poses[k]) for k in range(n)]


@pytest.mark.parametrize("storage", ["f32", "f16", "s16"])
@pytest.mark.parametrize("merge", ["simple", "grouped"])
def test_batch_equals_sequential(vbx, storage, merge):
    frames = room(320, 240, 5, 21)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge=merge, storage=storage,
                  w_max=2000.0)     # low cap so that saturation happens inside the batch
    seq = gpu_map(vbx, params)
    bat = gpu_map(vbx, params)
    bat2 = gpu_map(vbx, params)
    for p, pose in frames:
        seq.integrate(dev(p), pose)
    bat.integrate_frames([(dev(p), pose, 320) for p, pose in frames])
    bat2.integrate_batch([dev(p) for p, _ in frames], np.stack([q for _, q in frames]))
    assert seq.sync() == 0 and bat.sync() == 0 and bat2.sync() == 0
    assert same_export(seq, bat) and same_export(seq, bat2)
    o = oracle_map(params)
    for p, pose in frames:
        o.integrate(p, pose)
    compare_export(bat.export(), o.export(), params, storage=storage)


def test_multi_equals_alone(vbx):
    import synth
    specs = [(160, 120, 0.02), (320, 240, 0.05), (640, 480, 0.10), (320, 240, 0.02), (160, 120, 0.10)]
    alone, multi, frames = [], [], []
    for i, (w, h, v) in enumerate(specs):
        poses, frame = synth.room_sequence(w, h, 2, seed=synth.SEED_BASE + 100 + i, phase=0.3 * i)
        params = dict(voxel_size=v, trunc=3 * v, weighting="quad", merge="grouped", block_capacity=8192)
        frames.append([(frame(k), poses[k], w) for k in range(2)])
        alone.append(gpu_map(vbx, params))
        multi.append(gpu_map(vbx, params))
    for k in range(2):
        for i in range(len(specs)):
            p, pose, wd = frames[i][k]
            alone[i].integrate_frames([(dev(p), pose, wd)])
        vbx.integrate_multi(multi, [(dev(frames[i][k][0]), frames[i][k][1], frames[i][k][2])
                                    for i in range(len(specs))])
    for a, b in zip(alone, multi):
        assert a.sync() == 0 and b.sync() == 0
        assert same_export(a, b)
        ta, tb = a.last_touches(), b.last_touches()
        assert sorted(zip(map(tuple, ta[0].tolist()), ta[1].tolist())) == \
            sorted(zip(map(tuple, tb[0].tolist()), tb[1].tolist()))


def test_pool_full_leaves_map_unchanged_then_reserve(vbx):
    frames = room(160, 120, 2, 31)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", block_capacity=64)
    g = gpu_map(vbx, params)
    g.integrate(dev(frames[0][0][:200]), frames[0][1])        # a few blocks only
    assert g.sync() == 0
    before = g.export()
    nb = before[0].shape[0]
    assert 0 < nb < 64
    g.integrate(dev(frames[1][0]), frames[1][1])               # needs more than 64 blocks
    assert g.sync() == vbx.ERR_POOL_FULL
    after = g.export()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    g.integrate(dev(frames[0][0][:200]), frames[0][1])          # skipped while the error is set
    assert g.sync() == vbx.ERR_POOL_FULL
    assert np.array_equal(g.export()[1], before[1])
    g.reserve(4096)
    assert g.sync() == 0
    assert np.array_equal(g.export()[1], before[1])
    g.integrate(dev(frames[1][0]), frames[1][1])
    assert g.sync() == 0
    o = oracle_map(params)
    o.integrate(frames[0][0][:200], frames[0][1])
    o.integrate(frames[1][0], frames[1][1])
    compare_export(g.export(), o.export(), params)


def test_export_import_roundtrip(vbx):
    frames = room(320, 240, 4, 41)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped")
    a = gpu_map(vbx, params)
    for p, pose in frames[:3]:
        a.integrate(dev(p), pose)
    coords, dw = a.export()
    b = gpu_map(vbx, params)
    b.import_blocks(coords, dw)
    assert same_export(a, b)
    a.integrate(dev(frames[3][0]), frames[3][1])
    b.integrate(dev(frames[3][0]), frames[3][1])
    assert a.sync() == 0 and b.sync() == 0
    assert same_export(a, b)


def test_clear_and_reserve(vbx):
    frames = room(160, 120, 3, 51)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", block_capacity=2048)
    a = gpu_map(vbx, params)
    for p, pose in frames:
        a.integrate(dev(p), pose)
    a.clear()
    for p, pose in frames[:2]:
        a.integrate(dev(p), pose)
    a.reserve(6000)
    a.integrate(dev(frames[2][0]), frames[2][1])
    fresh = gpu_map(vbx, dict(params, block_capacity=8192))
    for p, pose in frames:
        fresh.integrate(dev(p), pose)
    assert a.sync() == 0 and fresh.sync() == 0
    assert same_export(a, fresh)
    assert a.stats()["calls"] == 3


def test_profile_records_every_stage(vbx):
    frames = room(160, 120, 2, 61)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped")
    a = gpu_map(vbx, params)
    a.profile(True)
    a.integrate_frames([(dev(p), pose, 160) for p, pose in frames])
    prof = a.profile_read()
    # raycasting counts its crossings in the cross stage: "bins" is projection mapping's
    for stage in ("points", "groups", "cross", "resolve", "commit", "scan", "scatter",
                  "update", "finish"):
        assert prof[stage][1] >= 1 and prof[stage][0] > 0, stage
    assert prof["bins"][1] == 0


def test_profile_of_selected_stages_only(vbx):
    """Timing only some stages records only those, leaves results unchanged, and a mask with a
    bit past the last stage is refused."""
    frames = room(160, 120, 2, 62)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped")
    a = gpu_map(vbx, params)
    b = gpu_map(vbx, params)
    a.profile(True, stages=["update", "points"])
    for m in (a, b):
        m.integrate_frames([(dev(p), pose, 160) for p, pose in frames])
    prof = a.profile_read()
    for stage, (ms, launches) in prof.items():
        if stage in ("update", "points"):
            assert launches == 1 and ms > 0, stage
        else:
            assert launches == 0 and ms == 0.0, stage
    assert same_export(a, b)
    L = vbx.lib()
    assert L.vbx_map_profile_stages(a.handle, 1 << vbx.PROFILE_STAGES) == vbx.ERR_INVALID_ARG
    a.profile(False)
    a.integrate_frames([(dev(p), pose, 160) for p, pose in frames])
    assert all(v[1] == 0 for v in a.profile_read().values())


def test_full_sequence_640x480x100_bench_configuration(vbx):
    """The benchmark workload at full size, in the launch configuration the benchmark times
    (one call over all 100 organised frames), against the oracle integrating frame by frame."""
    from concurrent.futures import ThreadPoolExecutor
    import synth
    w = synth.config2(n_frames=100)
    with ThreadPoolExecutor(max_workers=16) as ex:
        frames = list(ex.map(w.frame, range(100)))
    P = dict(w.params)
    log("c2 640x480x100 grouped quad f32: GPU")
    host = np.stack(frames)
    d = dev(host)
    g = gpu_map(vbx, dict(P, block_capacity=16384, keep_touches=False))
    g.integrate_frames([(d[k], w.poses[k], 640) for k in range(100)])
    assert g.sync() == 0
    log("c2: oracle")
    o = oracle_map(P)
    for k in range(100):
        o.integrate(frames[k], w.poses[k])
    res = compare_export(g.export(), o.export(), P)
    log(f"  ok: {res}")
    st = g.stats()
    assert st["points"] == 100 * 640 * 480


def test_grouped_tile_pairs_with_an_odd_tile_count(vbx):
    """A grouped call with more tiles than four times the waves the chip holds, so that the
    partial-group sort walks two tiles per wave, and an odd tile count, so that the last wave
    has one: 101 frames of 656x496 pixels (21 x 31 tiles each, the last tile column half
    full), eleven distinct frames in turn, against the oracle integrating them one by one."""
    import synth
    w, h, n_distinct, n = 656, 496, 11, 101
    tiles = ((w + 31) // 32) * ((h + 15) // 16) * n
    assert tiles % 2 == 1 and tiles >= 4 * 256 * 32 * 2
    poses, frame = synth.room_sequence(w, h, n_distinct, seed=synth.SEED_BASE + 91)
    frames = [frame(k) for k in range(n_distinct)]
    order = [k % n_distinct for k in range(n)]
    P = dict(voxel_size=0.05, trunc=0.15, max_range=5.0, weighting="quad", merge="grouped",
             block_capacity=16384, keep_touches=False)
    log(f"{n} x {w}x{h} grouped ({tiles} tiles): GPU")
    d = [dev(f) for f in frames]
    g = gpu_map(vbx, P)
    g.integrate_frames([(d[k], poses[k], w) for k in order])
    assert g.sync() == 0
    log("  oracle")
    o = oracle_map(P)
    for k in order:
        o.integrate(frames[k], poses[k])
    res = compare_export(g.export(), o.export(), P)
    log(f"  ok: {res}")
    assert g.stats()["points"] == n * w * h


def test_tuning_never_changes_results_and_autotune_leaves_map(vbx):
    frames = room(320, 240, 3, 71)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped")
    outs = []
    for split, columns, threads in vbx.TUNING_LIST:
        g = gpu_map(vbx, params)
        g.set_tuning(split, threads, columns)
        g.integrate_frames([(dev(p), pose, 320) for p, pose in frames])
        assert g.sync() == 0
        outs.append(g.export())
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    g = gpu_map(vbx, params)
    g.integrate(dev(frames[0][0]), frames[0][1])
    before = g.export()
    res = g.autotune([(dev(p), pose, 320) for p, pose in frames])
    best = res["best"]
    assert (best["update_split"], best["update_columns"], best["update_threads"]) in vbx.TUNING_LIST
    assert len(res["ms"]) == len(vbx.TUNING_LIST) and all(x > 0 for x in res["ms"])
    after = g.export()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    assert g.tuning() == res["best"]


def test_reused_map_and_scratch_repeat_bit_identical(vbx):
    """Repeated clear + integrate on one map (the benchmark's pattern: scratch tables reused
    across calls) gives the same map every time, equal to a fresh map's."""
    frames = room(640, 480, 8, 81)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped",
                  block_capacity=8192, keep_touches=False)
    batch = [(dev(p), pose, 640) for p, pose in frames]
    g = gpu_map(vbx, params)
    ref = None
    for rep in range(5):
        g.clear()
        g.integrate_frames(batch)
        assert g.sync() == 0
        out = g.export()
        if ref is None:
            ref = out
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), rep
    fresh = gpu_map(vbx, params)
    fresh.integrate_frames(batch)
    assert fresh.sync() == 0
    assert same_export(fresh, g)


class _TorchAllocator:
    """Allocator hook backed by torch's caching allocator; fails on request when told to."""

    def __init__(self):
        self.live = {}
        self.calls = 0
        self.fail_from = None      # the call index from which every request fails

    def alloc(self, n):
        self.calls += 1
        if self.fail_from is not None and self.calls >= self.fail_from:
            return 0
        p = torch.cuda.caching_allocator_alloc(n)
        self.live[p] = n
        return p

    def free(self, p):
        self.live.pop(p)
        torch.cuda.caching_allocator_delete(p)


def test_allocator_hook_owns_the_map_storage(vbx):
    """The hash table, block pool and device state come from the caller's allocator: the map
    integrates, grows (the old storage handed back) and is destroyed with every block returned;
    its result equals a default-allocated map's, bit for bit."""
    frames = room(320, 240, 3, 51)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped",
                  block_capacity=64, keep_touches=False)
    A = _TorchAllocator()
    kw = {k: v for k, v in params.items() if k != "keep_touches"}
    hooked = vbx.Map(**kw, allocator=(A.alloc, A.free))
    plain = gpu_map(vbx, params)
    assert len(A.live) == 4                      # state, hash keys, hash slots, pool
    for m in (hooked, plain):
        m.integrate(dev(frames[0][0]), frames[0][1])
        full = m.sync() == vbx.ERR_POOL_FULL
        m.reserve(4096)
        if full:
            m.integrate(dev(frames[0][0]), frames[0][1])
        for p, pose in frames[1:]:
            m.integrate(dev(p), pose)
        assert m.sync() == 0
    assert same_export(hooked, plain)
    assert len(A.live) == 4 and A.calls == 7     # the grown hash and pool replaced the old ones
    hooked.close()
    assert A.live == {}


def test_allocator_hook_failure_leaves_no_leak_and_the_map_usable(vbx):
    frames = room(160, 120, 2, 52)
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", block_capacity=256)
    # the pool (the fourth request) cannot be had: no map, and the three granted requests returned
    A = _TorchAllocator()
    A.fail_from = 4
    with pytest.raises(vbx.VbxError) as err:
        vbx.Map(**params, allocator=(A.alloc, A.free))
    assert err.value.status == vbx.ERR_OUT_OF_MEMORY and A.live == {}
    # growth that cannot be had: VBX_ERR_OUT_OF_MEMORY, and the map keeps its storage and content
    B = _TorchAllocator()
    m = vbx.Map(**params, allocator=(B.alloc, B.free))
    m.integrate(dev(frames[0][0]), frames[0][1])
    assert m.sync() == 0
    before = m.export()
    held = dict(B.live)
    B.fail_from = B.calls + 2                    # the new hash keys succeed, the slots do not
    with pytest.raises(vbx.VbxError) as err:
        m.reserve(8192)
    assert err.value.status == vbx.ERR_OUT_OF_MEMORY
    assert B.live == held
    after = m.export()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    m.integrate(dev(frames[1][0]), frames[1][1])
    assert m.sync() == 0
    o = oracle_map(params)
    for p, pose in frames:
        o.integrate(p, pose)
    compare_export(m.export(), o.export(), params)
    m.close()
    assert B.live == {}
