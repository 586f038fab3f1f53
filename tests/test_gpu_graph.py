"""Captured calls (HIP graphs): every replay must give the map the eager call gives, bit for
bit, including when eager work and host synchronisations run between the replays."""
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


# uneven clouds over maps of three voxel sizes, one frame per map per tick
SPECS = [(160, 120, 0.02), (320, 240, 0.05), (640, 480, 0.10), (320, 240, 0.02), (160, 120, 0.10)]


def tick_frames(n_ticks, seed):
    import synth
    out = []
    for i, (w, h, v) in enumerate(SPECS):
        poses, frame = synth.room_sequence(w, h, n_ticks, seed=synth.SEED_BASE + seed + i, phase=0.4 * i)
        out.append([(frame(k), poses[k], w) for k in range(n_ticks)])
    return out


@pytest.mark.parametrize("merge,storage", [("grouped", "f32"), ("grouped", "f16"), ("grouped", "s16"), ("simple", "f32")])
def test_graph_replays_equal_eager_multi(vbx, merge, storage):
    T = 3
    frames = tick_frames(T, 300)
    params = [dict(voxel_size=v, trunc=3 * v, weighting="quad", merge=merge, storage=storage,
                   block_capacity=8192) for (_, _, v) in SPECS]
    eager = [gpu_map(vbx, p) for p in params]
    graphed = [gpu_map(vbx, p) for p in params]
    # inputs of every tick live in their own buffers; the graph's frames are swapped per launch
    dev_frames = [[(dev(frames[i][k][0]), frames[i][k][1], frames[i][k][2]) for i in range(len(SPECS))]
                  for k in range(T)]
    g = vbx.Graph(graphed, dev_frames[0])
    scratch = torch.zeros(1 << 20, device="cuda")
    for k in range(T):
        log(f"graph {merge} {storage}: tick {k}")
        vbx.integrate_multi(eager, dev_frames[k])
        g.launch(dev_frames[k])
        # the program's own eager work and a host synchronisation between replays
        scratch.add_(1.0)
        torch.cuda.synchronize()
        for a, b in zip(eager, graphed):
            assert a.sync() == 0 and b.sync() == 0
            assert same_export(a, b), f"tick {k}"
            # touch records come out in completion order: compare them as multisets
            ta, tb = a.last_touches(), b.last_touches()
            assert sorted(zip(map(tuple, ta[0].tolist()), ta[1].tolist())) == \
                sorted(zip(map(tuple, tb[0].tolist()), tb[1].tolist()))
    # launching again without new frames integrates the last tick's frames a second time
    vbx.integrate_multi(eager, dev_frames[T - 1])
    g.launch()
    for a, b in zip(eager, graphed):
        assert a.sync() == 0 and b.sync() == 0
        assert same_export(a, b)
    g.close()
    # and the result is the oracle's
    o = oracle_map(params[1])
    for k in range(T):
        o.integrate(frames[1][k][0], frames[1][k][1])
    o.integrate(frames[1][T - 1][0], frames[1][T - 1][1])
    compare_export(graphed[1].export(), o.export(), params[1], storage=storage)


def test_graph_several_frames_per_map_equal_batch(vbx):
    import synth
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", block_capacity=8192)
    poses_a, fa = synth.room_sequence(320, 240, 3, seed=synth.SEED_BASE + 310)
    poses_b, fb = synth.room_sequence(160, 120, 3, seed=synth.SEED_BASE + 311, phase=1.0)
    A = [(dev(fa(k)), poses_a[k], 320) for k in range(3)]
    B = [(dev(fb(k)), poses_b[k], 160) for k in range(3)]
    frames = [A[0], B[0], A[1], B[1], B[2], A[2]]
    owner = [0, 1, 0, 1, 1, 0]
    ga, gb = gpu_map(vbx, params), gpu_map(vbx, params)
    g = vbx.Graph([ga, gb], frames, owner=owner)
    g.launch()
    g.launch()
    ea, eb = gpu_map(vbx, params), gpu_map(vbx, params)
    ea.integrate_frames(A + A)
    eb.integrate_frames(B + B)
    for a, b in ((ea, ga), (eb, gb)):
        assert a.sync() == 0 and b.sync() == 0
        assert same_export(a, b)
    g.close()


def test_graph_rejects_changed_shapes_and_moved_storage(vbx):
    import synth
    params = dict(voxel_size=0.05, trunc=0.15, weighting="quad", merge="grouped", block_capacity=2048)
    poses, frame = synth.room_sequence(160, 120, 2, seed=synth.SEED_BASE + 320)
    p0 = dev(frame(0))
    m = gpu_map(vbx, params)
    g = vbx.Graph([m], [(p0, poses[0], 160)])
    with pytest.raises(vbx.VbxError):
        g.launch([(p0[:1000], poses[0], 0)])              # another point count
    with pytest.raises(vbx.VbxError):
        g.launch([(p0, poses[0], 0)])                     # another organisation
    g.launch([(p0, poses[1], 160)])                       # a new pose is fine
    assert m.sync() == 0
    m.reserve(4096)                                       # storage reallocated
    with pytest.raises(vbx.VbxError):
        g.launch()
    g.close()
    g2 = vbx.Graph([m], [(p0, poses[0], 160)])
    g2.launch()
    assert m.sync() == 0
    g2.close()
    ref = gpu_map(vbx, params)
    ref.integrate_frames([(p0, poses[1], 160)])
    ref.integrate_frames([(p0, poses[0], 160)])
    assert ref.sync() == 0
    assert same_export(ref, m)
