#!/usr/bin/env python3
"""Throughput benchmark of TSDF integration on one MI355X.

Default workload (--workload c2): the 100-frame 640x480 depth sequence of a 10x10x3 m
furnished room (camera on a 1.5 m circle), voxel 0.05 m, truncation 0.15 m, 1/z^2 weighting
with drop-off, grouped raycasting, binary32 storage.  One step integrates the whole sequence
(one vbx_integrate_frames call over the 100 frames, organised 640-wide) into an emptied map;
the frames are resident in HBM before timing starts.

--workload c4: 32 maps per tick (8 x 160x120, 16 x 320x240, 8 x 640x480 depth frames, voxel
0.02 / 0.05 / 0.10 m by map, truncation 3 voxels, 1/z^2, grouped), one frame per map per
tick, binary16 storage; one step is one tick, replayed from a captured graph.  The eager
multi-map call and binary32 storage are timed beside it.

--workload c3: 50 sweeps of a 64x2048 LiDAR along a street (voxel 0.20 m, range 60 m, constant
weight, per-point raycasting), batched in one call; the same sweeps streamed one call each from
a 256-block pool that the host doubles whenever a sweep finds it full.

--workload accuracy: the accuracy evaluation (trilinear lookup of noise-free surface points in
maps built at voxel sizes 0.05 / 0.10 / 0.20 m with constant and 1/z^2 weighting) and the
rate of that distance query.

--workload c5: 64 robots (the four sensor classes above plus a 64x2048 LiDAR) send frames
as Poisson streams of 5-30 Hz each; a 10 s seeded trace is replayed in real time through
the map server, which batches whatever has arrived into each tick.  Reports served points/s
and arrival-to-completion latency percentiles.

Prints one JSON line: points/s as the value, voxel updates/s beside it, the roofline of the
dominant kernel stage (timed live with HIP events on the map's stream), and the CPU oracle
timed on a bounded sample of the same frames.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E vendor peak


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1611_03631_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def read_traffic(stage: str, sha: str, workload: str, tuning=None):
    """HBM bytes per launch of `stage` from committed rocprofv3 counter runs, if they were taken
    on the current kernel sources, on this workload and (where the file names one) with the
    same update variant (otherwise None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != sha or kv.get("workload") != workload:
        return None
    if "update_tuning" in kv:
        if tuning is None:
            return None
        if kv["update_tuning"] != f"{tuning['update_split']},{tuning['update_threads']},{tuning['update_columns']}":
            return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stage_roofline(prof, algo, steps, workload, tuning=None):
    """Roofline of the dominant stage among those with an algorithmic byte figure; `workload`
    (and the update variant `tuning`) select the counter runs that may supply the measured
    traffic."""
    dom = max(algo, key=lambda k: prof[k][0])
    ms_r, launches_r = prof[dom]
    per_launch_bytes = algo[dom] * steps / max(launches_r, 1)
    avg_launch_s = ms_r / max(launches_r, 1) / 1e3
    achieved = per_launch_bytes / avg_launch_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": read_traffic(dom, kernel_source_sha(), workload, tuning),
            "kernel_stage": dom, "launches_per_step": launches_r / steps,
            "avg_launch_ms": round(ms_r / max(launches_r, 1), 4),
            "algorithmic_bytes_per_launch": per_launch_bytes}


ALGO_STAGES = ("points", "update")   # stages with an algorithmic byte figure
BREAKDOWN_STEPS = 3


def stage_breakdown(m, step, candidates):
    """Per-stage times of a few untimed steps with every stage profiled, and the slowest of
    `candidates`.  Each profiled stage adds two event records per call, which cost the
    stream several microseconds each, so the timed steps afterwards profile only that stage."""
    m.profile(True)
    m.profile_read(reset=True)
    for _ in range(BREAKDOWN_STEPS):
        step()
    prof = m.profile_read(reset=True)
    m.profile(False)
    return prof, max(candidates, key=lambda k: prof[k][0])


def oracle_sample(w_list, budget_s, keep=False, keep_first=None):
    """Integrates frames of the given workloads in order with the single-threaded C oracle
    (binary64 values, no storage rounding) until the time budget is spent; returns (points,
    seconds of integration, frames done) and, with keep, the oracle's exports of the workloads
    it finished (None for the others, and for every workload after the first keep_first;
    exporting is not timed)."""
    import oracle
    pts = done = 0
    exports = []
    secs = 0.0
    for w, k_lo, k_hi in w_list:
        P = w.params
        om = oracle.OracleMap(P["voxel_size"], P["trunc"], weighting=P["weighting"],
                              merge=P["merge"], max_range=P["max_range"], storage="f32",
                              full_ray=P.get("full_ray", False))
        finished = True
        for k in range(k_lo, k_hi):
            if secs >= budget_s:
                finished = False
                break
            f = w.frame(k)
            t0 = time.perf_counter()
            om.integrate(f, w.poses[k])
            secs += time.perf_counter() - t0
            pts += f.shape[0]
            done += 1
        if keep:
            want = keep_first is None or len(exports) < keep_first
            exports.append(om.export() if finished and want else None)
        om.close()
        if secs >= budget_s:
            break
    return (pts, secs, done, exports) if keep else (pts, secs, done)


def host_cpu():
    """Model name of the host CPU and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "cores_available": avail}


def error_vs_oracle(np, gpu_export, orc_export, v, storage):
    """|D - D_oracle| / v over the voxels the GPU map holds as observed (W > 0), against the
    binary64 oracle on the same frames.  For binary32 storage, also the largest ratio to the
    parity bound the tests use (1e-4 v plus what the binary32 distance error can move D through
    the Eq. (5) ramp: 8 * 2^-24 (delta + v) (1 + 2 delta M / ((delta - v) W))); the 16-bit forms
    are held to 2e-3 v."""
    coords, dw = gpu_export
    oc, oD, oW, oM = orc_export[:4]
    if not np.array_equal(coords, oc):
        return {"error": "block sets differ"}
    W = dw[:, :, 1].astype(np.float64)
    sel = (W > 0) & (oW > 0)
    err = np.abs(dw[:, :, 0].astype(np.float64) - oD) / v
    e = err[sel]
    out = {"voxels": int(sel.sum()), "max_v": float(e.max(initial=0.0)),
           "rms_v": float(np.sqrt(np.mean(e ** 2))) if e.size else 0.0,
           "above_1e-4v": int((e > 1e-4).sum()), "above_2e-3v": int((e > 2e-3).sum())}
    if storage == "f32":
        return out
    out["bar_v"] = 2e-3
    out["meets_bar"] = bool(out["max_v"] <= 2e-3)
    return out


def bench_c2(args, np, torch, vbx, synth):
    w = synth.config2(n_frames=args.frames)
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        frames = list(ex.map(w.frame, range(w.n_frames)))
    gen_s = time.time() - t0
    host = np.stack(frames)                              # [F, N, 3] float32
    F, N = host.shape[0], host.shape[1]
    dev = torch.from_numpy(host).cuda()
    torch.cuda.synchronize()
    P = w.params
    stream = torch.cuda.current_stream()
    m = vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"],
                storage=args.storage, max_range=P["max_range"], block_capacity=16384,
                stream=stream)
    batch = [(dev[k], w.poses[k], w.width) for k in range(F)]
    frames_arr = vbx.make_frames(batch)
    L = vbx.lib()

    def step():
        L.vbx_map_clear(m.handle)
        rc = L.vbx_integrate_frames(m.handle, frames_arr, F)
        if rc != 0:
            raise vbx.VbxError(rc, "vbx_integrate_frames")

    # ---------------------------------------------------------------- tuning (untimed)
    tune = None
    if not args.no_autotune:
        tune = m.autotune(batch)
        tune["ms"] = [round(x, 4) for x in tune["ms"]]

    # ---------------------------------------------------------------- warm-up
    step()
    assert m.sync() == 0
    first_export = m.export()          # every step must rebuild exactly this map
    for _ in range(max(args.warmup - 1, 0)):
        step()
    assert m.sync() == 0
    prof_all, dom = stage_breakdown(m, step, ALGO_STAGES)
    m.profile(True, stages=[dom])
    m.profile_read(reset=True)

    # ---------------------------------------------------------------- timed
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t_wall = time.perf_counter()
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t_wall
    status = m.sync()
    if status != 0:
        raise vbx.VbxError(status, "device status after the timed steps")
    ms_total = ev0.elapsed_time(ev1)
    last_export = m.export()
    if not (np.array_equal(first_export[0], last_export[0]) and
            np.array_equal(first_export[1], last_export[1])):
        raise RuntimeError("the last timed step did not reproduce the first step's map bit-for-bit")
    prof = m.profile_read(reset=True)    # the dominant stage only, timed live
    m.profile(False)
    st = m.stats()           # the map was cleared before the last step: one step's counts
    ms_per_step = ms_total / args.steps
    points_per_step = F * N
    value = points_per_step / (ms_per_step / 1e3)
    vox_updates = st["touches"] / (ms_per_step / 1e3)

    # ---------------------------------------------------------------- roofline of the dominant stage
    s_v = 8 if args.storage == "f32" else 4
    algo = {   # algorithmic bytes per step of each stage with a defined figure
        "points": 12.0 * points_per_step + 48.0 * F,
        "update": 2.0 * s_v * st["cells"] + 4096.0 * s_v * st["new_blocks"],
    }
    roofline = stage_roofline(prof, algo, args.steps, w.name, m.tuning())
    whole = (algo["points"] + algo["update"]) / (ms_per_step / 1e3) / 1e9
    # the whole call: algorithmic bytes, and the HBM bytes the counters measured over all its
    # kernels (when taken on these sources, this workload and this update variant)
    call_traffic = read_traffic("call", kernel_source_sha(), w.name, m.tuning())
    whole_call = {"algorithmic_GBps": round(whole, 1), "algorithmic_frac": round(whole / HBM_PEAK_GBS, 4),
                  "measured_bytes_per_step": call_traffic,
                  "measured_GBps": None if call_traffic is None else round(call_traffic / (ms_per_step / 1e3) / 1e9, 1),
                  "measured_frac": None if call_traffic is None
                  else round(call_traffic / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                  "peak_GBps": HBM_PEAK_GBS}
    stages = {k: round(v[0] / BREAKDOWN_STEPS, 4) for k, v in prof_all.items()}

    # ---------------------------------------------------------------- forms compared on this GPU
    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    forms = {}
    form_exports = {"batched_" + args.storage: last_export}
    if not args.no_forms:
        plain = vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"],
                        storage="f32", max_range=P["max_range"], block_capacity=16384, stream=stream)
        pose_ptrs = [np.ascontiguousarray(w.poses[k], np.float32).reshape(12) for k in range(F)]

        def per_frame():      # one vbx_integrate call per frame, binary32 storage
            L.vbx_map_clear(plain.handle)
            for k in range(F):
                rc = L.vbx_integrate(plain.handle, dev[k].data_ptr(), N, pose_ptrs[k].ctypes.data)
                if rc != 0:
                    raise vbx.VbxError(rc, "vbx_integrate")
        forms["plain_per_frame_f32_ms"] = round(timed(per_frame, 3), 4)
        form_exports["plain_per_frame_f32"] = plain.export()
        forms["batched_" + args.storage + "_ms"] = round(ms_per_step, 4)
        form_exports["batched_" + args.storage] = last_export
        harr = vbx.make_frames(batch)
        for other in ("f32", "f16", "s16"):
            if other == args.storage:
                continue
            half = vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"],
                           storage=other, max_range=P["max_range"], block_capacity=16384, stream=stream)
            half.set_tuning(**m.tuning())

            def batched_other():
                L.vbx_map_clear(half.handle)
                rc = L.vbx_integrate_frames(half.handle, harr, F)
                if rc != 0:
                    raise vbx.VbxError(rc, "vbx_integrate_frames")
            forms["batched_" + other + "_ms"] = round(timed(batched_other, 5), 4)
            if half.sync() != 0:
                raise RuntimeError("device status after the compared forms")
            form_exports["batched_" + other] = half.export()
            half.close()
        for other in ("f16", "s16"):
            forms[f"batched_{other}_vs_plain_per_frame_f32"] = round(
                forms["plain_per_frame_f32_ms"] / forms[f"batched_{other}_ms"], 3)
        if plain.sync() != 0:
            raise RuntimeError("device status after the compared forms")
        plain.close()

    # ------------------------------------------- the other integration forms on the same frames
    variants = {}
    if not args.no_forms:
        def variant(tag, fn_make, reps=5):
            vm, run = fn_make()
            ms = timed(run, reps)
            if vm.sync() != 0:
                raise RuntimeError(f"device status after the {tag} form")
            vs = vm.stats()
            variants[tag] = {"ms_per_step": round(ms, 4), "points_per_s": round(F * N / (ms / 1e3), 1),
                             "blocks": vs["blocks"], "touches": vs["touches"]}
            vm.close()

        def make_map(**kw):
            return vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"],
                           storage="f32", max_range=P["max_range"], stream=stream, **kw)

        def projective():      # projection mapping (Sec. IV-B) of the same frames
            vm = make_map(block_capacity=16384)
            K = np.array([100.0 * w.width / 160.0, 100.0 * w.width / 160.0, w.width / 2.0, w.height / 2.0],
                         np.float32)
            arr = vbx.make_frames(batch)

            def run():
                L.vbx_map_clear(vm.handle)
                rc = L.vbx_integrate_projective(vm.handle, arr, F, K.ctypes.data)
                if rc != 0:
                    raise vbx.VbxError(rc, "vbx_integrate_projective")
            return vm, run
        variant("projective_f32", projective)

        def full_ray():        # raycasting from the sensor (free space carved), grouped
            vm = make_map(block_capacity=65536, full_ray=True)
            vm.set_tuning(**m.tuning())
            arr = vbx.make_frames(batch)

            def run():
                L.vbx_map_clear(vm.handle)
                rc = L.vbx_integrate_frames(vm.handle, arr, F)
                if rc != 0:
                    raise vbx.VbxError(rc, "vbx_integrate_frames")
            return vm, run
        variant("full_ray_grouped_f32", full_ray, reps=3)

        cols = [torch.from_numpy(synth.point_colors(frames[k], w.poses[k], synth.SEED_BASE + 1, k).view(np.int32)).cuda()
                for k in range(F)]

        def color():           # colour fused with the distances (Sec. IV-B), grouped
            vm = make_map(block_capacity=16384, color=True)
            vm.set_tuning(**m.tuning())
            arr = vbx.make_frames([(dev[k], w.poses[k], w.width, cols[k]) for k in range(F)])

            def run():
                L.vbx_map_clear(vm.handle)
                rc = L.vbx_integrate_frames(vm.handle, arr, F)
                if rc != 0:
                    raise vbx.VbxError(rc, "vbx_integrate_frames")
            return vm, run
        variant("color_grouped_f32", color)

    # ---------------------------------------------------------------- CPU oracle sample
    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        wo = synth.config2(n_frames=args.frames)
        wo.frame_fn = lambda k: frames[k]
        pts, cpu_s, done, oexp = oracle_sample([(wo, 0, F)], args.cpu_seconds, keep=True)
        cpu = {"value": round(pts / cpu_s, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"first {done} of {F} frames of the same sequence, integrated in order "
                         f"by the single-threaded C oracle in binary64 ({cpu_s:.1f} s)"}
        if oexp[0] is not None:
            # every compared form holds the whole sequence: check each against the oracle's map
            v = float(np.float32(P["voxel_size"]))
            accuracy = {k: error_vs_oracle(np, e, oexp[0], v, k.split("_")[-1])
                        for k, e in form_exports.items()}

    return {
        "metric": "points/s & voxel-updates/s TSDF integration; p50/p99 frame latency (served)",
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else args.storage + "-storage/f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {F} frames x {w.width}x{w.height} depth, furnished "
                               "10x10x3 m room, voxel 0.05 m, truncation 0.15 m, 1/z^2 weighting, "
                               f"grouped raycasting, {args.storage} storage",
                   "frames": F, "points_per_frame": N, "storage": args.storage},
        "voxel_updates_per_s": round(vox_updates, 1),
        "touches_per_step": st["touches"],
        "rays_per_step": st["rays"],
        "blocks": st["blocks"],
        "whole_step_algorithmic_GBps": round(whole, 1),
        "whole_call_hbm": whole_call,
        "stage_ms_per_step": stages,
        "forms_ms_per_step": forms,
        "other_forms": variants,
        "error_vs_binary64_oracle": accuracy,
        "wall_s": round(wall_s, 3),
        "repeat_bit_identical": True,
        "tuning": m.tuning(),
        "autotune": tune,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "input_generation_s": round(gen_s, 1),
        "kernel_source_sha": kernel_source_sha(),
    }


C4_CAPACITY = {0.02: 16384, 0.05: 4096, 0.10: 2048}
ERR_TICKS = 10   # c4: ticks integrated from empty maps for the error against the oracle


def bench_c4(args, np, torch, vbx, synth):
    T = args.ticks
    M = 32
    ws = [synth.config4_map(m, n_ticks=T) for m in range(M)]
    t0 = time.time()
    jobs = [(m, k) for m in range(M) for k in range(T)]
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        flat = list(ex.map(lambda mk: ws[mk[0]].frame(mk[1]), jobs))
    gen_s = time.time() - t0
    dev = []
    for m in range(M):
        dev.append(torch.from_numpy(np.stack(flat[m * T:(m + 1) * T])).cuda())
    del flat
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    pts_tick = sum(int(d.shape[1]) for d in dev)

    def tick(k):
        return [(dev[m][k], ws[m].poses[k], ws[m].width) for m in range(M)]

    def make_maps(storage):
        out = []
        for m in range(M):
            P = ws[m].params
            out.append(vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"],
                               storage=storage, max_range=P["max_range"],
                               block_capacity=C4_CAPACITY[round(P["voxel_size"], 2)], stream=stream))
        return out

    def clear(maps):
        for mp in maps:
            mp.clear()

    def run(maps, graph, steps, warm):
        """warm + steps ticks from emptied maps; returns ms per timed tick."""
        clear(maps)
        for k in range(warm):
            graph.launch(tick(k % T)) if graph else vbx.integrate_multi(maps, tick(k % T))
        clear(maps)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(steps):
            graph.launch(tick(k % T)) if graph else vbx.integrate_multi(maps, tick(k % T))
        e1.record(stream)
        torch.cuda.synchronize()
        for mp in maps:
            st = mp.sync()
            if st != 0:
                raise vbx.VbxError(st, "device status after the timed ticks")
        return e0.elapsed_time(e1) / steps

    results = {}
    err_maps = (0, 1, 2)          # one map per voxel class (0.02 / 0.05 / 0.10 m)
    err_exports = {}
    for storage in ("f16", "s16", "f32"):
        maps = make_maps(storage)
        # launch tuning: one graph per update variant, a few ticks each (untimed)
        tune = None
        if not args.no_autotune:
            tune = {}
            for split, columns, threads in vbx.TUNING_LIST:
                maps[0].set_tuning(split, threads, columns)
                g = vbx.Graph(maps, tick(0))
                tune[f"{split}{'c' if columns else 'z'}x{threads}"] = round(run(maps, g, 5, 2), 4)
                g.close()
            best = min(tune, key=tune.get)
            sc, th = best.split("x")
            maps[0].set_tuning(int(sc[:-1]), int(th), 1 if sc[-1] == "c" else 0)
        g = vbx.Graph(maps, tick(0))
        ms_graph = run(maps, g, args.steps, args.warmup)
        ref = [maps[i].export() for i in (0, 3, 17)]
        stats = [mp.stats() for mp in maps]
        ms_eager = run(maps, None, args.steps, args.warmup)
        for j, i in enumerate((0, 3, 17)):
            e = maps[i].export()
            if not (np.array_equal(e[0], ref[j][0]) and np.array_equal(e[1], ref[j][1])):
                raise RuntimeError("graph replay and eager calls built different maps")
        # stage profile of a few eager ticks (the graph replays the same kernels)
        clear(maps)
        maps[0].profile(True)
        maps[0].profile_read(reset=True)
        n_prof = min(args.steps, 10)
        before = [mp.stats() for mp in maps]
        for k in range(n_prof):
            vbx.integrate_multi(maps, tick(k % T))
        torch.cuda.synchronize()
        prof = maps[0].profile_read(reset=True)
        maps[0].profile(False)
        after = [mp.stats() for mp in maps]
        # the maps after ERR_TICKS ticks from empty, for the error against the binary64 oracle
        clear(maps)
        for k in range(ERR_TICKS):
            vbx.integrate_multi(maps, tick(k % T))
        for mp in maps:
            if mp.sync() != 0:
                raise RuntimeError("device status after the error ticks")
        err_exports[storage] = {i: maps[i].export() for i in err_maps}
        cells = sum(a["cells"] - b["cells"] for a, b in zip(after, before))
        new_blocks = sum(a["new_blocks"] - b["new_blocks"] for a, b in zip(after, before))
        s_v = 8 if storage == "f32" else 4
        algo = {"points": (12.0 * pts_tick + 48.0 * M) * n_prof,
                "update": 2.0 * s_v * cells + 4096.0 * s_v * new_blocks}
        algo = {k: v / n_prof for k, v in algo.items()}
        results[storage] = {
            "ms_per_tick_graph": round(ms_graph, 4), "ms_per_tick_eager": round(ms_eager, 4),
            "points_per_s": round(pts_tick / (ms_graph / 1e3), 1),
            "voxel_updates_per_s": round(sum(s["touches"] for s in stats) / args.steps / (ms_graph / 1e3), 1),
            "blocks_per_class": {f"v{v}": sum(stats[m]["blocks"] for m in range(M)
                                               if abs(ws[m].params["voxel_size"] - v) < 1e-6)
                                 for v in synth.MULTI_VOXEL},
            "stage_ms_per_tick": {k: round(v[0] / n_prof, 4) for k, v in prof.items()},
            "roofline": stage_roofline(prof, algo, n_prof, f"c4_multi_map_{storage}", maps[0].tuning()),
            "tuning": maps[0].tuning(), "autotune": tune}
        g.close()
        for mp in maps:
            mp.close()
        del maps
    main_r = results["f16"]
    ms = main_r["ms_per_tick_graph"]
    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        # maps in order (err_maps first), ERR_TICKS ticks each, until the budget is spent
        order = list(err_maps) + [m for m in range(M) if m not in err_maps]
        sample = [(ws[m], 0, ERR_TICKS) for m in order]
        pts, cpu_s, done, oexp = oracle_sample(sample, args.cpu_seconds, keep=True,
                                               keep_first=len(err_maps))
        cpu = {"value": round(pts / cpu_s, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"the first {ERR_TICKS} ticks of the maps in turn (maps {list(err_maps)}, "
                         f"one per voxel class, first): {done} frames integrated by the "
                         f"single-threaded C oracle in binary64 ({cpu_s:.1f} s)"}
        accuracy = {}
        for storage, ex in err_exports.items():
            for j, i in enumerate(err_maps):
                if oexp[j] is None:
                    continue
                v = float(np.float32(ws[i].params["voxel_size"]))
                accuracy[f"{storage}_v{ws[i].params['voxel_size']:g}"] = error_vs_oracle(
                    np, ex[i], oexp[j], v, storage)
    return {
        "metric": "points/s & voxel-updates/s TSDF integration; p50/p99 frame latency (served)",
        "value": main_r["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32",
        "data": "synthetic",
        "config": {"workload": f"c4_multi_map: {M} maps per tick (8x160x120, 16x320x240, 8x640x480 "
                               "depth), voxel 0.02/0.05/0.10 m, truncation 3 voxels, 1/z^2, grouped, "
                               "f16 storage, one captured graph per tick",
                   "maps": M, "points_per_tick": pts_tick, "ticks": T},
        "voxel_updates_per_s": main_r["voxel_updates_per_s"],
        "graph_vs_eager_speedup": round(main_r["ms_per_tick_eager"] / ms, 3),
        "f16_vs_f32_speedup": round(results["f32"]["ms_per_tick_graph"] / ms, 3),
        "s16_vs_f32_speedup": round(results["f32"]["ms_per_tick_graph"] /
                                    results["s16"]["ms_per_tick_graph"], 3),
        "error_vs_binary64_oracle": accuracy,
        "storage": results,
        "repeat_bit_identical": True,
        "roofline": main_r["roofline"],
        "cpu_baseline": cpu,
        "input_generation_s": round(gen_s, 1),
        "kernel_source_sha": kernel_source_sha(),
    }


C3_INITIAL_CAPACITY = 256   # blocks: the streamed sweeps grow the pool several times


def bench_c3(args, np, torch, vbx, synth):
    """50 LiDAR sweeps along a street: batched into one call, and streamed sweep by sweep from
    a small pool that the host grows (vbx_map_reserve) whenever it fills.  With --full-ray every
    ray is walked from the sensor to the truncation distance behind its point (the free space is
    carved too), and the map grows to tens of thousands of blocks."""
    S = 50
    w = synth.config3(n_sweeps=S)
    if args.full_ray:
        w.params = dict(w.params, full_ray=True)
    if args.voxel:
        # a finer map of the same street: truncation three voxels, as in the other workloads
        w.params = dict(w.params, voxel_size=args.voxel, trunc=3.0 * args.voxel)
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        frames = list(ex.map(w.frame, range(S)))
    gen_s = time.time() - t0
    dev = torch.from_numpy(np.stack(frames)).cuda()
    torch.cuda.synchronize()
    P = w.params
    stream = torch.cuda.current_stream()
    N = int(dev.shape[1])
    batch = [(dev[k], w.poses[k], w.width) for k in range(S)]
    L = vbx.lib()

    full = bool(P.get("full_ray", False))
    # streamed: one call per sweep, pool doubled by the host when a sweep finds it full
    m = vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"], storage="f32",
                max_range=P["max_range"], block_capacity=C3_INITIAL_CAPACITY, stream=stream, full_ray=full)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    rehash = 0
    t_wall = time.perf_counter()
    e0.record(stream)
    for k in range(S):
        m.integrate_frames([batch[k]])
        if m.sync() == vbx.ERR_POOL_FULL:         # the map is as it was before the sweep
            cap = m.params["block_capacity"] * 2
            while True:
                m.reserve(cap)
                m.params["block_capacity"] = cap
                rehash += 1
                m.integrate_frames([batch[k]])
                if m.sync() != vbx.ERR_POOL_FULL:
                    break
                cap *= 2
    e1.record(stream)
    torch.cuda.synchronize()
    stream_wall = time.perf_counter() - t_wall
    stream_ms = e0.elapsed_time(e1)
    st_stream = m.stats()
    hash_stream = m.hash_stats()
    ref = m.export()
    cap = m.params["block_capacity"]
    m.close()

    # batched: the whole sequence in one call into a pool of the final size
    b = vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"], storage="f32",
                max_range=P["max_range"], block_capacity=cap, stream=stream, full_ray=full)
    arr = vbx.make_frames(batch)

    def step():
        L.vbx_map_clear(b.handle)
        rc = L.vbx_integrate_frames(b.handle, arr, S)
        if rc != 0:
            raise vbx.VbxError(rc, "vbx_integrate_frames")
    tune = None
    if not args.no_autotune:
        tune = b.autotune(batch)
        tune["ms"] = [round(x, 4) for x in tune["ms"]]
    for _ in range(max(args.warmup, 1)):
        step()
    if b.sync() != 0:
        raise RuntimeError("device status after warm-up")
    out_b = b.export()
    if not (np.array_equal(out_b[0], ref[0]) and np.array_equal(out_b[1], ref[1])):
        raise RuntimeError("batched sweeps and streamed sweeps built different maps")
    prof_all, dom = stage_breakdown(b, step, ALGO_STAGES)
    b.profile(True, stages=[dom])
    b.profile_read(reset=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    if b.sync() != 0:
        raise RuntimeError("device status after the timed steps")
    ms = e0.elapsed_time(e1) / args.steps
    prof = b.profile_read(reset=True)
    b.profile(False)
    st = b.stats()
    hstats = b.hash_stats()
    tuning = b.tuning()
    b.close()
    algo = {"points": 12.0 * S * N + 48.0 * S,
            "update": 2.0 * 8 * st["cells"] + 4096.0 * 8 * st["new_blocks"]}
    cpu = None
    if not args.no_cpu_baseline:
        w.frame_fn = lambda k: frames[k]
        pts, cpu_s, done = oracle_sample([(w, 0, S)], args.cpu_seconds)
        cpu = {"value": round(pts / cpu_s, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"first {done} of {S} sweeps in order by the single-threaded C oracle ({cpu_s:.1f} s)"}
    return {
        "metric": "points/s & voxel-updates/s TSDF integration; p50/p99 frame latency (served)",
        "value": round(S * N / (ms / 1e3), 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {S} sweeps of a 64x2048 LiDAR along a street, "
                               f"voxel {P['voxel_size']:g} m, truncation {P['trunc']:g} m, range 60 m, "
                               "constant weight, per-point raycasting"
                               + (" of the whole ray from the sensor" if full else " of the truncation band")
                               + ", f32",
                   "sweeps": S, "points_per_sweep": N, "full_ray": full, "voxel_size": P["voxel_size"]},
        "voxel_updates_per_s": round(st["touches"] / (ms / 1e3), 1),
        "blocks": st["blocks"],
        "blocks_allocated_per_s": round(st["new_blocks"] / (ms / 1e3), 1),
        "block_hash": {"batched": hstats, "streamed": hash_stream},
        "streamed": {"ms_total": round(stream_ms, 3), "wall_s": round(stream_wall, 3),
                     "rehashes": rehash, "initial_capacity": C3_INITIAL_CAPACITY, "final_capacity": cap,
                     "points_per_s": round(S * N / (stream_ms / 1e3), 1),
                     "blocks": st_stream["blocks"]},
        "stage_ms_per_step": {k: round(v[0] / BREAKDOWN_STEPS, 4) for k, v in prof_all.items()},
        "repeat_bit_identical": True,
        "tuning": tuning,
        "autotune": tune,
        "roofline": stage_roofline(prof, algo, args.steps, w.name, tuning),
        "cpu_baseline": cpu,
        "input_generation_s": round(gen_s, 1),
        "kernel_source_sha": kernel_source_sha(),
    }


C5_CLASSES = (("depth", 160, 120, 0.02), ("depth", 320, 240, 0.05), ("depth", 640, 480, 0.10),
              ("lidar", 2048, 64, 0.20))
C5_CAPACITY = {0.02: 4096, 0.05: 1024, 0.10: 512, 0.20: 16384}


def bench_c5(args, np, torch, vbx, synth):
    """64 robots served from one device: seeded open-loop Poisson trace replayed in real time."""
    R = 64
    K = 8                                   # distinct frames per robot, cycled
    seed = synth.SEED_BASE + 5
    rng = np.random.default_rng(seed)
    rates = rng.uniform(5.0, 30.0, size=R) * args.load
    trace = []
    for i in range(R):
        t = rng.exponential(1.0 / rates[i])
        j = 0
        while t < args.duration:
            trace.append((t, i, j))
            j += 1
            t += rng.exponential(1.0 / rates[i])
    trace.sort()
    robots = []
    for i in range(R):
        kind, w, h, v = C5_CLASSES[i % 4]
        if kind == "depth":
            poses, frame = synth.room_sequence(w, h, K, seed=seed + 1000 * (i + 1), phase=2.0 * np.pi * i / R)
            params = dict(voxel_size=v, trunc=3 * v, weighting="quad", merge="grouped", storage="f16",
                          max_range=5.0, block_capacity=C5_CAPACITY[v])
        else:
            wl = synth.config3(n_sweeps=K, seed=seed + 1000 * (i + 1), cache=False)
            poses, frame = wl.poses, wl.frame_fn
            params = dict(voxel_size=v, trunc=3 * v, weighting="const", merge="grouped", storage="f16",
                          max_range=60.0, block_capacity=C5_CAPACITY[v])
        robots.append((kind, w, h, params, poses, frame))
    t0 = time.time()
    jobs = [(i, k) for i in range(R) for k in range(K)]
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        flat = list(ex.map(lambda ik: robots[ik[0]][5](ik[1]), jobs))
    gen_s = time.time() - t0
    dev = [torch.from_numpy(np.stack(flat[i * K:(i + 1) * K])).cuda() for i in range(R)]
    torch.cuda.synchronize()

    srv = vbx.Server(budget_bytes=200 * 10**9, grow=True)
    ids = []
    rejected = 0
    for i in range(R):
        try:
            ids.append(srv.add_map(**robots[i][3]))
        except vbx.VbxError:
            ids.append(None)
            rejected += 1

    def submit(i, j, t_arr):
        k = j % K
        srv.submit(ids[i], dev[i][k], robots[i][4][k], robots[i][1], t_arrival=t_arr)

    # warm-up: one frame per admitted robot (scratch growth, first touch), then reset
    for i in range(R):
        if ids[i] is not None:
            submit(i, 0, 0.0)
    srv.drain()
    srv.reset_stats()

    # real-time replay of the trace; arrival times are the trace's, so submitter lateness
    # counts as latency
    clock = vbx.Server.clock
    start = clock() + 0.2
    late = 0.0
    for t, i, j in trace:
        if ids[i] is None:
            continue
        due = start + t
        while True:
            now = clock()
            if now >= due:
                break
            if due - now > 0.002:
                time.sleep(due - now - 0.001)
        late = max(late, clock() - due)
        submit(i, j, due)
    srv.drain()
    st = srv.stats()
    offered_pts = sum(int(dev[i].shape[1]) for _, i, _ in trace if ids[i] is not None)
    # a robot served in the mix equals its frames integrated alone, in order
    identical = True
    for i in (2, 3):
        if ids[i] is None:
            continue
        seq = [(t, j) for t, ii, j in trace if ii == i]
        alone = vbx.Map(**robots[i][3])
        alone.integrate_frames([(dev[i][0], robots[i][4][0], robots[i][1])])      # the warm-up frame
        for _, j in seq:
            alone.integrate_frames([(dev[i][j % K], robots[i][4][j % K], robots[i][1])])
        assert alone.sync() == 0
        a = alone.export()
        b = srv.map(ids[i]).export()
        identical = identical and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        alone.close()
    srv.close()
    if not identical:
        raise RuntimeError("a served map differs from the same frames integrated alone")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        pts = 0
        t1 = time.perf_counter()
        for t, i, j in trace:
            if time.perf_counter() - t1 >= args.cpu_seconds:
                break
            P = robots[i][3]
            om = oracle.OracleMap(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"],
                                  max_range=P["max_range"], storage="f16")
            f = flat[i * K + j % K]
            om.integrate(f, robots[i][4][j % K])
            pts += f.shape[0]
            om.close()
        cpu_s = time.perf_counter() - t1
        cpu = {"value": round(pts / cpu_s, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu(),
               "sample": f"the trace's first requests, each into a fresh map, by the single-threaded C "
                         f"oracle in binary16-emulating mode ({cpu_s:.1f} s)"}
    return {
        "metric": "points/s & voxel-updates/s TSDF integration; p50/p99 frame latency (served)",
        "value": round(st["points_per_s"], 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": int(st["completed"]),
        "warmup": R - rejected,
        "ms_per_step": round(st["mean_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32",
        "data": "synthetic",
        "config": {"workload": f"c5_served: {R} robots, Poisson U(5,30) Hz each"
                               + (f" x {args.load:g}" if args.load != 1.0 else "") + f", {args.duration:g} s "
                               "open-loop trace in real time; 160x120 / 320x240 / 640x480 depth and "
                               "64x2048 LiDAR at voxel 0.02 / 0.05 / 0.10 / 0.20 m; f16; 200 GB budget",
                   "robots": R, "requests": len(trace), "duration_s": args.duration, "load": args.load},
        "latency_ms": {"p50": round(st["p50_ms"], 4), "p99": round(st["p99_ms"], 4),
                       "max": round(st["max_ms"], 4), "mean": round(st["mean_ms"], 4)},
        "offered_points_per_s": round(offered_pts / args.duration, 1),
        "served": {k: st[k] for k in ("completed", "failed", "ticks", "replays", "maps", "rejected_maps",
                                      "used_bytes", "budget_bytes")},
        "mean_frames_per_tick": round(st["mean_frames_per_tick"], 3),
        "max_submit_lateness_ms": round(late * 1e3, 3),
        "mix_equals_alone": identical,
        "roofline": None,
        "cpu_baseline": cpu,
        "input_generation_s": round(gen_s, 1),
        "kernel_source_sha": kernel_source_sha(),
    }


def bench_accuracy(args, np, torch, vbx, synth):
    """The accuracy evaluation of Sec. VI-A on synthetic ground truth, and the query's speed.

    A 40-frame 320x240 sequence of the furnished room (the C2 camera path and depth noise) is
    integrated at voxel sizes 0.05, 0.10 and 0.20 m with truncation 4 v (as in that
    evaluation), grouped raycasting, constant and 1/z^2 weighting.  The exact surface points
    of the same frames (no noise, no dropouts) are then looked up by trilinear interpolation;
    the error of a known point is |distance| capped at the truncation distance.  The value
    reported is the query rate of the largest map on 2^24 such points, timed with HIP events
    on the map's stream."""
    F, Wd, Hd = 40, 320, 240
    seed = synth.SEED_BASE + 1
    poses, frame = synth.room_sequence(Wd, Hd, F, seed)
    _, frame_gt = synth.room_sequence(Wd, Hd, F, seed, invalid_rate=0.0, noise_scale=0.0)
    frames = [frame(k) for k in range(F)]
    gt = []
    for k in range(F):
        P = frame_gt(k).astype(np.float64)
        T = poses[k].astype(np.float64)
        gt.append(P[np.all(np.isfinite(P), axis=1)] @ T[:, :3].T + T[:, 3])
    gt = np.concatenate(gt).astype(np.float32)
    rng = np.random.default_rng(seed)
    gt = gt[rng.choice(gt.shape[0], size=min(1 << 20, gt.shape[0]), replace=False)]
    dev_frames = [torch.from_numpy(f).cuda() for f in frames]
    q = torch.from_numpy(gt).cuda()
    stream = torch.cuda.current_stream()
    table = {}
    big = None
    for v in (0.05, 0.10, 0.20):
        row = {}
        for weighting in ("const", "quad"):
            m = vbx.Map(v, 4 * v, weighting=weighting, merge="grouped", max_range=5.0,
                        block_capacity=65536, stream=stream)
            m.integrate_frames([(dev_frames[k], poses[k], Wd) for k in range(F)])
            d = m.interpolate(q)
            if m.sync() != 0:
                raise vbx.VbxError(m.sync(), "accuracy map")
            dist = d.cpu().numpy().astype(np.float64)
            known = np.isfinite(dist)
            err = np.minimum(np.abs(dist[known]), 4 * v)     # error capped at the truncation
            row[weighting] = {"mean_m": round(float(err.mean()), 6),
                              "rms_m": round(float(np.sqrt(np.mean(err * err))), 6),
                              "known": int(known.sum()), "of": int(dist.size)}
            if v == 0.05 and weighting == "quad":
                big = m
        table[f"v{v:.2f}"] = row
    # query speed: 2^24 ground-truth points (the sample repeated) on the 0.05 m map
    nq = 1 << 24
    reps = (nq + q.shape[0] - 1) // q.shape[0]
    qq = q.repeat(reps, 1)[:nq].contiguous()
    for _ in range(args.warmup):
        big.interpolate(qq)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        big.interpolate(qq)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    rate = nq / (ms * 1e-3)
    algo = 12 + 4 + 8 * 8          # query in, distance out, eight corner voxels (binary32 D, W)
    achieved = algo * nq / (ms * 1e-3) / 1e9
    return {
        "metric": "trilinear distance queries/s (accuracy evaluation)",
        "value": round(rate, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"accuracy_room_{Wd}x{Hd}x{F}: voxel 0.05/0.10/0.20 m, truncation 4 v, "
                               "grouped, const and 1/z^2 weighting; ground truth = noise-free surface "
                               "points of the same frames", "queries_per_step": nq},
        "accuracy": table,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(achieved / 8000.0, 4), "traffic": None,
                     "kernel_stage": "interpolate", "algorithmic_bytes_per_query": algo},
        "kernel_source_sha": kernel_source_sha(),
    }


def bench_esdf(args, np, torch, vbx, synth):
    """The ESDF layer (Sec. V-A): its update rate on the furnished-room map of the default
    workload (batch from the whole 100-frame TSDF, and incrementally after every frame), and the
    simulated ESDF benchmark of Sec. VI-B (error against the scene's exact distance field for a
    one-voxel band, a band of half the truncation distance, and occupancy)."""
    stream = torch.cuda.current_stream()
    # ---------------------------------------------------------------- rate on the C2 room map
    w = synth.config2(n_frames=args.frames)
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        frames = list(ex.map(w.frame, range(w.n_frames)))
    dev = torch.from_numpy(np.stack(frames)).cuda()
    F = dev.shape[0]
    P = w.params
    v = float(np.float32(P["voxel_size"]))
    gamma, d_max = v, 2.0
    m = vbx.Map(P["voxel_size"], P["trunc"], weighting=P["weighting"], merge=P["merge"], storage="f32",
                max_range=P["max_range"], block_capacity=16384, stream=stream)
    m.esdf_enable(gamma, d_max)
    batch = [(dev[k], w.poses[k], w.width) for k in range(F)]

    def batch_update():
        m.clear()
        m.integrate_frames(batch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = m.esdf_update()
        return (time.perf_counter() - t0) * 1e3, st

    for _ in range(max(args.warmup, 1)):
        batch_update()
    runs = [batch_update() for _ in range(args.steps)]
    batch_ms = float(np.median([r[0] for r in runs]))
    bst = runs[-1][1]
    first = m.esdf_export()
    # per-frame: integrate one frame, then update the ESDF from the blocks it changed
    m.clear()
    torch.cuda.synchronize()
    inc_ms, dirty = [], []
    for k in range(F):
        m.integrate_frames([batch[k]])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = m.esdf_update()
        inc_ms.append((time.perf_counter() - t0) * 1e3)
        dirty.append(st["dirty_blocks"])
    inc = m.esdf_export()
    same = (np.array_equal(first[0], inc[0]) and np.array_equal(first[1], inc[1]) and
            np.array_equal(first[2], inc[2]))
    if m.sync() != 0:
        raise RuntimeError("device status after the ESDF updates")
    observed = int(((first[2] & 1) > 0).sum())
    voxels = int(bst["voxels"])
    # algorithmic bytes of a batch update: every voxel of the changed blocks reads its TSDF voxel
    # (8 B) and reads and writes its ESDF word (16 B)
    algo = 24.0 * voxels
    roof = {"bound": "hbm", "achieved": round(algo / (batch_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(algo / (batch_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel_stage": "esdf_update (whole call, host-timed)", "algorithmic_bytes_per_launch": algo}
    m.close()

    # ---------------------------------------------------------------- Sec. VI-B accuracy
    poses, frame_fn, dist_fn = synth.esdf_benchmark()
    sframes = [frame_fn(k) for k in range(len(poses))]
    sdev = [torch.from_numpy(f).cuda() for f in sframes]
    accuracy = {}
    for vs in (0.05, 0.10, 0.20):
        vv = float(np.float32(vs))
        trunc = 4.0 * vs
        def tsdf(dist):
            g = vbx.Map(vs, trunc, weighting="quad", merge="grouped", storage="f32", max_range=5.0,
                        block_capacity=65536, stream=stream, dist=dist)
            g.integrate_frames([(sdev[k], poses[k], 320) for k in range(len(poses))])
            if g.sync() != 0:
                raise RuntimeError("device status after the simulated sequence")
            out = g.export()
            g.close()
            return out
        c, dw = tsdf("eq1")
        # the same TSDF with the distance along the ray (the projective distance of Sec. I)
        c_ray, dw_ray = tsdf("ray")
        assert np.array_equal(c_ray, c)
        from_voxel = (16 * c[:, None, :] + np.stack([np.arange(4096) & 15, (np.arange(4096) >> 4) & 15,
                                                     np.arange(4096) >> 8], axis=1)[None]).reshape(-1, 3)
        gt = dist_fn((from_voxel + 0.5) * vv).reshape(c.shape[0], 4096)
        variants = {"band_1v": (dw, vv), "band_half_trunc": (dw, float(np.float32(trunc / 2.0))),
                    "band_1v_along_ray": (dw_ray, vv),
                    "band_half_trunc_along_ray": (dw_ray, float(np.float32(trunc / 2.0)))}
        occ = dw.copy()
        neg = occ[:, :, 0] < 0
        occ[:, :, 0] = np.where(neg, 0.0, np.maximum(occ[:, :, 0], np.float32(1e-3 * vv)))
        variants["occupancy"] = (occ, float(np.float32(1e-3 * vv)))
        res = {}
        for name, (tsdf, gam) in variants.items():
            e = vbx.Map(vs, trunc, weighting="quad", merge="grouped", storage="f32", max_range=5.0,
                        block_capacity=65536, stream=stream)
            e.write_blocks(c, tsdf)
            e.esdf_enable(gam, 2.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e.esdf_update()
            ms = (time.perf_counter() - t0) * 1e3
            ec, ed, ei = e.esdf_export()
            e.close()
            assert np.array_equal(ec, c)
            # free space that the field covers: observed, outside objects, below d_max
            sel = ((ei & 1) > 0) & (gt > 0) & (gt < 2.0) & (np.abs(ed) < 2.0)
            err = (ed.astype(np.float64) - gt)[sel]
            res[name] = {"voxels": int(sel.sum()), "mean_abs_m": round(float(np.mean(np.abs(err))), 5),
                         "rms_m": round(float(np.sqrt(np.mean(err ** 2))), 5),
                         "mean_signed_m": round(float(np.mean(err)), 5),
                         "p95_abs_m": round(float(np.percentile(np.abs(err), 95)), 5) if err.size else None,
                         "fixed": int(((ei & 2) > 0).sum()), "update_ms": round(ms, 3)}
        accuracy[f"v{vs:g}"] = res

    return {
        "metric": "points/s & voxel-updates/s TSDF integration; p50/p99 frame latency (served)",
        "value": round(voxels / (batch_ms / 1e3), 1),
        "unit": "ESDF voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(batch_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"esdf: ESDF (gamma = 1 voxel, d_max 2 m, 26-neighbour quasi-Euclidean) "
                               f"of the {F}-frame 640x480 furnished-room TSDF (voxel 0.05 m), built in one "
                               f"update and updated after every frame; plus the simulated ESDF benchmark "
                               f"(50 noiseless 320x240 views, voxel 0.05/0.10/0.20 m, truncation 4 voxels)",
                   "frames": F},
        "esdf_batch": {"ms": round(batch_ms, 3), "voxels": voxels, "observed": observed,
                       "raise_rounds": bst["raise_rounds"], "lower_rounds": bst["lower_rounds"]},
        "esdf_per_frame": {"mean_ms": round(float(np.mean(inc_ms)), 3),
                           "p50_ms": round(float(np.median(inc_ms)), 3),
                           "max_ms": round(float(np.max(inc_ms)), 3),
                           "mean_dirty_blocks": round(float(np.mean(dirty)), 1)},
        "incremental_equals_batch": bool(same),
        "simulated_benchmark": accuracy,
        "roofline": roof,
        "cpu_baseline": None,
        "kernel_source_sha": kernel_source_sha(),
    }


# ------------------------------------------------------------------------------------------
# rocprofv3 summaries (host only): the tables under profiles/ are written by this function
# ------------------------------------------------------------------------------------------
def _short_kernel(name: str) -> str:
    """A kernel's name without its argument list (template arguments kept)."""
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def summarize_profiles(args):
    """Writes a markdown summary of rocprofv3 output to args.summary_out:
    * the kernel-trace statistics of every `*_kernel_stats.csv` under args.summary_stats;
    * for every directory of args.summary_pmc, the per-dispatch counters of its
      `*_counter_collection.csv`, averaged per kernel; the dispatches of the plain copy kernel
      give the HBM scaling factors (copy bytes / FETCH_SIZE and / WRITE_SIZE), applied to every
      kernel's FETCH_SIZE and WRITE_SIZE.
    args.summary_cmd lists the commands that produced the files, quoted in the summary."""
    import csv
    import glob
    lines = [f"# {args.summary_title}", ""]
    lines += ["Commands (from the repository root on one MI355X, TMPDIR=/tmp):", ""]
    lines += [f"    {c}" for c in args.summary_cmd] + [""]
    lines += [f"Kernel sources: sha {kernel_source_sha()} (bench.py kernel_source_sha).", ""]
    for d in args.summary_stats or []:
        for f in sorted(glob.glob(os.path.join(d, "**", "*_kernel_stats.csv"), recursive=True)):
            rows = list(csv.DictReader(open(f)))
            lines += ["## Kernel durations (kernel trace)", "",
                      "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
            for r in rows:
                lines.append(f"| {_short_kernel(r['Name'])} | {r['Calls']} | "
                             f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.2f} | "
                             f"{float(r['Percentage']):.2f} |")
            lines.append("")
    per = {}        # kernel -> counter -> [values per dispatch]
    for d in args.summary_pmc or []:
        for f in sorted(glob.glob(os.path.join(d, "**", "*_counter_collection.csv"), recursive=True)):
            acc = {}
            for r in csv.DictReader(open(f)):
                key = (_short_kernel(r["Kernel_Name"]), r["Dispatch_Id"], r["Counter_Name"])
                acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])   # summed over the row's dimensions
            for (k, _, c), v in acc.items():
                per.setdefault(k, {}).setdefault(c, []).append(v)
    if per:
        counters = sorted({c for k in per.values() for c in k})
        copy = next((k for k in per if "copyBuffer" in k or "elementwise_kernel" in k), None)
        scale = {}
        if copy and args.summary_copy_bytes:
            for c in ("FETCH_SIZE", "WRITE_SIZE"):
                if c in per[copy]:
                    vals = sorted(per[copy][c])
                    scale[c] = args.summary_copy_bytes / (vals[-1] * 1024.0)   # the largest copy dispatch
        lines += ["## Counters per dispatch (averaged over the kernel's dispatches)", ""]
        if scale:
            lines += ["HBM scaling from the largest dispatch of the plain copy kernel "
                      f"(`{copy}`, {args.summary_copy_bytes / 2 ** 30:.0f} GiB read and written): "
                      + ", ".join(f"bytes = {c} KiB x 1024 x {v:.3f}" for c, v in scale.items()), ""]
        head = "| kernel | dispatches | " + " | ".join(counters) + (" | HBM MB (scaled) |" if scale else " |")
        lines += [head, "|---|---:|" + "---:|" * (len(counters) + (1 if scale else 0))]
        for k in sorted(per, key=lambda k: -max((sum(v) / len(v)) for v in per[k].values())):
            n = max(len(v) for v in per[k].values())
            avg = {c: (sum(per[k][c]) / len(per[k][c]) if c in per[k] else None) for c in counters}
            cells = [f"{avg[c]:.4g}" if avg[c] is not None else "" for c in counters]
            hbm = ""
            if scale:
                mb = sum(avg[c] * 1024.0 * scale[c] for c in scale if avg.get(c) is not None) / 1e6
                hbm = f" {mb:.2f} |"
            lines.append(f"| {k} | {n} | " + " | ".join(cells) + " |" + hbm)
        lines.append("")
        if "SQ_INSTS_VALU" in counters and "SQ_WAVES" in counters:
            lines += ["Derived: VALU instructions per wave, and the share of the wave cycles spent "
                      "issuing VALU instructions (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES; both count "
                      "per wave, in quad-cycles on this hardware):", "",
                      "| kernel | VALU / wave | LDS / wave | VALU-active / wave cycles | busy-wait / wave cycles |",
                      "|---|---:|---:|---:|---:|"]
            for k in per:
                a = {c: sum(per[k][c]) / len(per[k][c]) for c in per[k]}
                if not a.get("SQ_WAVES"):
                    continue
                r1 = a.get("SQ_INSTS_VALU", 0) / a["SQ_WAVES"]
                r2 = a.get("SQ_INSTS_LDS", 0) / a["SQ_WAVES"]
                wc = a.get("SQ_WAVE_CYCLES")
                r3 = f"{a['SQ_ACTIVE_INST_VALU'] / wc:.3f}" if wc and "SQ_ACTIVE_INST_VALU" in a else ""
                r4 = f"{a['SQ_WAIT_INST_ANY'] / wc:.3f}" if wc and "SQ_WAIT_INST_ANY" in a else ""
                lines.append(f"| {k} | {r1:.1f} | {r2:.1f} | {r3} | {r4} |")
            lines.append("")
    # HBM bytes of a whole call: every kernel of the library that runs at least once per call,
    # its average bytes per dispatch times its dispatches, over the calls (the dispatches of the
    # kernel named by --summary-call-kernel, which runs once per call)
    call_bytes = None
    if args.summary_call_kernel and per and len(scale) == 2:
        ck = next((k for k in per if args.summary_call_kernel in k), None)
        if ck is None:
            raise SystemExit(f"no counters of a kernel matching {args.summary_call_kernel!r}")
        n_calls = len(per[ck]["FETCH_SIZE"])
        rows = []
        for k in per:
            if "vbx::" not in k or any(c not in per[k] for c in scale):
                continue
            n = len(per[k]["FETCH_SIZE"])
            if n < n_calls:
                continue   # set-up work outside the calls' common path
            tot = sum(sum(per[k][c]) * 1024.0 * scale[c] for c in scale)
            rows.append((k, n / n_calls, tot / n_calls))
        call_bytes = int(round(sum(r[2] for r in rows)))
        lines += [f"## HBM bytes per call ({n_calls} calls, kernels dispatched at least once per call)", "",
                  "| kernel | dispatches per call | HBM MB per call |", "|---|---:|---:|"]
        for k, dpc, b in sorted(rows, key=lambda r: -r[2]):
            lines.append(f"| {k} | {dpc:.0f} | {b / 1e6:.2f} |")
        lines += [f"| **whole call** | | **{call_bytes / 1e6:.2f}** |", ""]
    with open(args.summary_out, "w") as fh:
        fh.write("\n".join(lines))
    if call_bytes is not None:
        text = (f"# HBM bytes per call (every kernel of the call, summed) on {args.summary_workload},\n"
                f"# " + " + ".join(f"{c} x {scale[c]:.3f}" for c in scale) + " (KiB x 1024), from:\n"
                + "".join(f"#   {c}\n" for c in args.summary_cmd if "FETCH_SIZE" in c or "WRITE_SIZE" in c)
                + "# valid only for this workload, this update variant (split, threads, columns) and the\n"
                "# kernel sources with this sha (bench.py kernel_source_sha)\n"
                f"workload = {args.summary_workload}\nupdate_tuning = {args.summary_update_tuning}\n"
                f"source_sha = {kernel_source_sha()}\nhbm_bytes_per_launch = {call_bytes}\n")
        with open(os.path.join(args.summary_traffic_dir, "traffic_call.txt"), "w") as fh:
            fh.write(text)
    # per-stage HBM bytes that the benchmark reads back as roofline.traffic
    for spec in args.summary_traffic or []:
        stage, sub = spec.split(":", 1)
        k = next((k for k in per if sub in k), None)
        if k is None or len(scale) != 2:
            raise SystemExit(f"no counters of a kernel matching {sub!r}, or no copy calibration")
        avg = {c: sum(per[k][c]) / len(per[k][c]) for c in scale}
        hbm = int(round(sum(avg[c] * 1024.0 * scale[c] for c in scale)))
        tun = ""
        if stage == "update":
            tun = "update_tuning = " + args.summary_update_tuning + "\n"
        text = (f"# HBM bytes per launch of the {stage} stage kernel ({k}) on {args.summary_workload},\n"
                f"# " + " + ".join(f"{c} x {scale[c]:.3f}" for c in scale) + " (KiB x 1024), from:\n"
                + "".join(f"#   {c}\n" for c in args.summary_cmd if "FETCH_SIZE" in c or "WRITE_SIZE" in c)
                + "# valid only for this workload" + (", this update variant (split, threads, columns)"
                                                      if stage == "update" else "")
                + " and the kernel sources with this sha (bench.py kernel_source_sha)\n"
                f"workload = {args.summary_workload}\n{tun}source_sha = {kernel_source_sha()}\n"
                f"hbm_bytes_per_launch = {hbm}\n")
        with open(os.path.join(args.summary_traffic_dir, f"traffic_{stage}.txt"), "w") as fh:
            fh.write(text)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "accuracy", "esdf"])
    ap.add_argument("--no-forms", action="store_true",
                    help="c2: skip timing the plain per-frame f32 and batched f16 forms")
    ap.add_argument("--duration", type=float, default=10.0, help="c5: trace length in seconds")
    ap.add_argument("--load", type=float, default=1.0,
                    help="c5: multiplies every robot's request rate (1: the workload's 5-30 Hz)")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (c2, c3: 10; c4: 100 ticks)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=100, help="c2: frames of the sequence")
    ap.add_argument("--ticks", type=int, default=100, help="c4: distinct ticks generated")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "s16"], help="c2 storage")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="wall-clock budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch tuning instead of timing the candidates first")
    ap.add_argument("--voxel", type=float, default=None,
                    help="c3: voxel size (metres) instead of the workload's 0.20 m; truncation 3 voxels")
    ap.add_argument("--full-ray", action="store_true",
                    help="c3: walk every ray from the sensor (free space carved; the map grows far larger)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--summarize", action="store_true",
                    help="host only: write a markdown summary of rocprofv3 output (no GPU work)")
    ap.add_argument("--summary-title", default="Kernel statistics")
    ap.add_argument("--summary-stats", nargs="*", help="directories holding *_kernel_stats.csv")
    ap.add_argument("--summary-pmc", nargs="*", help="directories holding *_counter_collection.csv")
    ap.add_argument("--summary-cmd", action="append", default=[], help="a command that produced the files")
    ap.add_argument("--summary-copy-bytes", type=float, default=float(1 << 30),
                    help="bytes the calibration copy reads (and writes)")
    ap.add_argument("--summary-out", default="profile_summary.md")
    ap.add_argument("--summary-traffic", nargs="*",
                    help="stage:kernel-substring pairs whose HBM bytes go to profiles/traffic_<stage>.txt")
    ap.add_argument("--summary-traffic-dir", default=os.path.join(ROOT, "profiles"),
                    help="where the traffic_*.txt files go (the benchmark reads them from profiles/)")
    ap.add_argument("--summary-call-kernel", default=None,
                    help="a kernel that runs once per call: the whole call's HBM bytes go to "
                         "profiles/traffic_call.txt")
    ap.add_argument("--summary-workload", default="c2_room_640x480x100")
    ap.add_argument("--summary-update-tuning", default="1,1024,0")
    args = ap.parse_args()
    if args.summarize:
        summarize_profiles(args)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the integrator runs on a single MI355X "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 100 if args.workload == "c4" else 10

    import numpy as np
    import torch

    import synth
    import paper_1611_03631_amd as vbx

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    vbx.lib()   # raises if the HIP library is missing: no fallback

    if args.workload == "c2":
        out = bench_c2(args, np, torch, vbx, synth)
    elif args.workload == "c3":
        out = bench_c3(args, np, torch, vbx, synth)
    elif args.workload == "c4":
        out = bench_c4(args, np, torch, vbx, synth)
    elif args.workload == "accuracy":
        out = bench_accuracy(args, np, torch, vbx, synth)
    elif args.workload == "esdf":
        out = bench_esdf(args, np, torch, vbx, synth)
    else:
        out = bench_c5(args, np, torch, vbx, synth)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
