#!/usr/bin/env python3
"""Throughput benchmark of TSDF integration on one MI355X.

Workload: the 100-frame 640x480 depth sequence of a 10x10x3 m furnished room (camera on a
1.5 m circle), voxel 0.05 m, truncation 0.15 m, 1/z^2 weighting with drop-off, grouped
raycasting, binary32 storage.  One step integrates the whole sequence (one
vbx_integrate_frames call over the 100 frames, organised 640-wide) into an emptied map; the
frames are resident in HBM before timing starts.

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


def read_traffic(stage: str, sha: str):
    """HBM bytes per launch of `stage` from committed rocprofv3 counter runs, if they were taken
    on the current kernel sources (otherwise None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != sha:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="wall-clock budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch tuning instead of timing the candidates first")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the integrator runs on a single MI355X "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1611_03631_amd as vbx

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    vbx.lib()   # raises if the HIP library is missing: no fallback

    # ---------------------------------------------------------------- inputs
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
    m.profile(True)
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
    prof = m.profile_read(reset=True)
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
    dom = max(prof, key=lambda k: prof[k][0])
    ms_dom, launches = prof[dom]
    if dom not in algo:
        dom_for_roofline = max(algo, key=lambda k: prof[k][0])
    else:
        dom_for_roofline = dom
    ms_r, launches_r = prof[dom_for_roofline]
    per_launch_bytes = algo[dom_for_roofline] * args.steps / max(launches_r, 1)
    avg_launch_s = ms_r / max(launches_r, 1) / 1e3
    achieved = per_launch_bytes / avg_launch_s / 1e9
    sha = kernel_source_sha()
    traffic = read_traffic(dom_for_roofline, sha)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel_stage": dom_for_roofline, "launches_per_step": launches_r / args.steps,
                "avg_launch_ms": round(ms_r / max(launches_r, 1), 4),
                "algorithmic_bytes_per_launch": per_launch_bytes}
    whole = (algo["points"] + algo["update"]) / (ms_per_step / 1e3) / 1e9
    stages = {k: round(v[0] / args.steps, 4) for k, v in prof.items()}

    # ---------------------------------------------------------------- CPU oracle sample
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        om = oracle.OracleMap(P["voxel_size"], P["trunc"], weighting=P["weighting"],
                              merge=P["merge"], max_range=P["max_range"], storage=args.storage)
        done, pts = 0, 0
        t0 = time.perf_counter()
        while done < F and time.perf_counter() - t0 < args.cpu_seconds:
            om.integrate(frames[done], w.poses[done])
            pts += N
            done += 1
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(pts / cpu_s, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
               "sample": f"first {done} of {F} frames of the same sequence, integrated in order "
                         f"by the single-threaded C oracle ({cpu_s:.1f} s)"}
        om.close()

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    out = {
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
        "dtype": "f32" if args.storage == "f32" else "f16-storage/f32",
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
        "stage_ms_per_step": stages,
        "wall_s": round(wall_s, 3),
        "repeat_bit_identical": True,
        "tuning": m.tuning(),
        "autotune": tune,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "input_generation_s": round(gen_s, 1),
        "kernel_source_sha": sha,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
