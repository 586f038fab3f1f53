"""Host-side contract of bench.py (no GPU needed): one GPU only, the workloads it accepts, and
measured traffic taken only from counter runs on the same sources, workload and variant."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused_with_a_message():
    for wl in ("c2", "accuracy"):
        r = run_bench("--gpus", "2", "--workload", wl)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout == ""


def test_unknown_workload_is_refused():
    r = run_bench("--workload", "nonesuch")
    assert r.returncode != 0 and "invalid choice" in r.stderr


def _traffic_file(stage):
    kv = {}
    for line in open(os.path.join(ROOT, "profiles", f"traffic_{stage}.txt")):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_traffic_is_read_only_for_matching_sources_workload_and_variant():
    sys.path.insert(0, ROOT)
    import bench
    pts = _traffic_file("points")
    got = bench.read_traffic("points", pts["source_sha"], pts["workload"])
    assert got == float(pts["hbm_bytes_per_launch"])
    assert bench.read_traffic("points", "0" * 16, pts["workload"]) is None
    assert bench.read_traffic("points", pts["source_sha"], "another_workload") is None
    upd = _traffic_file("update")
    split, threads, columns = (int(x) for x in upd["update_tuning"].split(","))
    tuning = {"update_split": split, "update_threads": threads, "update_columns": columns}
    assert bench.read_traffic("update", upd["source_sha"], upd["workload"], tuning) == \
        float(upd["hbm_bytes_per_launch"])
    assert bench.read_traffic("update", upd["source_sha"], upd["workload"], None) is None
    other = dict(tuning, update_threads=threads // 2)
    assert bench.read_traffic("update", upd["source_sha"], upd["workload"], other) is None
