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


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w") as fh:
        fh.write('"Kernel_Name","Dispatch_Id","Counter_Name","Counter_Value"\n')
        for name, disp, counter, value in rows:
            fh.write(f'"{name}",{disp},"{counter}",{value}\n')


def test_whole_call_traffic_sums_every_per_call_kernel(tmp_path):
    """The per-call HBM figure: the copy kernel's largest dispatch sets the scales (a 1 GiB copy
    reading 2^19 KiB of FETCH_SIZE and 2^20 KiB of WRITE_SIZE gives 2 and 1), every library
    kernel dispatched at least once per call counts with all its dispatches, set-up kernels
    dispatched fewer times do not, and other programs' kernels never do."""
    copy = "__amd_rocclr_copyBuffer"
    fetch, write = [], []
    d = 0
    for f, w in ((2 ** 19, 2 ** 20), (8, 8)):          # the calibration copy and a small copy
        d += 1
        fetch.append((copy, d, "FETCH_SIZE", f))
        write.append((copy, d, "WRITE_SIZE", w))
    for _ in range(3):                                  # three calls
        d += 1
        fetch.append(("vbx::k_a(int)", d, "FETCH_SIZE", 100))
        write.append(("vbx::k_a(int)", d, "WRITE_SIZE", 50))
        for _ in range(2):                              # a kernel launched twice per call
            d += 1
            fetch.append(("vbx::k_b(int)", d, "FETCH_SIZE", 10))
            write.append(("vbx::k_b(int)", d, "WRITE_SIZE", 10))
        d += 1
        fetch.append(("at::native::other(int)", d, "FETCH_SIZE", 10 ** 6))
        write.append(("at::native::other(int)", d, "WRITE_SIZE", 10 ** 6))
    d += 1                                              # set-up work outside the calls
    fetch.append(("vbx::k_setup(int)", d, "FETCH_SIZE", 10 ** 5))
    write.append(("vbx::k_setup(int)", d, "WRITE_SIZE", 10 ** 5))
    _counter_csv(str(tmp_path / "pmcF"), fetch)
    _counter_csv(str(tmp_path / "pmcW"), write)
    out = tmp_path / "summary.md"
    r = run_bench("--summarize", "--summary-pmc", str(tmp_path / "pmcF"), str(tmp_path / "pmcW"),
                  "--summary-out", str(out), "--summary-call-kernel", "k_a",
                  "--summary-traffic-dir", str(tmp_path), "--summary-workload", "wl",
                  "--summary-cmd", "rocprofv3 --pmc FETCH_SIZE run", "--summary-cmd",
                  "rocprofv3 --pmc WRITE_SIZE run")
    assert r.returncode == 0, r.stderr
    kv = {}
    for line in open(tmp_path / "traffic_call.txt"):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    per_a = (100 * 2 + 50 * 1) * 1024            # bytes per dispatch of k_a
    per_b = (10 * 2 + 10 * 1) * 1024
    assert int(kv["hbm_bytes_per_launch"]) == per_a + 2 * per_b
    assert kv["workload"] == "wl"
    text = out.read_text()
    assert "k_setup" not in text.split("## HBM bytes per call")[1]
    assert "other" not in text.split("## HBM bytes per call")[1]
