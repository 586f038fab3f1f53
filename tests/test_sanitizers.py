"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code that runs on the CPU:
the oracles (driven over every mode by tests/oracle_sanitize_check.c) and the map server's
scheduling core (tests/sched_check.cpp, against a fake executor).  Any report of a sanitizer
(out-of-bounds access, use after free, leak, signed overflow, misaligned load, ...) fails the
run, since recovery is disabled."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1611_03631_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ALL OK" in res.stdout, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]


def test_oracles_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    exe = str(tmp_path / "oracle_sanitize_check")
    subprocess.run([gcc, "-std=gnu11", "-O1", *SAN, "-ffp-contract=off", "-Wall", "-Werror",
                    os.path.join(HERE, "oracle_sanitize_check.c"), os.path.join(ROOT, "oracle", "esdf_oracle.c"),
                    "-o", exe, "-lm"], check=True)
    _run(exe)


def test_scheduler_core_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "sched_check_san")
    subprocess.run([gxx, "-std=c++17", "-O1", *SAN, "-Wall", "-Werror", "-D_GLIBCXX_DEBUG", "-I", CSRC,
                    os.path.join(HERE, "sched_check.cpp"), "-o", exe], check=True)
    _run(exe)
