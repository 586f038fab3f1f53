"""The map server's scheduling core (admission under a budget, tick formation, per-map
order, replay of requests a full pool turned away) on the host, against a fake executor."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1611_03631_amd", "csrc")


def test_scheduler_core(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "sched_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-D_GLIBCXX_DEBUG", "-I", CSRC,
                    os.path.join(HERE, "sched_check.cpp"), "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ALL OK" in res.stdout
