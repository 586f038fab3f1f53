"""The block sequence of a traversal from its block-changing steps alone (vbx_walk.h, used by
the crossing kernel) against the distinct blocks of the voxel walk, on the host: 3.6 million
random, dyadic (exact ties at block faces, edges and corners), axis-aligned and zero-length
segments, band-length to 700 voxels long."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1611_03631_amd", "csrc")


def test_block_walk_matches_voxel_walk(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "walk_check")
    # binary32 arithmetic in program order, as on the device (no contraction into fused
    # multiply-adds, no reassociation)
    subprocess.run([gxx, "-std=c++17", "-O2", "-ffp-contract=off", "-Wall", "-Werror",
                    "-Wno-unknown-pragmas", "-I", CSRC, os.path.join(HERE, "walk_check.cpp"), "-o", exe],
                   check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ALL OK" in res.stdout
