"""The kernels' lane layouts (the header the stencil and finalize kernels
include, compiled for the host): every layout covers its tile exactly once
-- a missing or doubled cell would be a lost update or a race -- and in FP32
each half-wave touches 32 distinct LDS banks; the pair staging of the LDS
tiles stages every cell and gives each exactly one owning thread."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_lane_layouts_cover_their_tiles_without_bank_conflicts(tmp_path):
    exe = tmp_path / "lane_layouts_check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                           "-I", os.path.join(ROOT, "paper_1909_04153_amd", "csrc"),
                           os.path.join(ROOT, "tests", "lane_layouts_check.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("staging checked") == 12, r.stdout
    assert r.stdout.count("checked") == 19, r.stdout
