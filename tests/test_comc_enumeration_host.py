"""Host check of the colour-sampled colour-ordered enumeration (CPU only).

Builds tests/native/comc_enumeration_check.hip with hipcc (the device
functions of comc.hip are also host functions) and runs it on the CPU: the
closed-form counts of closing orderings (BEST theorem), the per-prefix
counts and the split enumeration order must equal a plain depth-first walk
with the delta-chain condition of eq. color_decomposition_colorflow.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "comc_enumeration_check.hip")


def test_enumeration_matches_plain_walk(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "comc_check")
    cmd = [hipcc, "-std=c++17", "-O0", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2106_06507_amd", "csrc"), SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
