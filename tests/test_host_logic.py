"""Host-side logic of the library checked without a GPU: small C++ programs
built with hipcc against the library's own headers and run on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1801_04984_amd", "csrc")


def _run(src, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "check")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "host", src), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def test_xcd_tile_order_is_a_contiguous_permutation(tmp_path):
    _run("xcd_order_check.cpp", tmp_path)
