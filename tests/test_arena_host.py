"""Host-only check of the serving scheduler's workspace arena: compiled with
the host C++ compiler (no GPU, no HIP) from the same header the library
uses."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_admission_and_random_traffic(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "arena_check")
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_2508_10202_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "arena_check.cpp"), "-o", exe], check=True)
    res = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=60)
    assert res.returncode == 0, res.stdout
    assert res.stdout.strip().startswith("OK")
