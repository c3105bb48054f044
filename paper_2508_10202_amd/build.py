"""Compile the HIP library ``libftm.so`` in-tree for gfx950 with hipcc.

Every call recompiles (the translation units in parallel) and then
atomically replaces ``paper_2508_10202_amd/libftm.so``.  Objects go to
``_build/`` at the repository root.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libftm.so")
SOURCES = ("ftm_api.hip", "ftm_fft.hip", "ftm_gemv.hip", "ftm_gemm.hip", "ftm_server.hip", "ftm_sbgemv.hip")
# ftm_fft_fixed.hip is compiled once per transform length with a fixed plan;
# the list matches FTM_FIXED_LENGTHS in ftm_fft.hip.
FIXED_SRC = "ftm_fft_fixed.hip"
FIXED_LENGTHS = (128, 256, 400, 512, 1024, 2000)
ARCH = "gfx950"

# Packed-FP32 instructions are switched off for every device compile; hipcc's
# host pass warns that it does not know the feature, which is harmless.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
                "-Wno-unused-function", "-Wno-unused-command-line-argument",
                "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc() -> str:
    cand = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cand):
        raise RuntimeError(f"hipcc not found (looked for {cand})")
    return cand


def _run(cmd: list[str]) -> None:
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"command failed ({res.returncode}): {' '.join(cmd)}\n{res.stdout}")


def build(verbose: bool = False) -> str:
    """Compile and link; returns the path of the library."""
    cc = hipcc()
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        jobs.append((obj, [cc, *COMMON_FLAGS, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]))
    for n in FIXED_LENGTHS:
        obj = os.path.join(bdir, f"ftm_fft_fixed_{n}.o")
        jobs.append((obj, [cc, *COMMON_FLAGS, *DEVICE_FLAGS, f"-DFTM_FIXED_N={n}", "-c",
                           os.path.join(CSRC, FIXED_SRC), "-o", obj]))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        for fut in [ex.submit(_run, cmd) for _, cmd in jobs]:
            fut.result()
    tmp = LIB_PATH + ".tmp"
    _run([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *[o for o, _ in jobs]])
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
