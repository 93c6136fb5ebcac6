"""Builds libsgpdeconv.so in-tree for gfx950 with hipcc.

Every FFT length gets its own object (csrc/inst.hip compiled with -DSGP_L=L);
objects compile in parallel.  ``python -m paper_1210_2258_amd.build`` or
``build()`` rebuilds everything.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsgpdeconv.so")
SIZES = (16, 32, 64, 128, 256, 512, 1024, 2048, 80, 160, 320, 640, 1280)
ARCH = os.environ.get("SGP_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def _jobs():
    jobs = []
    for L in SIZES:
        jobs.append(([HIPCC] + CFLAGS + [f"-DSGP_L={L}", "-c", os.path.join(CSRC, "inst.hip"),
                                           "-o", os.path.join(BUILD, f"inst_{L}.o")],
                     os.path.join(BUILD, f"inst_{L}.o")))
    jobs.append(([HIPCC] + CFLAGS + ["-c", os.path.join(CSRC, "dispatch.hip"),
                                     "-o", os.path.join(BUILD, "dispatch.o")],
                 os.path.join(BUILD, "dispatch.o")))
    jobs.append(([HIPCC] + CFLAGS + ["-c", os.path.join(CSRC, "cnn.hip"),
                                     "-o", os.path.join(BUILD, "cnn.o")],
                 os.path.join(BUILD, "cnn.o")))
    jobs.append(([HIPCC] + CFLAGS + ["-x", "hip", "-c", os.path.join(CSRC, "solver.cpp"),
                                     "-o", os.path.join(BUILD, "solver.o")],
                 os.path.join(BUILD, "solver.o")))
    return jobs


def build(verbose: bool = False, workers: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = _jobs()
    workers = workers or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        futs = [ex.submit(_run, cmd) for cmd, _ in jobs]
        for fut in futs:
            out = fut.result()
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + [o for _, o in jobs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
