"""The library's host code (argument checks, per-shape workspaces, the batch
driver with its per-item stops, compaction and graph re-capture) under
AddressSanitizer on the CPU: solver.cpp is compiled for the host only and
linked against a CPU stand-in for the HIP runtime whose graphs record and
replay the launches and whose iteration end stops each batched item at a
known count.  The harness checks every item's iteration count in its report,
for batches and for single problems through the stepping loop (graph replays
and the eager launches of the entry point that allocates nothing), and that
the run has no invalid memory access or bad free."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_asan")
CSRC = os.path.join(ROOT, "paper_1210_2258_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None, reason="needs hipcc and g++")
def test_batch_host_logic_under_asan(tmp_path):
    san = ["-g", "-O1", "-fno-omit-frame-pointer"]
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]

    def sh(cmd):
        r = subprocess.run(cmd, cwd=tmp_path, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:]
        return r

    host = [HIPCC, "-x", "hip", "--cuda-host-only", "-std=c++17", *san, "-Xarch_host", "-fsanitize=address", *inc]
    sh(host + ["-c", os.path.join(CSRC, "solver.cpp"), "-o", "solver.o"])
    sh(host + ["-c", os.path.join(HERE, "shim.cpp"), "-o", "shim.o"])
    # the host pass references the (absent) device-code blob by name
    nm = sh(["nm", "-u", "solver.o"]).stdout
    blobs = [ln.split()[-1] for ln in nm.splitlines() if "__hip_fatbin_" in ln]
    (tmp_path / "blob.cpp").write_text("".join(f'extern "C" {{ char {b}[16] = {{0}}; }}\n' for b in blobs))
    sh(["g++", "-std=c++17", *san, "-fsanitize=address", *inc, "-c", os.path.join(HERE, "harness.cpp"), "-o",
        "harness.o"])
    sh(["g++", "-c", "blob.cpp", "-o", "blob.o"])
    sh(["g++", "-no-pie", "-fsanitize=address", "-o", "harness", "harness.o", "solver.o", "shim.o", "blob.o"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([str(tmp_path / "harness")], cwd=tmp_path, capture_output=True, text=True, timeout=600,
                       env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ALL OK" in r.stdout and "AddressSanitizer" not in out, out[-4000:]
    assert r.stdout.count("single max_iter") == 3, r.stdout[-2000:]
