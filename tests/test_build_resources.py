"""The hot-path kernels must not touch scratch (private) memory: a copy of
the argument block that spills there costs every workgroup a round trip
through memory.  Compiles the 2048-point kernels and the per-pixel kernels
for gfx950 and reads the compiler's resource report (no GPU needed)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1210_2258_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _resources(src, defines, tmp_path):
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *defines, "-c",
           os.path.join(CSRC, src), "-o", str(tmp_path / "k.o"), "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert out.returncode == 0, out.stdout[-2000:]
    names = re.findall(r"Function Name: (\S+)", out.stdout)
    scratch = [int(v) for v in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out.stdout)]
    assert names and len(names) == len(scratch)
    return dict(zip(names, scratch))


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("src,defines", [("inst.hip", ["-DSGP_L=2048"]), ("dispatch.hip", [])])
def test_no_kernel_uses_scratch(src, defines, tmp_path):
    res = _resources(src, defines, tmp_path)
    assert any("row_kernel" in n or "pix_kernel" in n for n in res)
    bad = {n: v for n, v in res.items() if v}
    assert not bad, bad
