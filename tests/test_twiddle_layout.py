"""The pass-ordered twiddle table (csrc/fft.hpp, tw_pass_index): entry
NS - r0 + (i - 1) NS + k of the pass with stride NS and radix R holds
W_L^m with m = i k L / (NS R), for every supported length and each of its
transform plans; the entries of all passes tile [0, L - r0) exactly once.  The index function is compiled
for the host from the library's header and compared with the layout
written out here from the radix plans (no GPU needed)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1210_2258_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SIZES = (16, 32, 64, 128, 256, 512, 1024, 2048, 80, 160, 320, 640, 1280)


def _plans():
    """{(L, A): radices} from the plan table of fft.hpp."""
    src = open(os.path.join(CSRC, "fft.hpp")).read()
    out = {}
    pat = r"SGP_FFT_PLAN\((\d+), (\d), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+)\)"
    for m in re.finditer(pat, src):
        L, A, NP = int(m.group(1)), int(m.group(2)), int(m.group(4))
        out[(L, A)] = [int(m.group(i)) for i in range(5, 10)][:NP]
    return out


def _expected(L, radices):
    r0 = radices[0]
    table = {}
    ns = r0
    for R in radices[1:]:
        for i in range(1, R):
            for k in range(ns):
                t = ns - r0 + (i - 1) * ns + k
                assert t not in table
                table[t] = i * k * (L // (ns * R))
        ns *= R
    assert ns == L
    return table


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_pass_ordered_twiddle_index(tmp_path):
    prog = tmp_path / "tw.cpp"
    plans = _plans()
    keys = sorted(k for k in plans if k[0] in SIZES)
    assert {L for L, _ in keys} == set(SIZES) and any(A == 1 for _, A in keys)
    body = "".join(f'  for (int t = 0; t < {L}; ++t) std::printf("{L} {A} %d %d\\n", t, '
                   f'sgp::tw_pass_index<sgp::FftPlan<{L}, {A}>>(t));\n' for L, A in keys)
    prog.write_text('#include <cstdio>\n#include "fft.hpp"\nint main() {\n' + body + "  return 0;\n}\n")
    exe = tmp_path / "tw"
    r = subprocess.run([HIPCC, "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I", CSRC, str(prog), "-o", str(exe)],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-3000:]
    got = {}
    for line in subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True, check=True).stdout.split("\n"):
        if line:
            L, A, t, m = map(int, line.split())
            got[(L, A, t)] = m
    for L, A in keys:
        exp = _expected(L, plans[(L, A)])
        r0 = plans[(L, A)][0]
        assert sorted(exp) == list(range(L - r0))
        for t in range(L):
            assert got[(L, A, t)] == exp.get(t, -1), (L, A, t, got[(L, A, t)], exp.get(t, -1))
