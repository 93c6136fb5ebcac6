"""The Armijo decision of the solver (csrc/finalize.hpp, fin_armijo and
armijo_needs_more, compiled for the host): a candidate whose sum is
+infinity (its model value left the domain of J in FP32) fails the test and
the search goes on; a NaN sum stops the run as a numerical failure; the first
candidate that satisfies J(f + lam d) <= J(f) + beta lam grad^T d is taken
(Algorithm 1, step 5).  No GPU needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1210_2258_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

PROG = r'''
#include <cmath>
#include <cstdio>
#include "finalize.hpp"
using namespace sgp;
static void init(DevState& st) {
  st = DevState{};
  st.max_backtracks = 40;
  st.beta = 1e-4;
  st.theta = 0.4;
  st.gd = -1.0;
  double lam = 1.0;
  for (int m = 0; m < kMaxCand; ++m) { st.lam_tab[m] = lam; lam *= st.theta; }
}
int main() {
  DevState st;
  const double inf = INFINITY, nan = NAN;
  // +inf for lambda = 1, a decrease for theta: theta is taken
  init(st);
  double a[2] = {inf, -1e-3};
  int needs = armijo_needs_more(&st, a, 0, 2);
  fin_armijo(&st, a, 0, 2);
  std::printf("%d %d %d %d %.17g\n", needs, st.done, st.reason, st.nback, st.lam);
  // both +inf: further candidates are needed, nothing committed
  init(st);
  double b[2] = {inf, inf};
  needs = armijo_needs_more(&st, b, 0, 2);
  fin_armijo(&st, b, 0, 2);
  std::printf("%d %d %d %d\n", needs, st.done, st.need_more, st.f_pending);
  // NaN: a numerical failure
  init(st);
  double c[2] = {nan, -1e-3};
  needs = armijo_needs_more(&st, c, 0, 2);
  fin_armijo(&st, c, 0, 2);
  std::printf("%d %d %d\n", needs, st.done, st.reason);
  // too small a decrease for lambda = 1 (above beta lam gd), enough for theta
  init(st);
  double d[2] = {-0.5e-4, -0.5e-4};
  fin_armijo(&st, d, 0, 2);
  std::printf("%d %d %.17g\n", st.done, st.nback, st.lam);
  return 0;
}
'''


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_out_of_domain_candidate_is_rejected(tmp_path):
    src = tmp_path / "armijo.cpp"
    src.write_text(PROG)
    exe = tmp_path / "armijo"
    r = subprocess.run([HIPCC, "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I", CSRC, str(src), "-o", str(exe)],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-3000:]
    out = subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True, check=True).stdout.split("\n")
    # theta accepted after an out-of-domain lambda = 1: not done, one reduction, lam = 0.4
    needs, done, reason, nback, lam = out[0].split()
    assert (needs, done, nback) == ("0", "0", "1") and float(lam) == 0.4
    # both out of the domain: the search continues past them
    assert out[1].split() == ["1", "0", "1", "0"]
    # NaN: stop, reason 6 (numerical failure)
    assert out[2].split() == ["0", "1", "6"]
    # the sufficient-decrease bar: -0.5e-4 > beta * 1 * gd = -1e-4 fails for lambda = 1,
    # and <= beta * 0.4 * gd = -0.4e-4 passes for theta
    done, nback, lam = out[3].split()
    assert (done, nback) == ("0", "1") and float(lam) == 0.4
