"""How long FP32 SGP stays within the parity bar of the FP64 oracle: the
iteration at which the relative KL gap |J_gpu / J_oracle - 1| first exceeds
1e-6, on the GPU and in the CPU model of FP32 rounding
(tests/fp32_emulation.py, which rounds fields, transforms and pointwise terms
to float32 and keeps sums and scalar rules in float64).  Both come from the
same inputs and the same iteration; the emulation is not bit-identical to
the kernels (its transforms round in another order), so the two crossings are
compared within a margin.  The fixed-count parity windows of the other GPU
tests lie before the GPU's crossing."""
import numpy as np
import pytest

import fp32_emulation as E
from oracle import sgp as O
from synth import workloads as W

pytestmark = pytest.mark.gpu

BAR = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_2258_amd as m
    m.load()
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _gpu_history(torch, w, n):
    """J(f^(1..n)) of a GPU run, from its per-iteration trace."""
    import paper_1210_2258_amd as m
    if w.domain is not None:
        _, rep = m.sgp_boundary_deconv(_dev(torch, w.g), _dev(torch, w.psf), w.b, w.domain, max_iter=n, trace=True)
    elif w.p > 1:
        _, rep = m.sgp_multi_deconv(_dev(torch, w.g), _dev(torch, w.psf), w.b, max_iter=n, trace=True)
    else:
        _, rep = m.sgp_deconv(_dev(torch, w.g[0]), _dev(torch, w.psf[0]), float(w.b[0]), max_iter=n, trace=True)
    assert rep["iters"] == n
    return np.asarray(rep["trace"]["J"][:n], np.float64)


CASES = {
    # name: (workload, iterations run, parity window of the fixed-count tests)
    "single_64x80": (lambda: W.small_single(64, 80), 40, 8),
    "multi_3x64": (lambda: W.small_multi(64, 64, p=3), 40, 4),
    "boundary_64x48_in_80x64": (lambda: W.small_boundary(80, 64, 64, 48, 8, 8), 40, 4),
    "single_c0_256": (W.config0, 60, 12),
}


@pytest.mark.parametrize("case", list(CASES))
def test_kl_gap_crossing_gpu_vs_fp32_model(torch_dev, case):
    make, n, window = CASES[case]
    w = make()
    print(f"drift {case}", flush=True)
    P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
    _, io = P.sgp(P.start("flat"), O.Params(max_iter=n))
    Jo = np.asarray(io["history"], np.float64)           # J^(0..n)
    _, Je, _ = E.sgp_fp32(P, n)
    Jg = _gpu_history(torch_dev, w, n)                   # J^(1..n)
    gap_g = np.abs(Jg / Jo[1:n + 1] - 1.0)
    gap_e = np.abs(Je[1:n + 1] / Jo[1:n + 1] - 1.0)
    kg = int(np.argmax(gap_g > BAR)) + 1 if (gap_g > BAR).any() else None
    ke = int(np.argmax(gap_e > BAR)) + 1 if (gap_e > BAR).any() else None
    print(f"{case}: KL gap first above {BAR:g} at iteration GPU {kg}, FP32 model {ke}; "
          f"GPU gap at 5/10/20: {gap_g[4]:.1e} {gap_g[9]:.1e} {gap_g[min(19, n - 1)]:.1e}; "
          f"model {gap_e[4]:.1e} {gap_e[9]:.1e} {gap_e[min(19, n - 1)]:.1e}", flush=True)
    # the fixed-count window ends before the GPU's crossing, and the GPU
    # leaves the bar no earlier than FP32 arithmetic itself does (within two
    # iterations: the model's transforms round in another order)
    assert kg is None or kg > window, (kg, window)
    assert ke is not None and (kg is None or kg >= ke - 2), (kg, ke)
