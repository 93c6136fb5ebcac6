"""Linear relaxation of RL (Sect. 1, Eq. (RL2), Armijo line search along the
RL direction) on the GPU against the FP64 oracle: fixed iteration counts on
the single, three-image and boundary cases and the 256x256 star field, the
discrepancy stop at the oracle's iteration, and the argument checks.

Tolerances.  The first step tried is the nonnegativity bound
1 / (1 - min q) over the support, q the RL factor, which FP32 transforms give
to ~1e-6; as the step grows (lam up to ~4 here) the bound's relative error
grows with it (d lam / lam = lam dq), so accepted steps agree to ~1e-5
(measured: at most 3e-5 over 40 iterations), and since J is still falling
steeply at a step cut short by the bound (an early step lowers J by tens of
percent) the KL gap follows at ~1e-5 (measured 1e-7..1e-5).  The bars are
therefore steps 1e-4, f 1e-4 and KL 3e-5 over 20 iterations.  On the
boundary problem the bounding pixels lie on the rim of R, where the weights
M_R / alpha reach 1 / sigma_R = 1e3 and q = 1 + w v carries the absolute
FP32 transform error of v (~1e-7 of its largest value) times w: ~1e-4 in q
there, so steps and KL agree to ~2e-4 from the first iteration (bars 1e-3
over 3 iterations)."""
import numpy as np
import pytest

from oracle import sgp as O
from synth import workloads as W

pytestmark = pytest.mark.gpu

F_TOL = 1e-4


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


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


CASES = {
    "single_64x80": lambda: W.small_single(64, 80),
    "single_c0_256": W.config0,
    "multi_3x64": lambda: W.small_multi(64, 64, p=3),
    "boundary_64x48_in_80x64": lambda: W.small_boundary(80, 64, 64, 48, 8, 8),
}


def _gpu(torch, w, **kw):
    import paper_1210_2258_amd as m
    kw = {"rl_line_search": 1, **kw}
    if w.domain is not None:
        return m.rl_boundary_deconv(_dev(torch, w.g), _dev(torch, w.psf), w.b, w.domain, **kw)
    if w.p > 1:
        return m.rl_multi_deconv(_dev(torch, w.g), _dev(torch, w.psf), w.b, **kw)
    return m.rl_deconv(_dev(torch, w.g[0]), _dev(torch, w.psf[0]), float(w.b[0]), **kw)


# case: (iterations, step tolerance, f tolerance, KL tolerance)
BARS = {
    "single_64x80": (20, 1e-4, 1e-4, 3e-5),
    "single_c0_256": (20, 1e-4, 1e-4, 3e-5),
    "multi_3x64": (20, 1e-4, 1e-4, 3e-5),
    "boundary_64x48_in_80x64": (3, 1e-3, 1e-3, 1e-3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_rl_linear_fixed_iterations(torch_dev, case):
    torch = torch_dev
    w = CASES[case]()
    n, lam_tol, f_tol, kl_tol = BARS[case]
    print(f"rl2 {case} n={n}", flush=True)
    f, rep = _gpu(torch, w, max_iter=n, trace=True)
    P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
    fo, io = P.rl_linear(P.start("flat"), n)
    assert rep["iters"] == io["iters"] == n
    lam_g = np.asarray(rep["trace"]["lam"][:n])
    err = _rel(f.cpu().numpy(), fo)
    print(f"rl2 {case}: steps max rel diff {np.max(np.abs(lam_g / io['lam'] - 1)):.1e}, f {err:.1e}, "
          f"KL {abs(rep['kl'] / io['kl'] - 1):.1e}", flush=True)
    np.testing.assert_allclose(lam_g, io["lam"], rtol=lam_tol)
    assert err <= f_tol, err
    assert abs(rep["kl"] - io["kl"]) <= kl_tol * io["kl"], (rep["kl"], io["kl"])


def test_rl_linear_discrepancy_stop(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    w = W.small_single(64, 80)
    f, rep = _gpu(torch, w, max_iter=3000, stop=m.STOP_DISCREPANCY)
    P = O.Problem(w.g, w.psf, w.b)
    fo, io = P.rl_linear(P.start("flat"), 3000, O.Params(max_iter=3000, stop=O.STOP_DISCREPANCY))
    _, rl = _gpu(torch, w, max_iter=3000, stop=m.STOP_DISCREPANCY, rl_line_search=0)
    print(f"rl2 to discrepancy: GPU {rep['iters']}, oracle {io['iters']}, RL {rl['iters']}", flush=True)
    assert rep["reason"] == "discrepancy"
    assert abs(rep["iters"] - io["iters"]) <= 1
    assert rep["iters"] < 0.75 * rl["iters"]


def test_rl_linear_argument_checks(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    w = W.small_single(64, 80)
    g, psf = _dev(torch, w.g[0]), _dev(torch, w.psf[0])
    with pytest.raises(m.SgpError):
        m.rl_deconv(g, psf, 10.0, max_iter=2, rl_line_search=1, rl_alpha=1.5)
    with pytest.raises(m.SgpError):
        m.rl_deconv(g, psf, 10.0, max_iter=2, rl_line_search=1, rl_lambda_cap=0.5)
    with pytest.raises(m.SgpError):
        m.sgp_deconv(g, psf, 10.0, max_iter=2, rl_line_search=1)
