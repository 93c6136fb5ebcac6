"""Reconstruction-error stop of Sect. 3.3 on the GPU against the FP64 oracle:
RL, OSEM and SGP on the small extended-object case (one image and three
fringe images), where the error reaches its minimum after some ten
iterations.  The run must stop at the oracle's index, return the iterate of
the minimum (f within 1e-4, KL within 1e-6 of the oracle's), and a stepping
solver advanced a few iterations at a time must end on the same iterate
bit for bit."""
import numpy as np
import pytest

from oracle import sgp as O
from synth import workloads as W

pytestmark = pytest.mark.gpu

F_TOL, KL_TOL = 1e-4, 1e-6


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


CASES = [("rl", 1), ("sgp", 1), ("osem", 3), ("sgp", 3), ("rl", 3)]


def _gpu(torch, method, w, **kw):
    import paper_1210_2258_amd as m
    g, psf, ft = _dev(torch, w.g), _dev(torch, w.psf), _dev(torch, w.f_true)
    kw = {"max_iter": 300, "stop": m.STOP_RMSE, "f_true": ft, **kw}
    if w.p == 1:
        fn = {"rl": m.rl_deconv, "sgp": m.sgp_deconv}[method]
        return fn(g[0], psf[0], float(w.b[0]), **kw)
    fn = {"rl": m.rl_multi_deconv, "sgp": m.sgp_multi_deconv, "osem": m.osem_deconv}[method]
    return fn(g, psf, w.b, **kw)


@pytest.mark.parametrize("method,p", CASES)
def test_rmse_stop_matches_oracle(torch_dev, method, p):
    torch = torch_dev
    w = W.small_galaxy(p=p)
    print(f"rmse stop {method} p={p}", flush=True)
    f, rep = _gpu(torch, method, w)
    P = O.Problem(w.g, w.psf, w.b)
    prm = O.Params(max_iter=300, stop=O.STOP_RMSE, f_true=w.f_true)
    fo, io = P.sgp(P.start("flat"), prm) if method == "sgp" else getattr(P, method)(P.start("flat"), 300, prm)
    assert rep["reason"] == "rmse" and io["reason"] == O.REASON_RMSE
    assert rep["iters"] == io["iters"], (rep["iters"], io["iters"])
    err = _rel(f.cpu().numpy(), fo)
    assert err <= F_TOL, err
    assert abs(rep["kl"] - io["kl"]) <= KL_TOL * io["kl"], (rep["kl"], io["kl"])


@pytest.mark.parametrize("method", ["rl", "sgp"])
def test_rmse_stop_stepping_equals_one_call(torch_dev, method):
    """A solver stepped 3 iterations at a time (pauses fall before, at and
    after the minimum) ends on the one-call result, bit for bit."""
    import paper_1210_2258_amd as m
    torch = torch_dev
    w = W.small_galaxy()
    f1, rep1 = _gpu(torch, method, w)
    kind = m.KIND_RL if method == "rl" else m.KIND_SGP
    S = m.Solver(kind, _dev(torch, w.g[0]), _dev(torch, w.psf[0]), float(w.b[0]), max_iter=300,
                 stop=m.STOP_RMSE, f_true=_dev(torch, w.f_true))
    for _ in range(200):
        if S.step(3):
            break
    rep = S.report()
    f2 = S.f.clone()
    S.close()
    assert rep["reason"] == "rmse" and rep["iters"] == rep1["iters"]
    assert torch.equal(f1, f2)
    assert rep["kl"] == rep1["kl"]


def test_rmse_stop_argument_checks(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    w = W.small_galaxy()
    g, psf = _dev(torch, w.g[0]), _dev(torch, w.psf[0])
    with pytest.raises(m.SgpError):
        m.sgp_deconv(g, psf, 10.0, max_iter=5, stop=m.STOP_RMSE)          # no true object
    with pytest.raises(ValueError):
        m.sgp_deconv(g, psf, 10.0, max_iter=5, stop=m.STOP_RMSE, f_true=g[:32])


@pytest.mark.parametrize("method", ["rl", "sgp"])
def test_rmse_stop_at_the_iteration_cap(torch_dev, method):
    """With max_iter one past the minimum the last iterate is still tested
    (stop by the error, the minimum returned); with max_iter at the minimum
    the cap ends the run there."""
    torch = torch_dev
    w = W.small_galaxy()
    _, rep = _gpu(torch, method, w)
    k = rep["iters"]
    f1, r1 = _gpu(torch, method, w, max_iter=k + 1)   # the keyword overrides max_iter=300
    assert r1["reason"] == "rmse" and r1["iters"] == k
    f2, r2 = _gpu(torch, method, w, max_iter=k)
    assert r2["reason"] == "maxiter" and r2["iters"] == k
    assert torch.equal(f1, f2)
