"""Pins of the reconstruction-error stop of Sect. 3.3 (a simulation study
knows the true object f~; the run stops when rho^(k) = ||f^(k) - f~|| / ||f~||
reaches its minimum and returns that iterate).

Each stopped run of RL, OSEM and SGP is checked against the iterates of an
independent fixed-count trajectory, with rho evaluated here from its
definition: rho is non-increasing up to the returned index k, grows at
k + 1, and the returned f, KL and iteration count are those of f^(k).  Two
plausible mistakes are planted in the oracle (on the CPU) and must fail the
pin: returning the iterate after the minimum, and stopping on a comparison
with the starting error only."""
import numpy as np
import pytest

from oracle import sgp as O
from synth import workloads as W


def _rho(f, ft):
    return np.sqrt(np.sum((f - ft) ** 2) / np.sum(ft ** 2))


def _trajectory(P, method, n):
    """f^(0..n) of a fixed-count run (no stop rule), one call per length for
    SGP (its state is not resumable), one step at a time for RL / OSEM."""
    f0 = P.start("flat")
    if method == "sgp":
        return [P.sgp(f0, O.Params(max_iter=m))[0] for m in range(n + 1)]
    step = P.rl_step if method == "rl" else P.osem_cycle
    out = [f0]
    for _ in range(n):
        out.append(step(out[-1]))
    return out


def _stopped(P, method, ft):
    prm = O.Params(max_iter=300, stop=O.STOP_RMSE, f_true=ft)
    f0 = P.start("flat")
    if method == "sgp":
        return P.sgp(f0, prm)
    return getattr(P, method)(f0, 300, prm)


def pin_rmse_stop(method, p):
    w = W.small_galaxy(p=p)
    P = O.Problem(w.g, w.psf, w.b)
    f, io = _stopped(P, method, w.f_true)
    k = io["iters"]
    assert io["reason"] == O.REASON_RMSE
    traj = _trajectory(P, method, k + 1)
    r = [_rho(x, w.f_true) for x in traj]
    assert all(r[m + 1] <= r[m] for m in range(k)), (method, p, k, r)
    assert r[k + 1] > r[k], (method, p, k, r[k], r[k + 1])
    np.testing.assert_allclose(f, traj[k], rtol=0, atol=1e-12 * np.abs(traj[k]).max())
    assert io["kl"] == pytest.approx(P.kl(traj[k]), rel=1e-12)
    return k


CASES = [("rl", 1), ("osem", 3), ("sgp", 1), ("sgp", 3), ("rl", 3)]


@pytest.mark.parametrize("method,p", CASES)
def test_rmse_stop_returns_the_minimum(method, p):
    k = pin_rmse_stop(method, p)
    assert k >= 2    # a real minimum inside the run, not the start


def _after_minimum(orig):
    """Planted mistake: the iterate after the minimum is returned."""
    def run(self, f0, n_iter, params=None):
        f, io = orig(self, f0, n_iter, params)
        if io["reason"] == O.REASON_RMSE:
            f = self.rl_step(f)
        return f, io
    return run


def test_pin_catches_the_iterate_after_the_minimum(monkeypatch):
    monkeypatch.setattr(O.Problem, "rl", _after_minimum(O.Problem.rl))
    with pytest.raises(AssertionError):
        pin_rmse_stop("rl", 1)


def test_pin_catches_a_comparison_with_the_start(monkeypatch):
    """Planted mistake: each iterate's error compared with rho^(0) instead
    of the previous iterate's (the run goes on far past the minimum)."""

    def rl(self, f0, n_iter, params=None):
        f = f0.copy()
        rho0 = O.rel_error(f, params.f_true)
        k = 0
        while k < n_iter:
            f_new = self.rl_step(f)
            if O.rel_error(f_new, params.f_true) > rho0:
                break
            f, k = f_new, k + 1
        return f, dict(iters=k, kl=self.kl(f), history=[], reason=O.REASON_RMSE)

    monkeypatch.setattr(O.Problem, "rl", rl)
    with pytest.raises(AssertionError):
        pin_rmse_stop("rl", 1)
