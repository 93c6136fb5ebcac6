"""Pins of the linear relaxation of RL, Eq. (RL2), with the Armijo line
search along the RL direction (Sect. 1):

* with the largest step capped at 1 every iteration is the RL step, so the
  run equals rl() to 1e-13 (single, several images, boundary);
* each accepted step is at least 1, keeps f >= 0, satisfies the Armijo test
  on a KL evaluated independently (brute-force convolution and
  scipy.special's relative entropy), and the candidate before it (lam /
  theta, when one was tried) fails that test;
* the first step tried is the nonnegativity bound: a step 1% longer makes a
  pixel negative (unless the cap binds);
* the KL decreases monotonically and the discrepancy level is reached in
  fewer iterations than by RL (the gain the paper reports for this
  relaxation);
* planted mistakes (direction without the factor f, the Armijo test with
  the slope's sign flipped, no nonnegativity bound) fail these pins."""
import numpy as np
import pytest
from scipy import special

from oracle import sgp as O
from synth import workloads as W


def _kl_independent(P, f):
    tot = 0.0
    for j in range(P.p):
        y = P.A_direct(j, f) + P.b[j]
        tot += float(np.sum(special.rel_entr(P.g[j], y) + y - P.g[j]))
    return tot


def _tiny(p=1, domain=None, seed=7):
    rng = np.random.default_rng(seed)
    shape = (12, 10)
    NY, NX = shape if domain is None else domain[:2]
    psf = np.stack([W.gaussian_psf(NY, NX, 1.3 + 0.3 * j) for j in range(p)])
    obj = 30.0 * rng.random((NY, NX)) ** 4
    g = np.stack([rng.poisson(W.blur_periodic(obj, psf[j])[:shape[0], :shape[1]] + 2.0) for j in range(p)])
    return O.Problem(g.astype(float), psf, 2.0, domain=domain)


@pytest.mark.parametrize("case", ["single", "multi", "boundary"])
def test_rl_linear_with_unit_cap_is_rl(case):
    w = {"single": lambda: W.small_single(64, 80), "multi": W.small_multi,
         "boundary": W.small_boundary}[case]()
    P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
    n = 15
    f1, i1 = P.rl_linear(P.start("flat"), n, O.Params(max_iter=n, rl_lambda_cap=1.0))
    f2, i2 = P.rl(P.start("flat"), n)
    assert np.linalg.norm(f1 - f2) <= 1e-13 * np.linalg.norm(f2)
    assert all(l == 1.0 for l in i1["lam"])


def pin_steps(P, n=8):
    # a large beta makes the sufficient-decrease test bind on these steps
    prm = O.Params(max_iter=n, beta=0.3)
    f = P.start("flat")
    J = _kl_independent(P, f)
    for k in range(n):
        fk1, io = P.rl_linear(f, 1, prm)
        lam = io["lam"][0]
        G = P.grad(f)
        d = -P.invw * f * G
        gd = float(np.sum(G * d))
        assert lam >= 1.0
        assert fk1.min() >= 0.0
        np.testing.assert_allclose(fk1, np.maximum(0.0, f + lam * d), rtol=0, atol=1e-12 * f.max())
        # a step at the nonnegativity bound zeroes the pixel that bounds it
        ng = d < 0
        if ng.any() and lam == float(np.min(f[ng] / -d[ng])):
            i = np.argmin(np.where(ng, f / np.where(ng, -d, 1.0), np.inf))
            assert fk1.flat[i] == 0.0
        Jn = _kl_independent(P, fk1)
        assert Jn <= J + prm.beta * lam * gd + 1e-9 * J, (k, lam)
        neg = d < 0
        lam_max = min(prm.rl_lambda_cap, float(np.min(f[neg] / -d[neg]))) if neg.any() else prm.rl_lambda_cap
        assert lam <= lam_max * (1 + 1e-12), (k, lam, lam_max)
        if lam < lam_max * (1 - 1e-12) and lam > 1.0:
            prev = lam / prm.theta
            Jp = _kl_independent(P, np.maximum(0.0, f + prev * d))
            assert Jp > J + prm.beta * prev * gd, (k, lam, prev)
        if lam_max < prm.rl_lambda_cap:
            assert (f + 1.01 * lam_max * d).min() < 0.0
        assert Jn <= J
        f, J = fk1, Jn
    return f


@pytest.mark.parametrize("p,domain", [(1, None), (2, None), (1, (16, 14, 2, 2))])
def test_rl_linear_steps(p, domain):
    pin_steps(_tiny(p, domain))


def test_rl_linear_is_faster_than_rl_to_the_discrepancy_level():
    w = W.small_single(64, 80)
    P = O.Problem(w.g, w.psf, w.b)
    prm = O.Params(max_iter=3000, stop=O.STOP_DISCREPANCY)
    _, i1 = P.rl_linear(P.start("flat"), 3000, prm)
    _, i2 = P.rl(P.start("flat"), 3000, prm)
    assert i1["reason"] == i2["reason"] == O.REASON_DISCREPANCY
    assert i1["iters"] < 0.75 * i2["iters"], (i1["iters"], i2["iters"])
    h = np.asarray(i1["history"])
    assert np.all(np.diff(h) <= 0)


def _patched_rl_linear(mutation):
    """A copy of the line search with one plausible mistake."""
    def run(self, f0, n_iter, params=None):
        prm = params or O.Params(max_iter=n_iter)
        f = f0.copy()
        J = self.kl(f)
        lams = []
        for _ in range(n_iter):
            G = self.grad(f)
            d = -self.invw * G if mutation == "no_f" else -self.invw * f * G
            gd = float(np.sum(G * d))
            neg = d < 0
            lam_max = prm.rl_lambda_cap
            if neg.any() and mutation != "no_bound":
                lam_max = min(lam_max, float(np.min(f[neg] / -d[neg])))
            lam = lam_max
            slope = -gd if mutation == "sign" else gd
            while lam > 1.0:
                f_new = np.maximum(0.0, f + lam * d)
                J_new = self.kl(f_new)
                if J_new <= J + prm.beta * lam * slope:
                    break
                lam *= prm.theta
            if lam <= 1.0:
                lam, f_new = 1.0, np.maximum(0.0, f + d)
                J_new = self.kl(f_new)
            f, J = f_new, J_new
            lams.append(lam)
        return f, dict(iters=n_iter, kl=J, lam=lams)
    return run


@pytest.mark.parametrize("mutation", ["no_f", "sign", "no_bound"])
def test_pins_catch_planted_mistakes(monkeypatch, mutation):
    monkeypatch.setattr(O.Problem, "rl_linear", _patched_rl_linear(mutation))
    P = _tiny()
    with pytest.raises(AssertionError):
        pin_steps(P)
