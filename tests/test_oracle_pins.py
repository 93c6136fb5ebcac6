"""Pins of the FP64 oracle against facts fixed outside it: brute-force
convolution, adjointness, finite differences, closed forms, library routines,
invariants the paper states (Sect. 1, 2, 3) and hand-computed steplength
tables.  CPU only."""
import os

import numpy as np
import pytest
from scipy import special, stats

from oracle import sgp as O
from synth import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_problem(rng, shape, p=1, domain=None, b=3.0, asym=True):
    NY, NX = shape if domain is None else domain[:2]
    ny, nx = shape
    psf = rng.random((p, NY, NX)) if asym else np.stack([W.gaussian_psf(NY, NX, 1.2)] * p)
    g = rng.poisson(20.0, (p, ny, nx)).astype(float)
    return O.Problem(g, psf, b, domain=domain)


# ----------------------------------------------------------------- O1 operators
@pytest.mark.parametrize("shape", [(5, 7), (8, 8), (16, 12), (10, 10)])
def test_fft_convolution_matches_direct(shape):
    rng = np.random.default_rng(1)
    P = _rand_problem(rng, shape)
    f = rng.random(shape)
    a = P.A(0, f)
    d = P.A_direct(0, f)
    assert np.linalg.norm(a - d) <= 1e-12 * np.linalg.norm(d)


def test_boundary_convolution_matches_direct():
    rng = np.random.default_rng(2)
    P = _rand_problem(rng, (6, 5), domain=(11, 9, 3, 2))
    f = rng.random((11, 9))
    a = P.A(0, f)
    d = P.A_direct(0, f)
    assert np.linalg.norm(a - d) <= 1e-12 * np.linalg.norm(d)


def test_psf_centre_convention():
    """A delta at n0 maps the PSF centre (ny//2, nx//2) onto n0."""
    rng = np.random.default_rng(3)
    ny, nx = 9, 12
    psf = rng.random((ny, nx))
    P = O.Problem(np.ones((ny, nx)), psf, 1.0)
    K = psf / psf.sum()
    n0 = (2, 7)
    f = np.zeros((ny, nx))
    f[n0] = 1.0
    Af = P.A(0, f)
    for dy in range(-4, 5):
        for dx in range(-6, 6):
            m = ((n0[0] + dy) % ny, (n0[1] + dx) % nx)
            assert abs(Af[m] - K[ny // 2 + dy, nx // 2 + dx]) < 1e-14


@pytest.mark.parametrize("kind", ["single", "multi", "boundary"])
def test_adjointness(kind):
    rng = np.random.default_rng(4)
    if kind == "single":
        P = _rand_problem(rng, (12, 10))
    elif kind == "multi":
        P = _rand_problem(rng, (12, 10), p=3)
    else:
        P = _rand_problem(rng, (8, 6), p=2, domain=(14, 12, 3, 4))
    f = rng.random((P.NY, P.NX))
    for j in range(P.p):
        y = rng.random((P.ny, P.nx))
        lhs = np.sum(P.A(j, f) * y)
        rhs = np.sum(f * P.AT(j, y))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_transpose_of_one_is_one_for_unit_psf():
    rng = np.random.default_rng(5)
    P = _rand_problem(rng, (10, 14), p=2)
    for j in range(2):
        assert np.max(np.abs(P.AT(j, np.ones((10, 14))) - 1.0)) < 1e-13


def test_boundary_weights():
    """alpha_j = K_j correlated with M_S: sums to |S|, is 1 deep inside S and
    ~0 far outside (Sect. 2.4 weights; reading: no g factor)."""
    NY, NX, ny, nx, oy, ox = 64, 64, 32, 32, 16, 16
    psf = W.gaussian_psf(NY, NX, 1.5)
    P = O.Problem(np.ones((ny, nx)), psf, 1.0, domain=(NY, NX, oy, ox))
    a = P.alpha_j[0]
    assert abs(a.sum() - ny * nx) < 1e-9
    assert abs(a[oy + 16, ox + 16] - 1.0) < 1e-12
    assert a[2, 2] < 1e-12
    R = P.MR > 0
    assert R[oy:oy + ny, ox:ox + nx].all()        # S inside R
    assert not R[0, 0]
    # A^T 1 = M_R o alpha_j
    assert np.allclose(P.AT(0, np.ones((ny, nx))), P.MR * a, atol=1e-13)


# ----------------------------------------------------------------- O2 KL
def test_kl_matches_library_and_gibbs():
    rng = np.random.default_rng(6)
    P = _rand_problem(rng, (12, 12), p=2, b=2.0)
    P.g[0, 0, 0] = 0.0
    f = rng.random((12, 12)) * 10
    J = P.kl(f)
    ref = sum(special.kl_div(P.g[j], P.A(j, f) + P.b[j]).sum() for j in range(2))
    assert abs(J - ref) <= 1e-12 * ref
    assert J > 0
    # equality case: noise-free data g = A f + b
    P2 = _rand_problem(rng, (12, 12), p=2, b=2.0)
    P2.g = np.stack([P2.A(j, f) + P2.b[j] for j in range(2)])
    assert abs(P2.kl(f)) < 1e-9


# ----------------------------------------------------------------- O3 gradient
@pytest.mark.parametrize("kind", ["single", "multi", "boundary"])
def test_gradient_finite_differences(kind):
    rng = np.random.default_rng(7)
    if kind == "single":
        P = _rand_problem(rng, (6, 6))
    elif kind == "multi":
        P = _rand_problem(rng, (6, 6), p=3)
    else:
        P = _rand_problem(rng, (4, 4), p=2, domain=(6, 6, 1, 1))
    f = (rng.random((P.NY, P.NX)) + 0.5) * 10 * P.MR
    G = P.grad(f)
    h = 1e-5
    for idx in np.ndindex(P.NY, P.NX):
        if P.MR[idx] == 0:
            continue
        e = np.zeros_like(f)
        e[idx] = h
        fd = (P.kl(f + e) - P.kl(f - e)) / (2 * h)
        assert abs(fd - G[idx]) <= 1e-6 * max(1.0, abs(G[idx]))


# ----------------------------------------------------------------- O4 RL
def test_rl_flux_conservation_and_positivity():
    rng = np.random.default_rng(8)
    P = _rand_problem(rng, (16, 12), b=0.0)
    f = P.start("flat")
    for _ in range(5):
        f = P.rl_step(f)
        assert f.min() >= 0
        assert abs(f.sum() - P.g.sum()) <= 1e-10 * P.g.sum()
    Pm = _rand_problem(rng, (16, 12), p=3, b=0.0)
    f = Pm.start("flat")
    for _ in range(3):
        f = Pm.rl_step(f)
        assert abs(f.sum() - Pm.g.sum() / 3) <= 1e-10 * Pm.g.sum()


@pytest.mark.parametrize("kind", ["single", "multi", "boundary"])
def test_rl_monotone_kl(kind):
    w = {"single": W.small_single(32, 24), "multi": W.small_multi(32, 32),
         "boundary": W.small_boundary(40, 32, 32, 24, 4, 4)}[kind]
    P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
    _, info = P.rl(P.start("flat"), 30)
    h = np.array(info["history"])
    assert np.all(np.diff(h) <= 1e-9 * h[:-1])


# ----------------------------------------------------------------- O6 bounds
def test_bounds_rule_delta_psf():
    """With a delta PSF, one RL step from flat c is c g / (c + b), so the
    Sect. 3.2 rule can be evaluated by hand."""
    ny, nx = 4, 4
    psf = np.zeros((ny, nx))
    psf[ny // 2, nx // 2] = 1.0
    b = 2.0
    g = np.full((ny, nx), 10.0)
    g[0, 0] = 30.0
    P = O.Problem(g, psf, b)
    c = (g - b).sum() / 16.0                       # flat start value
    L1, L2 = P.bounds(P.start("flat"))
    ymin, ymax = c * 10 / (c + b), c * 30 / (c + b)  # ratio 3 < 50
    assert np.isclose(L1, ymin / 10, rtol=1e-14) and np.isclose(L2, 10 * ymax, rtol=1e-14)
    g[1, 1] = 1.0
    g[2, 2] = 2000.0
    P = O.Problem(g, psf, b)
    c = (g - b).sum() / 16.0
    L1, L2 = P.bounds(P.start("flat"))
    assert np.isclose(L1, c * 1 / (c + b), rtol=1e-14) and np.isclose(L2, c * 2000 / (c + b), rtol=1e-14)


# ----------------------------------------------------------------- O7 SGP
def _golden_rules():
    rows = []
    with open(os.path.join(GOLDEN, "steplength_rules.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            rows.append(line.split("|"))
    return rows


def test_steplength_rules_hand_table():
    prm = O.Params()
    rows = _golden_rules()
    assert len(rows) >= 8
    for r in rows:
        k, alpha, tau = int(r[0]), float(r[1]), float(r[2])
        Q = [float(v) for v in r[3].split()] if r[3].strip() else []
        a, c1, c2, e = (float(v) for v in r[4].split())
        ea1, ea2, enext, etau, ealt = (float(v) for v in r[5].split())
        a1, a2, _, _, nxt, tau2, Q2, alt = O.steplength_update(alpha, tau, Q, k, a, c1, c2, e, prm)
        assert np.isclose(a1, ea1, rtol=1e-15), r
        assert np.isclose(a2, ea2, rtol=1e-15), r
        assert np.isclose(nxt, enext, rtol=1e-15), r
        assert np.isclose(tau2, etau, rtol=1e-15), r
        assert alt == int(ealt), r
        assert len(Q2) <= prm.m_alpha


@pytest.mark.parametrize("kind", ["single", "multi", "boundary"])
def test_sgp_reduces_to_rl(kind):
    """Eq. (RL2) with lambda = 1: alpha = 1, lambda = 1, no clipping makes an
    SGP step an RL step (also Eqs. multipleRL / boundaryRL with Dkbound)."""
    w = {"single": W.small_single(32, 24), "multi": W.small_multi(32, 32),
         "boundary": W.small_boundary(40, 32, 32, 24, 4, 4)}[kind]
    P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
    f0 = P.start("flat")
    f_rl = f0
    for _ in range(3):
        f_rl = P.rl_step(f_rl)
    f_sgp, _ = P.sgp(f0, O.Params(max_iter=3), force_alpha=1.0, force_lambda=1.0,
                     bounds=(0.0, np.inf))
    assert np.linalg.norm(f_sgp - f_rl) <= 1e-13 * np.linalg.norm(f_rl)


def test_sgp_delta_psf_reaches_closed_form():
    """K = delta makes J separable with minimiser max(0, g - b)."""
    rng = np.random.default_rng(9)
    ny, nx = 16, 16
    psf = np.zeros((ny, nx))
    psf[ny // 2, nx // 2] = 1.0
    b = 5.0
    g = rng.poisson(rng.uniform(0, 40, (ny, nx))).astype(float)
    P = O.Problem(g, psf, b)
    f, info = P.sgp(P.start("flat"), O.Params(max_iter=400))
    fstar = np.maximum(0.0, g - b)
    assert np.max(np.abs(f - fstar)) < 1e-3 * max(1.0, fstar.max())
    assert info["kl"] <= P.kl(fstar) + 1e-9 * P.kl(fstar)


def test_sgp_monotone_and_discrepancy_decreasing():
    w = W.small_single(64, 48)
    P = O.Problem(w.g, w.psf, w.b)
    f, info = P.sgp(P.start("flat"), O.Params(max_iter=60))
    h = np.array(info["history"])
    assert np.all(np.diff(h) <= 0)                 # Armijo monotone decrease
    Dk = 2 * h / P.nS
    assert Dk[0] > 1.0
    assert Dk[-1] < Dk[0]
    assert f.min() >= 0


def test_sgp_needs_fewer_iterations_than_rl():
    """Qualitative claim of the paper (Sect. 5): SGP reaches the data fit of
    RL in several times fewer iterations (here at least 2x, with the adaptive
    bounds of Sect. 3.2)."""
    w = W.small_single(64, 48)
    P = O.Problem(w.g, w.psf, w.b)
    f0 = P.start("flat")
    _, irl = P.rl(f0, 400)
    target = irl["history"][-1]
    _, isgp = P.sgp(f0, O.Params(max_iter=400))
    k = int(np.argmax(np.array(isgp["history"]) <= target))
    assert 0 < k < 400 / 2


def test_discrepancy_stop_first_hit():
    w = W.small_single(64, 48)
    P = O.Problem(w.g, w.psf, w.b)
    f, info = P.sgp(P.start("flat"), O.Params(max_iter=500, stop=O.STOP_DISCREPANCY))
    h = info["history"]
    assert info["reason"] == O.REASON_DISCREPANCY
    assert P.discrepancy(h[-1]) <= 1.0
    assert all(P.discrepancy(v) > 1.0 for v in h[:-1])


# ----------------------------------------------------------------- O8 flux
def test_flux_projection_kkt_and_library():
    from scipy.optimize import minimize
    rng = np.random.default_rng(10)
    for trial in range(5):
        n = 9
        z = rng.normal(0, 2, n)
        D = rng.uniform(0.2, 3.0, n)
        c = 4.0 + trial
        x = O.flux_projection(z, D, c)
        assert x.min() >= 0 and abs(x.sum() - c) < 1e-12 * c
        act = x > 0
        mus = (z[act] - x[act]) / D[act]
        assert np.ptp(mus) < 1e-12
        assert np.all(z[~act] - mus[0] * D[~act] <= 1e-12)
        res = minimize(lambda v: np.sum((v - z) ** 2 / D), np.full(n, c / n),
                       jac=lambda v: 2 * (v - z) / D, method="SLSQP",
                       bounds=[(0, None)] * n,
                       constraints=[{"type": "eq", "fun": lambda v: v.sum() - c}],
                       options=dict(ftol=1e-14, maxiter=500))
        assert np.max(np.abs(res.x - x)) < 1e-6


def test_flux_projection_bisection_agrees():
    rng = np.random.default_rng(11)
    z = rng.normal(1, 3, 500)
    D = rng.uniform(0.1, 2, 500)
    c = 300.0
    x = O.flux_projection(z, D, c)
    lo, hi = (z / D).min() - 1e3, (z / D).max() + 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.maximum(0, z - mid * D).sum() > c:
            lo = mid
        else:
            hi = mid
    xb = np.maximum(0, z - 0.5 * (lo + hi) * D)
    assert np.max(np.abs(xb - x)) < 1e-9


# ----------------------------------------------------------------- O9 discrepancy
def _poisson_expected_2kl(lam):
    """E[2 (g ln(g/lam) + lam - g)] for g ~ Poisson(lam), summed numerically."""
    out = np.empty_like(lam)
    for i, l in enumerate(lam):
        kmax = int(l + 12 * np.sqrt(l) + 30)
        k = np.arange(kmax + 1, dtype=float)
        pmf = stats.poisson.pmf(k, l)
        out[i] = 2 * np.sum(pmf * special.kl_div(k, l))
    return out


def test_discrepancy_of_true_object_near_one():
    """Sect. 3.3: E[J(f_true; g)] is close to N^2/2, so D(f_true) ~ 1."""
    w = W.config0()
    P = O.Problem(w.g, w.psf, w.b)
    D_true = P.discrepancy(P.kl(w.f_true))
    lam = (W.blur_periodic(w.f_true, w.psf[0].astype(np.float64)) + w.b[0]).ravel()
    grid = np.geomspace(lam.min() * 0.999, lam.max() * 1.001, 400)
    expect = np.interp(np.log(lam), np.log(grid), _poisson_expected_2kl(grid)).mean()
    # std of the mean of 2 KL terms over 65536 pixels is ~0.006
    assert abs(D_true - expect) < 0.03
    assert 0.9 < expect < 1.1


def test_sgp_flux_constraint_keeps_flux():
    """With the flux constraint every iterate has sum f = c and J decreases."""
    w = W.small_single(64, 80)
    P = O.Problem(w.g, w.psf, w.b)
    prm = O.Params(max_iter=25, flux_constraint=True)
    c = P.flux_value(prm)
    f, info = P.sgp(P.start("flat"), prm)
    assert abs(f.sum() - c) <= 1e-9 * c
    assert f.min() >= 0
    h = np.array(info["history"])
    assert np.all(np.diff(h) <= 0)
