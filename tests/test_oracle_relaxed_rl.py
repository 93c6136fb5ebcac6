"""Pins of the oracle's multiplicative relaxation of RL (Sect. 1, Eq. (RL1)):
closed forms for the identity operator, the fixed point of noise-free data,
the RL special case, the reading for several images, and the reduction of
the iteration count by about the exponent that the paper reports from the
cited work."""
import numpy as np
import pytest

from oracle import sgp as O
from synth import workloads as W


def _delta_problem(g, b):
    ny, nx = g.shape[-2:]
    psf = np.zeros((ny, nx))
    psf[ny // 2, nx // 2] = 1.0  # centred delta: A is the identity
    return O.Problem(g, psf, b)


@pytest.mark.parametrize("a", [1.0, 1.5, 1.9])
def test_identity_operator_closed_form(a):
    """A = I: one RL1 step is f (g / (f + b))^a, written out directly."""
    rng = np.random.default_rng(3)
    g = rng.poisson(40.0, (20, 24)).astype(np.float64)
    b = 2.5
    P = _delta_problem(g, b)
    f = rng.uniform(0.5, 80.0, (20, 24))
    ref = f * (g / (f + b)) ** a
    assert np.allclose(P.rl_step(f, a), ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("a", [1.3, 1.9])
def test_noise_free_data_is_a_fixed_point(a):
    """g = A f* + b exactly gives q(f*) = 1, so f* is left unchanged."""
    w = W.small_single(32, 40)
    P0 = O.Problem(w.g, w.psf, w.b)
    rng = np.random.default_rng(9)
    fs = rng.uniform(1.0, 50.0, (32, 40))
    g = P0.A(0, fs) + float(w.b[0])
    P = O.Problem(g[None], w.psf, w.b)
    assert np.allclose(P.rl_step(fs, a), fs, rtol=1e-10)


def test_exponent_one_is_rl():
    w = W.small_single(32, 40)
    P = O.Problem(w.g, w.psf, w.b)
    f0 = P.start("flat")
    fa, _ = P.rl(f0, 5, O.Params(max_iter=5, rl_alpha=1.0))
    # RL of Eq. (RL) written out with the operator only
    f = f0.copy()
    for _ in range(5):
        f = f * P.AT(0, P.g[0] / (P.A(0, f) + float(w.b[0])))
    assert np.allclose(fa, f, rtol=1e-12)


def test_multi_image_reading():
    """Several images: the relaxed factor is the RL factor of Eq. (multipleRL),
    (1/p) sum_j A_j^T (g_j / (A_j f + b_j)), raised to the power a."""
    w = W.small_multi(24, 24, p=3)
    P = O.Problem(w.g, w.psf, w.b)
    f = P.start("flat") * np.linspace(0.5, 1.5, 24 * 24).reshape(24, 24)
    s = sum(P.AT(j, P.g[j] / (P.A(j, f) + float(w.b[j]))) for j in range(3))
    assert np.allclose(P.rl_step(f, 1.7), f * (s / 3.0) ** 1.7, rtol=1e-12)


def test_boundary_support_is_kept():
    w = W.small_boundary(48, 40, 32, 24, 8, 8)
    P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
    f = P.rl_step(P.start("flat"), 1.6)
    assert np.all(f[P.MR == 0] == 0) and np.all(f >= 0)


def test_iterations_fall_by_about_the_exponent():
    """The relaxation cuts the iterations to a given level by roughly the
    exponent (Sect. 1, after Eq. (RL1)); measured on the 64 x 80 field:
    157 RL iterations to the discrepancy level, 105 at a = 1.5, 82 at 1.9."""
    w = W.small_single(64, 80)
    P = O.Problem(w.g, w.psf, w.b)
    f0 = P.start("flat")
    n = {}
    for a in (1.0, 1.5, 1.9):
        _, info = P.rl(f0, 2000, O.Params(max_iter=2000, stop=O.STOP_DISCREPANCY, rl_alpha=a))
        assert info["reason"] == O.REASON_DISCREPANCY
        n[a] = info["iters"]
    for a in (1.5, 1.9):
        assert 0.8 * a <= n[1.0] / n[a] <= 1.2 * a, (a, n)
