"""Pins of the oracle's OSEM (Algorithm 2, Eqs. (OSEMstep), (boundaryOSEM))
against what the mathematics fixes: with one image a cycle is the RL step of
Eq. (RL) written independently here, each sub-step of a periodic problem
with b = 0 carries the flux of its own image, a delta PSF with b = 0 gives
the last image exactly, and the weights vanish outside R."""
import numpy as np
import pytest

from oracle import sgp as O
from synth import workloads as W


def _rl_step_direct(g, psf, b, f):
    """Periodic single-image RL written out with numpy FFTs:
    f * K^T (g / (K f + b)), K the unit-sum PSF centred at (ny//2, nx//2)."""
    K = psf / psf.sum()
    Kh = np.fft.fft2(np.fft.ifftshift(K))
    y = np.real(np.fft.ifft2(Kh * np.fft.fft2(f))) + b
    return f * np.real(np.fft.ifft2(np.conj(Kh) * np.fft.fft2(g / y)))


def test_one_image_cycle_is_the_rl_step():
    w = W.small_single(32, 40)
    P = O.Problem(w.g, w.psf, w.b)
    f0 = P.start("flat")
    ref = _rl_step_direct(w.g[0].astype(np.float64), w.psf[0].astype(np.float64), float(w.b[0]), f0)
    assert np.allclose(P.osem_cycle(f0), ref, rtol=1e-12, atol=0)
    f, info = P.osem(f0, 5)
    fr, _ = P.rl(f0, 5)
    assert np.allclose(f, fr, rtol=1e-11) and info["iters"] == 5


def test_each_substep_keeps_its_image_flux():
    """b = 0, periodic, unit-sum PSF: sum h^(j) = sum g_j after sub-step j
    (sum_n h A^T(g/Ah) = sum_m Ah (g/Ah) = sum g)."""
    w = W.small_multi(32, 32, p=3)
    P = O.Problem(w.g, w.psf, np.zeros(3))
    h = P.start("flat") + 1.0
    for j in range(3):
        h = P.osem_weight(j) * h * P.AT(j, P.g[j] / P.y(j, h))
        assert abs(h.sum() - P.g[j].sum()) <= 1e-9 * P.g[j].sum(), j
    assert np.allclose(P.osem_cycle(P.start("flat") + 1.0), h, rtol=1e-12)


def test_delta_psf_gives_the_last_image():
    rng = np.random.default_rng(5)
    g = rng.poisson(50.0, (3, 16, 16)).astype(np.float64) + 1.0
    psf = np.zeros((3, 16, 16))
    psf[:, 8, 8] = 1.0
    P = O.Problem(g, psf, np.zeros(3))
    f = P.osem_cycle(np.full((16, 16), 7.0))
    assert np.allclose(f, g[2], rtol=1e-12)


def test_boundary_weights_and_support():
    w = W.small_boundary(48, 40, 32, 24, 8, 8)
    P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
    for j in range(P.p):
        wj = P.osem_weight(j)
        assert np.all(wj[P.MR == 0] == 0)
        inR = P.MR > 0
        assert np.allclose(wj[inR] * P.alpha_j[j][inR], 1.0)
    f = P.osem_cycle(P.start("flat"))
    assert np.all(f[P.MR == 0] == 0) and np.all(f >= 0)
    # with one image the boundary cycle is the boundary RL step of Eq. (boundaryRL)
    assert np.allclose(f, P.rl_step(P.start("flat")), rtol=1e-12)


def test_osem_cycle_lowers_kl_on_a_multi_image_problem():
    w = W.small_multi(32, 32, p=3)
    P = O.Problem(w.g, w.psf, w.b)
    f, info = P.osem(P.start("flat"), 10)
    h = info["history"]
    assert h[-1] < h[0] and len(h) == 11


def test_boundary_multi_image_substep_flux():
    """b = 0 with boundary correction: alpha_j o h^(j) summed over R equals
    the flux of g_j on S (sum_n h A_j^T r = sum_S (A_j h) r), which singles out
    the per-image weight M_R / alpha_j of Eq. (boundaryOSEM)."""
    w = W.small_boundary(48, 40, 32, 24, 8, 8)
    NY, NX = w.domain[0], w.domain[1]
    g = np.stack([w.g[0], w.g[0][::-1, ::-1]]).astype(np.float64)
    psf = np.stack([w.psf[0], W.gaussian_psf(NY, NX, 3.0)]).astype(np.float64)
    P = O.Problem(g, psf, np.zeros(2), domain=w.domain)
    h = P.start("flat") + 1.0 * P.MR
    for j in range(2):
        h = P.osem_weight(j) * h * P.AT(j, P.g[j] / P.y(j, h))
        assert abs((P.alpha_j[j] * h).sum() - P.g[j].sum()) <= 1e-9 * P.g[j].sum(), j
    assert not np.allclose(P.osem_weight(0), P.invw)  # two images: alpha_j differs from sum_j alpha_j
