"""Fourier re-binning of the size sweep (Sect. 4.1, third experiment): the
spectrum of an image is zero-padded to twice the size around the zero
frequency and the zero-frequency coefficient is multiplied by four.  Checked
against what the construction fixes, on an image whose re-binning has no
ringing below zero (so the clip does not act):

* the mean level is kept (the background is unchanged);
* the zero-frequency coefficient of the result is four times the original's
  (a 4x larger array), every other in-band coefficient is the original's;
* nothing appears outside the original band;
* the samples at even positions equal mean + (g - mean) / 4, the closed form
  of band-limited interpolation with this normalisation;
* the sweep's series doubles the size at each step and keeps the PSF at
  unit volume."""
import numpy as np

from synth import workloads as W


def _image(n=32, seed=3):
    rng = np.random.default_rng(seed)
    g = 200.0 + rng.poisson(20.0, size=(n, n)).astype(np.float64)   # high background: no ringing below 0
    return g


def test_rebin_keeps_mean_and_scales_dc():
    g = _image()
    r = W.rebin_fourier(g)
    assert r.shape == (64, 64)
    assert r.min() > 0
    assert abs(r.mean() - g.mean()) <= 1e-12 * g.mean()
    Fg, Fr = np.fft.fft2(g), np.fft.fft2(r)
    assert abs(Fr[0, 0] - 4.0 * Fg[0, 0]) <= 1e-12 * abs(Fg[0, 0])


def test_rebin_adds_no_content_outside_the_band():
    g = _image()
    n = g.shape[0]
    Fg = np.fft.fftshift(np.fft.fft2(g))
    Fr = np.fft.fftshift(np.fft.fft2(W.rebin_fourier(g)))
    scale = np.abs(Fg).max()
    # the band |k| <= n/2 (the real part mirrors the unpaired Nyquist
    # row / column of the original to +n/2)
    inside = np.zeros(Fr.shape, bool)
    inside[n // 2:n // 2 + n + 1, n // 2:n // 2 + n + 1] = True
    assert np.abs(Fr[~inside]).max() <= 1e-11 * scale
    # in-band coefficients other than the zero frequency are the original's
    # (the real part taken at the end halves the unpaired Nyquist row/column)
    inner = Fr[n // 2 + 1:n // 2 + n, n // 2 + 1:n // 2 + n].copy()
    ref = Fg[1:, 1:].copy()
    c = n // 2 - 1
    inner[c, c] = ref[c, c] = 0.0   # the zero frequency (x4), checked above
    assert np.abs(inner - ref).max() <= 1e-11 * scale


def test_rebin_samples_closed_form():
    g = _image(24, seed=5)
    r = W.rebin_fourier(g)
    m = g.mean()
    np.testing.assert_allclose(r[::2, ::2], m + (g - m) / 4.0, rtol=0, atol=1e-10 * g.max())


def test_rebin_series_sizes_and_psf():
    w = W.rebin_base(size=64, total=1e5)
    ser = W.rebin_series(w, sizes=(64, 128, 256))
    assert [s for s, _, _ in ser] == [64, 128, 256]
    for s, g, psf in ser:
        assert g.shape == psf.shape == (s, s)
        assert g.dtype == np.float32 and g.min() >= 0
        assert abs(float(psf.astype(np.float64).sum()) - 1.0) < 1e-5
    # the mean level (background plus object) carries over from size to size
    means = [float(g.astype(np.float64).mean()) for _, g, _ in ser]
    assert max(means) - min(means) <= 1e-3 * means[0]
