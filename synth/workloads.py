"""Synthetic stand-ins for the paper's astronomical test images.

The paper's HST images, AO PSF and LINC-NIRVANA PSFs are not available; these
generators produce seeded images with the same kind of content (point sources,
extended profiles, Poisson counts over a constant background) at the sizes the
benchmarks use.  Recipe per workload:

* ``config0``: 256x256, 100 point sources at integer positions uniform on the
  torus, fluxes 10^U(2,5), Gaussian PSF sigma = 2 px, b = 10.
* ``config1``: 2048x2048, 20 circular Sersic profiles (n ~ U[0.5, 4],
  r_e ~ U[5, 80] px) plus 500 stars (fluxes 10^U(2,5)), total 1e8 counts;
  Airy PSF with first zero at 4 px (weight 0.99) plus a Gaussian halo of
  sigma 20 px (weight 0.01); b = 50.
* ``config2``: 3 images of 1024x1024 of one object (150-star cluster,
  Gaussian spatial sigma 80 px, plus an n=1 Sersic nebula with r_e = 150 px and
  axis ratio 0.7; 30 % / 70 % of 1e7 counts); PSF_j = Airy envelope (first
  zero 16.7 px) times cos^2 fringes of 8 px period at 0/60/120 degrees; b = 20.
* ``config3``: object on 1280x1280 (2000 stars plus a linear ramp from 5 to 50
  counts/px), Gaussian PSF sigma 6 px on 1280x1280, only the central 1024x1024
  observed; b = 30.
* ``config4``: 512 star fields as config0 with sizes uniform in
  {128, 256, 512, 1024}^2, PSF sigma ~ U[1, 4], b ~ U[5, 50].

Every random draw comes from ``numpy.random.default_rng`` seeded with
``SeedSequence(12102258, spawn_key=(cfg, img, purpose))``.  Blurring is a
periodic FFT convolution in float64 (clipped at 0), followed by Poisson noise;
images and PSFs are handed out as float32 (counts are exact integers).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 12102258

PURPOSE = {"object": 0, "noise": 1, "psf": 2, "size": 3, "train": 4, "misc": 5}


def rng_for(cfg: int, img: int, purpose: str | int) -> np.random.Generator:
    key = PURPOSE[purpose] if isinstance(purpose, str) else int(purpose)
    return np.random.default_rng(np.random.SeedSequence(ROOT_SEED, spawn_key=(cfg, img, key)))


@dataclass
class Workload:
    name: str
    g: np.ndarray              # [p, ny, nx] float32 counts
    psf: np.ndarray            # [p, NY, NX] float32, unit sum, centre (NY//2, NX//2)
    b: np.ndarray              # [p] float32 constant backgrounds
    f_true: np.ndarray         # [NY, NX] float64 object
    domain: tuple | None = None   # (NY, NX, oy, ox) for boundary problems
    extra: dict = field(default_factory=dict)

    @property
    def p(self):
        return self.g.shape[0]


def _centred_grid(ny, nx):
    y = np.arange(ny, dtype=np.float64) - ny // 2
    x = np.arange(nx, dtype=np.float64) - nx // 2
    return np.meshgrid(y, x, indexing="ij")


def gaussian_psf(ny, nx, sigma):
    """Pixel-centre-sampled Gaussian centred at (ny//2, nx//2), unit sum."""
    Y, X = _centred_grid(ny, nx)
    k = np.exp(-(X * X + Y * Y) / (2.0 * sigma * sigma))
    return k / k.sum()


def _airy(r, r0):
    from scipy.special import j1
    x = 3.8317059702075125 * r / r0
    out = np.ones_like(x)
    nz = x > 0
    out[nz] = (2.0 * j1(x[nz]) / x[nz]) ** 2
    return out


def airy_psf(ny, nx, r0=4.0, halo_sigma=20.0, halo_weight=0.01):
    """Airy pattern with first zero at r0 px plus a Gaussian halo, unit sum."""
    Y, X = _centred_grid(ny, nx)
    a = _airy(np.hypot(X, Y), r0)
    a /= a.sum()
    h = gaussian_psf(ny, nx, halo_sigma)
    k = (1.0 - halo_weight) * a + halo_weight * h
    return k / k.sum()


def fringe_psf(ny, nx, theta_deg, r0=16.7, period=8.0):
    """Interferometric PSF: Airy envelope times cos^2 fringes, unit sum."""
    Y, X = _centred_grid(ny, nx)
    a = _airy(np.hypot(X, Y), r0)
    th = np.deg2rad(theta_deg)
    fr = np.cos(np.pi * (X * np.cos(th) + Y * np.sin(th)) / period) ** 2
    k = a * fr
    return k / k.sum()


def blur_periodic(obj, psf):
    """Simulated imaging: periodic FFT blur of obj by a centred PSF."""
    K0 = np.fft.ifftshift(psf)
    out = np.fft.irfft2(np.fft.rfft2(K0) * np.fft.rfft2(obj), s=obj.shape)
    return np.maximum(out, 0.0)


def point_sources(ny, nx, n, rng, lo=2.0, hi=5.0):
    obj = np.zeros((ny, nx))
    ys = rng.integers(0, ny, n)
    xs = rng.integers(0, nx, n)
    fl = 10.0 ** rng.uniform(lo, hi, n)
    np.add.at(obj, (ys, xs), fl)
    return obj


def _sersic_bn(n):
    # Ciotti & Bertin (1999) asymptotic expansion of b_n
    return (2.0 * n - 1.0 / 3.0 + 4.0 / (405.0 * n) + 46.0 / (25515.0 * n ** 2)
            + 131.0 / (1148175.0 * n ** 3) - 2194697.0 / (30690717750.0 * n ** 4))


def sersic_image(ny, nx, cy, cx, n, re, q=1.0, pa=0.0):
    """Sersic profile on the torus (periodic distances), unnormalised."""
    y = np.arange(ny, dtype=np.float64) - cy
    x = np.arange(nx, dtype=np.float64) - cx
    y = (y + ny / 2) % ny - ny / 2
    x = (x + nx / 2) % nx - nx / 2
    Y, X = np.meshgrid(y, x, indexing="ij")
    c, s = np.cos(pa), np.sin(pa)
    u = X * c + Y * s
    v = (-X * s + Y * c) / q
    r = np.hypot(u, v)
    return np.exp(-_sersic_bn(n) * ((r / re) ** (1.0 / n) - 1.0))


def _observe(obj, psf, b, rng):
    lam = blur_periodic(obj, psf) + b
    return rng.poisson(lam).astype(np.float32)


def star_field(cfg, img, ny, nx, nstars, sigma, b):
    rng = rng_for(cfg, img, "object")
    obj = point_sources(ny, nx, nstars, rng)
    psf = gaussian_psf(ny, nx, sigma)
    g = _observe(obj, psf, b, rng_for(cfg, img, "noise"))
    return Workload(f"stars{ny}x{nx}", g[None], psf.astype(np.float32)[None],
                    np.array([b], np.float32), obj)


def config0():
    w = star_field(0, 0, 256, 256, 100, 2.0, 10.0)
    w.name = "c0_stars_256"
    return w


def config1(size=2048, total=1e8, seed_img=0):
    ny = nx = size
    rng = rng_for(1, seed_img, "object")
    stars = point_sources(ny, nx, 500, rng)
    gal = np.zeros((ny, nx))
    for _ in range(20):
        n = rng.uniform(0.5, 4.0)
        re = rng.uniform(5.0, 80.0) * size / 2048.0
        cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
        prof = sersic_image(ny, nx, cy, cx, n, re)
        gal += 10.0 ** rng.uniform(0.0, 2.0) * prof / prof.sum()
    rest = max(total - stars.sum(), 0.0)
    obj = stars + rest * gal / gal.sum()
    psf = airy_psf(ny, nx, 4.0 * size / 2048.0 if size < 2048 else 4.0)
    g = _observe(obj, psf, 50.0, rng_for(1, seed_img, "noise"))
    return Workload(f"c1_galaxy_{size}", g[None], psf.astype(np.float32)[None],
                    np.array([50.0], np.float32), obj)


def config2(size=1024, total=1e7, p=3):
    ny = nx = size
    rng = rng_for(2, 0, "object")
    sc = size / 1024.0
    nst = 150
    ys = np.clip(np.rint(ny / 2 + rng.normal(0, 80 * sc, nst)), 0, ny - 1).astype(int)
    xs = np.clip(np.rint(nx / 2 + rng.normal(0, 80 * sc, nst)), 0, nx - 1).astype(int)
    fl = 10.0 ** rng.uniform(2.0, 5.0, nst)
    stars = np.zeros((ny, nx))
    np.add.at(stars, (ys, xs), fl)
    neb = sersic_image(ny, nx, ny / 2, nx / 2, 1.0, 150.0 * sc, q=0.7, pa=0.4)
    obj = 0.3 * total * stars / stars.sum() + 0.7 * total * neb / neb.sum()
    angles = [0.0, 60.0, 120.0, 30.0, 90.0, 150.0][:p]
    psfs = np.stack([fringe_psf(ny, nx, a, r0=16.7 * sc, period=max(8.0 * sc, 2.5)) for a in angles])
    g = np.stack([_observe(obj, psfs[j], 20.0, rng_for(2, j, "noise"))[...] for j in range(p)])
    return Workload(f"c2_multi_{p}x{size}", g, psfs.astype(np.float32),
                    np.full(p, 20.0, np.float32), obj)


def config3(NS=1280, S=1024, nstars=2000):
    rng = rng_for(3, 0, "object")
    obj = point_sources(NS, NS, nstars, rng)
    ramp = np.linspace(5.0, 50.0, NS)[None, :] * np.ones((NS, 1))
    obj = obj + ramp
    psf = gaussian_psf(NS, NS, 6.0 * NS / 1280.0 if NS < 1280 else 6.0)
    o = (NS - S) // 2
    lam = blur_periodic(obj, psf)[o:o + S, o:o + S] + 30.0
    g = rng_for(3, 0, "noise").poisson(lam).astype(np.float32)
    return Workload(f"c3_boundary_{S}_in_{NS}", g[None], psf.astype(np.float32)[None],
                    np.array([30.0], np.float32), obj, domain=(NS, NS, o, o))


def config4(n_images=512, sizes=(128, 256, 512, 1024), purpose_base=0):
    """Heterogeneous batch of star fields; returns a list of Workloads."""
    out = []
    for i in range(n_images):
        r = rng_for(4, purpose_base + i, "size")
        sz = int(sizes[r.integers(0, len(sizes))])
        sigma = r.uniform(1.0, 4.0)
        b = float(r.uniform(5.0, 50.0))
        w = star_field(4, purpose_base + i, sz, sz, 100, sigma, b)
        w.name = f"c4_{i}_{sz}"
        out.append(w)
    return out


# ------------------------------------------------------------- small cases
def small_single(ny=64, nx=48, nstars=20, sigma=1.5, b=10.0, seed=0):
    """Small single-image problem (several FFT tiles, non-square)."""
    rng = rng_for(100, seed, "object")
    obj = point_sources(ny, nx, nstars, rng)
    obj += 20.0 * sersic_image(ny, nx, ny / 3, nx / 2, 1.0, 6.0)
    psf = gaussian_psf(ny, nx, sigma)
    g = _observe(obj, psf, b, rng_for(100, seed, "noise"))
    return Workload(f"small_{ny}x{nx}", g[None], psf.astype(np.float32)[None],
                    np.array([b], np.float32), obj)


def small_multi(ny=64, nx=64, p=3, seed=0):
    rng = rng_for(101, seed, "object")
    obj = point_sources(ny, nx, 15, rng) + 30.0 * sersic_image(ny, nx, ny / 2, nx / 2, 1.0, 8.0, 0.7, 0.3)
    angles = [0.0, 60.0, 120.0, 30.0][:p]
    psfs = np.stack([fringe_psf(ny, nx, a, r0=3.0, period=4.0) for a in angles])
    g = np.stack([_observe(obj, psfs[j], 5.0, rng_for(101, seed * 16 + j, "noise")) for j in range(p)])
    return Workload(f"smallmulti_{p}x{ny}x{nx}", g, psfs.astype(np.float32),
                    np.full(p, 5.0, np.float32), obj)


def small_boundary(NY=80, NX=64, ny=64, nx=48, oy=8, ox=8, sigma=2.0, b=8.0, seed=0):
    rng = rng_for(102, seed, "object")
    obj = point_sources(NY, NX, 30, rng) + np.linspace(2.0, 20.0, NX)[None, :]
    psf = gaussian_psf(NY, NX, sigma)
    lam = blur_periodic(obj, psf)[oy:oy + ny, ox:ox + nx] + b
    g = rng_for(102, seed, "noise").poisson(lam).astype(np.float32)
    return Workload(f"smallbnd_{ny}x{nx}_in_{NY}x{NX}", g[None], psf.astype(np.float32)[None],
                    np.array([b], np.float32), obj, domain=(NY, NX, oy, ox))


def small_galaxy(ny=64, nx=80, total=3e4, sigma=2.0, b=10.0, seed=0, p=1):
    """Small extended object (one exponential disc, axis ratio 0.7) at low
    counts: the reconstruction error of RL and SGP reaches its minimum after
    some ten iterations and then grows as noise is amplified.  p > 1: p
    images through fringe PSFs at 0, 60, 120 ... degrees (as small_multi)."""
    obj = sersic_image(ny, nx, 0.47 * ny, nx / 2, 1.0, 8.0, 0.7, 0.3)
    obj = total * obj / obj.sum()
    if p == 1:
        psfs = gaussian_psf(ny, nx, sigma)[None]
    else:
        psfs = np.stack([fringe_psf(ny, nx, 60.0 * j, r0=3.0, period=4.0) for j in range(p)])
    g = np.stack([_observe(obj, psfs[j], b, rng_for(103, seed * 16 + j, "noise")) for j in range(p)])
    return Workload(f"galaxy_{p}x{ny}x{nx}", g, psfs.astype(np.float32),
                    np.full(p, b, np.float32), obj)


# ---------------------------------------------------- Fourier re-binning
def rebin_fourier(img):
    """Doubles the size of an image by Fourier re-binning (Sect. 4.1, third
    experiment): its FFT is zero-padded to twice the size (centred), the
    zero-frequency coefficient is multiplied by four, and the real part of
    the inverse FFT is returned.  The mean level stays the same; no new high
    frequencies appear.  Ringing below zero is clipped (the solvers need
    g >= 0)."""
    a = np.asarray(img, dtype=np.float64)
    ny, nx = a.shape
    F = np.fft.fftshift(np.fft.fft2(a))
    G = np.zeros((2 * ny, 2 * nx), dtype=complex)
    G[ny // 2:ny // 2 + ny, nx // 2:nx // 2 + nx] = F
    G = np.fft.ifftshift(G)
    G[0, 0] *= 4.0
    return np.maximum(np.real(np.fft.ifft2(G)), 0.0)


def rebin_base(size=256, total=1e7, r0=4.0, b=50.0):
    """Starting image of the size sweep: the galaxy field of the 2048^2
    workload drawn at size^2 with total counts `total`, blurred by an Airy PSF
    whose first zero is at r0 pixels (as at 2048^2), background b, Poisson noise."""
    base = config1(size=size, total=total)
    psf = airy_psf(size, size, r0)
    g = _observe(base.f_true, psf, b, rng_for(5, size, "noise"))
    return Workload(f"rebin_base_{size}", g[None], psf.astype(np.float32)[None], np.array([b], np.float32),
                    base.f_true)


def rebin_series(w, sizes=(256, 512, 1024, 2048)):
    """[(size, g, psf)] starting from a single-image workload of the first
    size, each next one the Fourier re-binning of the previous (PSF re-binned
    the same way and renormalised to unit sum)."""
    g, psf = w.g[0].astype(np.float64), w.psf[0].astype(np.float64)
    out = [(g.shape[0], g.astype(np.float32), psf.astype(np.float32))]
    while out[-1][0] < sizes[-1]:
        g = rebin_fourier(g)
        psf = rebin_fourier(psf)
        psf /= psf.sum()
        out.append((g.shape[0], g.astype(np.float32), psf.astype(np.float32)))
    return [o for o in out if o[0] in sizes]
