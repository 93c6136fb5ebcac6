"""Pins of the oracle's mosaic of boundary-corrected subdomains: the tiles
cover the image once, a delta PSF with b = 0 makes every boundary RL step
return the data on its window so the mosaic is the image itself (this fixes
every offset of the stitching), and a single tile is the boundary problem."""
import numpy as np

from oracle import sgp as O
from synth import workloads as W


def test_tiles_cover_the_image_once():
    H, W_, core, margin, N = 64, 96, 32, 8, 64
    cover = np.zeros((H, W_), int)
    for cy, cx, wy, wx, (oy, ox) in O.mosaic_tiles(H, W_, core, margin, N):
        cover[cy[0]:cy[1], cx[0]:cx[1]] += 1
        assert wy[0] <= cy[0] and cy[1] <= wy[1] and wx[0] <= cx[0] and cx[1] <= wx[1]
        assert 0 <= oy and oy + (wy[1] - wy[0]) <= N and 0 <= ox and ox + (wx[1] - wx[0]) <= N
    assert np.all(cover == 1)


def test_delta_psf_mosaic_is_the_image():
    rng = np.random.default_rng(3)
    H, W_, core, margin, N = 64, 64, 32, 8, 64
    g = rng.poisson(40.0, (H, W_)).astype(np.float64) + 1.0
    psf = np.zeros((N, N))
    psf[N // 2, N // 2] = 1.0
    m, infos = O.mosaic(g, psf, 0.0, core, margin, method="rl", n_iter=1)
    assert np.allclose(m, g, rtol=1e-12)


def test_single_tile_is_the_boundary_problem():
    w = W.small_boundary(80, 64, 64, 48, 8, 8)
    g = w.g[0].astype(np.float64)[:48, :48]
    N = 80
    psf = W.gaussian_psf(N, N, 2.0)
    m, infos = O.mosaic(g, psf, 8.0, 48, 0, method="rl", n_iter=7)
    P = O.Problem(g, psf, 8.0, domain=(N, N, 16, 16))
    f, _ = P.rl(P.start("flat"), 7)
    assert np.allclose(m, f[16:64, 16:64], rtol=1e-13)
