"""Mosaic of boundary-corrected subdomains on the GPU (one batch of windows,
cores stitched) against the oracle's composition, plus the delta-PSF
identity and argument checks."""
import numpy as np
import pytest

from oracle import sgp as O
from synth import workloads as W

pytestmark = pytest.mark.gpu


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


def _case():
    # the paper's layout: 256 x 256 image, four 128 x 128 cores seen through
    # 160 x 160 windows, each in a 256 x 256 domain
    w = W.star_field(210, 0, 256, 256, 60, 2.0, 10.0)
    return w.g[0], W.gaussian_psf(256, 256, 2.0).astype(np.float32), 10.0


@pytest.mark.parametrize("method,n", [("rl", 20), ("sgp", 4)])
def test_mosaic_matches_oracle(torch_dev, method, n):
    import paper_1210_2258_amd as m
    torch = torch_dev
    g, psf, b = _case()
    kind = m.KIND_RL if method == "rl" else m.KIND_SGP
    f, rep = m.mosaic_deconv(_dev(torch, g), _dev(torch, psf), b, 128, 32, kind=kind, max_iter=n)
    fo, infos = O.mosaic(g, psf, b, 128, 32, method=method, n_iter=n)
    assert rep["iters"] == n
    assert _rel(f.cpu().numpy(), fo) <= 1e-4, _rel(f.cpu().numpy(), fo)
    assert abs(rep["kl"] - sum(i["kl"] for i in infos)) <= 1e-6 * sum(i["kl"] for i in infos)


def test_mosaic_delta_psf_returns_the_image(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    rng = np.random.default_rng(4)
    g = rng.poisson(40.0, (128, 192)).astype(np.float32) + 1.0
    N = 128
    psf = np.zeros((N, N), np.float32)
    psf[N // 2, N // 2] = 1.0
    f, rep = m.mosaic_deconv(_dev(torch, g), _dev(torch, psf), 0.0, 64, 16, kind=m.KIND_RL, max_iter=1)
    assert np.allclose(f.cpu().numpy(), g, rtol=2e-6)


def test_mosaic_rejects_bad_tilings(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    g = torch.ones((100, 128), device="cuda")
    psf = torch.ones((128, 128), device="cuda")
    with pytest.raises(m.SgpError) as e:
        m.mosaic_deconv(g, psf, 1.0, 64, 8)
    assert e.value.code == -1
    g = torch.ones((128, 128), device="cuda")
    with pytest.raises(m.SgpError) as e:
        m.mosaic_deconv(g, psf, 1.0, 64, 40)   # 64 + 80 > 128
    assert e.value.code == -1
