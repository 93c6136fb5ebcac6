"""The entry point that allocates nothing (sgp_deconv_noalloc, its workspace
in the library's static device array) against sgp_deconv on the same inputs:
two calls in a row, the second on a smaller image, then a size beyond the
static workspace (rejected before any device work) and one more call."""
import numpy as np
import pytest

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


def _check(torch, w, **kw):
    import paper_1210_2258_amd as m
    g, psf, b = _dev(torch, w.g[0]), _dev(torch, w.psf[0]), float(w.b[0])
    f_ref, r_ref = m.sgp_deconv(g, psf, b, **kw)
    f = torch.full_like(g, -7.0)
    f2, rep = m.sgp_deconv_noalloc(g, psf, b, f=f, **kw)
    torch.cuda.synchronize()
    print(f"noalloc {tuple(g.shape)} {kw}: iters {rep['iters']} vs {r_ref['iters']}", flush=True)
    assert f2.data_ptr() == f.data_ptr()
    assert rep["iters"] == r_ref["iters"] and rep["reason"] == r_ref["reason"]
    assert torch.equal(f, f_ref)       # same kernels, same reduction order: bit for bit
    assert rep["kl"] == r_ref["kl"] and rep["L1"] == r_ref["L1"] and rep["L2"] == r_ref["L2"]
    rel = float(torch.linalg.vector_norm(f - f_ref) / torch.linalg.vector_norm(f_ref))
    assert rel <= 1e-4


def test_noalloc_matches_sgp_deconv(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    _check(torch, W.config0(), max_iter=30)                          # 256 x 256
    _check(torch, W.small_single(64, 80), max_iter=20)               # then a smaller image
    _check(torch, W.small_single(64, 80), max_iter=400, stop=m.STOP_DISCREPANCY)
    # a size beyond the 64 MiB workspace is refused on the host
    g = torch.ones((2048, 2048), device="cuda")
    with pytest.raises(m.SgpError) as e:
        m.sgp_deconv_noalloc(g, g, 1.0, f=torch.empty_like(g), max_iter=1)
    assert e.value.code == -1 and "MiB" in str(e.value)
    _check(torch, W.config0(), max_iter=12)
