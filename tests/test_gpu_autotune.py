"""Tile variants of the FFT kernels and the autotuner on the GPU: variant
combinations (workgroup shapes and transform plans) against the oracle to
the parity bar (single, multi, boundary, full size), a batch under a
non-default schedule equal to its single runs, and the autotuner's choice
landing in the table."""
import numpy as np
import pytest

from oracle import sgp as O
from synth import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [16, 32, 64, 128, 256, 512, 1024, 2048, 80, 160, 320, 640, 1280]
# (row variant, column variant): bit 0 the workgroup shape, bit 1 the transform plan
COMBOS = [(0, 1), (1, 0), (1, 1), (2, 2), (3, 3), (2, 0), (0, 3)]


def _points(L, v):
    import paper_1210_2258_amd as m
    t = m.tile_info(L, v)
    return L * t["row_pairs"] // t["row_threads"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_2258_amd as m
    m.load()
    return torch


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    import paper_1210_2258_amd as m
    for L in SIZES:
        m.set_tile_schedule(L, 0, 0)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _solve(torch, w, n):
    import paper_1210_2258_amd as m
    if w.domain is not None:
        return m.sgp_boundary_deconv(_dev(torch, w.g), _dev(torch, w.psf), w.b, w.domain, max_iter=n, trace=True)
    if w.p > 1:
        return m.sgp_multi_deconv(_dev(torch, w.g), _dev(torch, w.psf), w.b, max_iter=n, trace=True)
    return m.sgp_deconv(_dev(torch, w.g[0]), _dev(torch, w.psf[0]), float(w.b[0]), max_iter=n, trace=True)


CASES = {
    "single_c0_256": (W.config0, 12),  # the fixed-count windows of test_gpu_parity.py
    "single_64x80": (lambda: W.small_single(64, 80), 6),
    "multi_3x64": (lambda: W.small_multi(64, 64), 4),
    "boundary_64x48_in_80x64": (lambda: W.small_boundary(80, 64, 64, 48, 8, 8), 4),
}


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("case", list(CASES))
def test_variant_parity(torch_dev, case, combo):
    import paper_1210_2258_amd as m
    make, n = CASES[case]
    w = make()
    NY, NX = (w.domain[0], w.domain[1]) if w.domain is not None else w.g.shape[-2:]
    m.set_tile_schedule(NX, combo[0], m.get_tile_schedule(NX)[1])
    m.set_tile_schedule(NY, m.get_tile_schedule(NY)[0], combo[1])
    f, rep = _solve(torch_dev, w, n)
    m.set_tile_schedule(NX, 0, 0)
    m.set_tile_schedule(NY, 0, 0)
    f0, rep0 = _solve(torch_dev, w, n)
    P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
    fo, io = P.sgp(P.start("flat"), O.Params(max_iter=n))
    assert rep["iters"] == n
    for k in range(n):
        assert int(rep["trace"]["backtracks"][k]) == io["log"][k]["backtracks"], k
    assert _rel(f.cpu().numpy(), fo) <= 1e-4
    assert abs(rep["kl"] - io["kl"]) <= 1e-6 * io["kl"]
    # under the default transform plans the variants share the per-pixel
    # arithmetic: only the grouping of the FP64 partial sums may differ
    # (another plan rounds the transforms differently: the oracle bar above)
    if _points(NX, combo[0]) == _points(NX, 0) and _points(NY, combo[1]) == _points(NY, 0):
        assert _rel(f.cpu().numpy(), f0.cpu().numpy().astype(np.float64)) <= 1e-6
        assert abs(rep["kl"] - rep0["kl"]) <= 1e-9 * rep0["kl"]


@pytest.fixture(scope="module")
def c1_oracle():
    w = W.config1()
    P = O.Problem(w.g, w.psf, w.b)
    return w, P.sgp(P.start("flat"), O.Params(max_iter=10))


@pytest.mark.parametrize("combo", COMBOS)
def test_variant_parity_full_size(torch_dev, c1_oracle, combo):
    """2048x2048 under 512-thread row workgroups and/or two-column
    workgroups (variants 2 and 3 equal 0 and 1 there: no second plan)."""
    import paper_1210_2258_amd as m
    w, (fo, io) = c1_oracle
    m.set_tile_schedule(2048, *combo)
    f, rep = _solve(torch_dev, w, 10)
    for k in range(10):
        assert int(rep["trace"]["backtracks"][k]) == io["log"][k]["backtracks"], k
    assert _rel(f.cpu().numpy(), fo) <= 1e-4
    assert abs(rep["kl"] - io["kl"]) <= 1e-6 * io["kl"]


@pytest.mark.parametrize("shape", [(2048, 2048), (2048, 160), (1024, 80), (1280, 1280), (512, 256),
                                   (256, 1024)])
@pytest.mark.parametrize("combo", COMBOS)
def test_operator_under_variants(torch_dev, shape, combo):
    """A and A^T under every tile combination (two-column register path at
    2048, two 640-thread columns at 1280, four points per thread from 128 to
    1280) against the oracle's FFT convolution."""
    import paper_1210_2258_amd as m
    torch = torch_dev
    ny, nx = shape
    rng = np.random.default_rng(ny + nx)
    psf = rng.random((ny, nx)) * W.gaussian_psf(ny, nx, 3.0)
    psf[ny // 2 + 1, nx // 2 - 2] += 0.3 * psf.max()   # asymmetric
    x = (rng.random((ny, nx)) * 100).astype(np.float32).astype(np.float64)
    P = O.Problem(np.ones((ny, nx)), psf.astype(np.float32), 1.0)
    m.set_tile_schedule(nx, combo[0], m.get_tile_schedule(nx)[1])
    m.set_tile_schedule(ny, m.get_tile_schedule(ny)[0], combo[1])
    for adj in (False, True):
        out = m.apply_operator(_dev(torch, psf), _dev(torch, x), adjoint=adj).cpu().numpy()
        ref = P.AT(0, x) if adj else P.A(0, x)
        assert _rel(out, ref) < 2e-6, (shape, combo, adj, _rel(out, ref))


def test_single_1024_parity(torch_dev):
    """A 1024x1024 star field (two columns per workgroup on the register
    path by default), 10 SGP iterations against the oracle."""
    w = W.star_field(300, 1024, 1024, 1024, 100, 2.0, 10.0)
    f, rep = _solve(torch_dev, w, 10)
    P = O.Problem(w.g, w.psf, w.b)
    fo, io = P.sgp(P.start("flat"), O.Params(max_iter=10))
    for k in range(10):
        assert int(rep["trace"]["backtracks"][k]) == io["log"][k]["backtracks"], k
    assert _rel(f.cpu().numpy(), fo) <= 1e-4
    assert abs(rep["kl"] - io["kl"]) <= 1e-6 * io["kl"]


def test_batch_under_variants_equals_single_runs(torch_dev):
    """A batch of uneven sizes under variant 1 everywhere: each item equals
    its own single run under the same schedule bit for bit."""
    import paper_1210_2258_amd as m
    torch = torch_dev
    for L in (64, 80, 128, 160, 256):
        m.set_tile_schedule(L, 1, 1)
    ws = [W.star_field(200, i, ny, nx, 30, 1.0 + 0.4 * i, 5.0 + 5 * i)
          for i, (ny, nx) in enumerate([(64, 64), (128, 128), (80, 160), (256, 256)])]
    gs = [_dev(torch, w.g[0]) for w in ws]
    ps = [_dev(torch, w.psf[0]) for w in ws]
    bs = [float(w.b[0]) for w in ws]
    fb, reps = m.batch_deconv(gs, ps, bs, max_iter=12)
    for i in range(len(ws)):
        f1, r1 = m.sgp_deconv(gs[i], ps[i], bs[i], max_iter=12)
        assert torch.equal(fb[i], f1), i
        assert reps[i]["kl"] == r1["kl"]


def test_autotune_sets_the_table(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    w = W.config0()
    g, psf = _dev(torch, w.g[0]), _dev(torch, w.psf[0])
    r, c, ms = m.autotune(g, psf, float(w.b[0]), iters=32)
    # at 256 every variant is distinct: two shapes under each of two plans
    assert (r, c) in ms and set(ms) == {(i, j) for i in range(4) for j in range(4)}
    assert all(t > 0 for t in ms.values())
    # the fastest, unless within 1% of the default shape
    if (r, c) == (0, 0):
        assert min(ms.values()) >= 0.99 * ms[(0, 0)], ms
    else:
        assert ms[(r, c)] == min(ms.values()) and ms[(r, c)] < 0.99 * ms[(0, 0)], ms
    assert m.get_tile_schedule(256) == (r, c)
    # a solve under the tuned schedule is still the oracle's
    f, rep = m.sgp_deconv(g, psf, float(w.b[0]), max_iter=20)
    P = O.Problem(w.g, w.psf, w.b)
    fo, io = P.sgp(P.start("flat"), O.Params(max_iter=20))
    assert _rel(f.cpu().numpy(), fo) <= 1e-4


def test_autotune_rejects_bad_arguments(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    w = W.small_single(64, 80)
    g, psf = _dev(torch, w.g[0]), _dev(torch, w.psf[0])
    m.set_tile_schedule(80, 1, 0)
    with pytest.raises(m.SgpError):
        m.autotune(g, psf, float(w.b[0]), iters=0)
    assert m.get_tile_schedule(80) == (1, 0)  # unchanged on error
