"""Batched runs of many uneven images: every item must equal its own single
run bit for bit (same kernels, same reduction order), stop on its own rule,
and match the oracle at the fixed-count bar."""
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


def _items():
    out = []
    for i, (ny, nx) in enumerate([(64, 64), (128, 128), (64, 64), (80, 160), (128, 128), (256, 256), (64, 64)]):
        w = W.star_field(200, i, ny, nx, 30, 1.0 + 0.4 * i, 5.0 + 5 * i)
        out.append(w)
    return out


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("stop", ["fixed", "discrepancy"])
def test_batch_equals_single_runs(torch_dev, stop):
    import paper_1210_2258_amd as m
    torch = torch_dev
    items = _items()
    gs = [_dev(torch, w.g[0]) for w in items]
    ps = [_dev(torch, w.psf[0]) for w in items]
    bs = [float(w.b[0]) for w in items]
    kw = dict(max_iter=25) if stop == "fixed" else dict(max_iter=400, stop=m.STOP_DISCREPANCY)
    fs, reps = m.batch_deconv(gs, ps, bs, **kw)
    for i in range(len(items)):
        f1, r1 = m.sgp_deconv(gs[i], ps[i], bs[i], **kw)
        assert r1["iters"] == reps[i]["iters"], (i, r1["iters"], reps[i]["iters"])
        assert r1["reason"] == reps[i]["reason"]
        assert torch.equal(f1, fs[i]), i
        assert r1["kl"] == reps[i]["kl"]
    if stop == "discrepancy":
        assert len({r["iters"] for r in reps}) > 1       # items stop on their own


def test_batch_matches_oracle(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    items = _items()[:4]
    n = 4  # small bright star fields drift fastest from FP32 rounding (see test_gpu_parity.py)
    fs, reps = m.batch_deconv([_dev(torch, w.g[0]) for w in items], [_dev(torch, w.psf[0]) for w in items],
                              [float(w.b[0]) for w in items], max_iter=n)
    for w, f, r in zip(items, fs, reps):
        P = O.Problem(w.g, w.psf, w.b)
        fo, io = P.sgp(P.start("flat"), O.Params(max_iter=n))
        assert np.linalg.norm(f.cpu().numpy() - fo) / np.linalg.norm(fo) <= 1e-4
        assert abs(r["kl"] - io["kl"]) <= 1e-6 * io["kl"]


def test_warm_start_fallback(torch_dev):
    """SGP_INIT_WARM keeps a good start and falls back to the flat start when
    the given start has the larger KL."""
    import paper_1210_2258_amd as m
    torch = torch_dev
    w = W.small_single(64, 80)
    g, psf, b = _dev(torch, w.g[0]), _dev(torch, w.psf[0]), float(w.b[0])
    good, _ = m.sgp_deconv(g, psf, b, max_iter=30)
    bad = torch.full_like(g, 1e6)
    fs, reps = m.batch_deconv([g, g], [psf, psf], [b, b], f0s=[good.clone(), bad], init=m.INIT_WARM, max_iter=5)
    assert reps[0]["used_fallback"] == 0 and reps[1]["used_fallback"] == 1
    f_flat, r_flat = m.sgp_deconv(g, psf, b, max_iter=5)
    assert torch.equal(fs[1], f_flat)
    assert reps[0]["kl"] < r_flat["kl"]


def test_batch_equals_single_large_and_boundary(torch_dev):
    """Batch items at the sizes of the 512-image benchmark batch (512^2,
    1024^2) and a boundary-corrected item on a 1280^2 domain (its 1024^2
    window at offset 128) equal their single runs bit for bit."""
    import paper_1210_2258_amd as m
    torch = torch_dev
    items = [W.star_field(201, 0, 512, 512, 100, 2.0, 20.0), W.star_field(201, 1, 1024, 1024, 100, 3.0, 10.0),
             W.config3(), W.star_field(201, 2, 256, 256, 100, 1.5, 40.0)]
    gs = [_dev(torch, w.g[0]) for w in items]
    ps = [_dev(torch, w.psf[0]) for w in items]
    bs = [float(w.b[0]) for w in items]
    doms = [w.domain for w in items]
    kw = dict(max_iter=20)
    fs, reps = m.batch_deconv(gs, ps, bs, domains=doms, **kw)
    for i, w in enumerate(items):
        if w.domain is None:
            f1, r1 = m.sgp_deconv(gs[i], ps[i], bs[i], **kw)
        else:
            f1, r1 = m.sgp_boundary_deconv(gs[i][None], ps[i][None], [bs[i]], w.domain, **kw)
        print(f"item {i} {tuple(gs[i].shape)} domain {w.domain}: iters {reps[i]['iters']}", flush=True)
        assert r1["iters"] == reps[i]["iters"] == 20, (i, r1["iters"], reps[i]["iters"])
        assert torch.equal(f1, fs[i]), i
        assert r1["kl"] == reps[i]["kl"], i


@pytest.mark.parametrize("alpha0", [1e2, 1e5])
def test_batch_equals_single_with_many_backtracks(torch_dev, alpha0):
    """A large first steplength sends every item's line search past the first
    two candidates into the Armijo kernel's candidate pass (and at 1e5 past
    theta^9 into its second stage); the pass takes the same workgroups per
    item in a batch as in a single run, so the batch still equals the single
    runs bit for bit."""
    import paper_1210_2258_amd as m
    torch = torch_dev
    items = _items()[:5]
    gs = [_dev(torch, w.g[0]) for w in items]
    ps = [_dev(torch, w.psf[0]) for w in items]
    bs = [float(w.b[0]) for w in items]
    kw = dict(max_iter=6, alpha0=alpha0)
    fs, reps = m.batch_deconv(gs, ps, bs, **kw)
    assert sum(r["backtracks"] for r in reps) >= 2 * len(items)
    for i in range(len(items)):
        f1, r1 = m.sgp_deconv(gs[i], ps[i], bs[i], **kw)
        assert r1["backtracks"] == reps[i]["backtracks"], i
        assert torch.equal(f1, fs[i]), i
        assert r1["kl"] == reps[i]["kl"], i
