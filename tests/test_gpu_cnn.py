"""Warm-start network kernels against the FP64 oracle (oracle/cnn.py): start
images, batch loss and weight gradients, Adam steps, determinism, argument
checks, and a loss that falls under training on the GPU."""
import numpy as np
import pytest

from oracle import cnn as OC
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


def _params(seed):
    """Seeded weights with non-zero biases, so every ReLU sees both signs."""
    theta = OC.init_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    o = 0
    for co, ci in OC.SHAPES:
        o += co * ci * OC.K * OC.K
        theta[o:o + co] = rng.normal(0.0, 0.2, co)
        o += co
    return theta.astype(np.float32)


def _batch(n, ny, nx, seed):
    items = [W.star_field(300, seed * 16 + i, ny, nx, 12, 1.5 + 0.5 * i, 8.0 + 4.0 * i) for i in range(n)]
    gs = [w.g[0].astype(np.float32) for w in items]
    bs = [float(w.b[0]) for w in items]
    ts = [w.f_true.astype(np.float32) for w in items]
    return gs, bs, ts


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("shape", [(48, 80), (16, 16), (128, 64)])
def test_forward_matches_oracle(torch_dev, shape):
    from paper_1210_2258_amd import CnnNet
    torch = torch_dev
    theta = _params(1)
    gs, bs, _ = _batch(3, *shape, seed=1)
    net = CnnNet(theta)
    f0 = net.infer([_dev(torch, g) for g in gs], bs)
    for i in range(3):
        # inference stores the hidden activations as bfloat16: the oracle
        # rounds them the same way.  Where the FP32 pre-activation and the
        # oracle's FP64 one fall on opposite sides of a bfloat16 rounding
        # point the two activations differ by one bfloat16 step (2^-8
        # relative), which moves the output pixels around it.  Perturbing
        # the oracle's pre-activations by relative 1e-7 (the size of FP32
        # accumulation error) moves these nine outputs by up to 5.8e-5 in
        # relative L2 (3e-7: up to 9e-4), so the bar is 2e-4; and the flips
        # are local: at most 1% of the pixels may differ by more than 1e-4.
        ref, _ = OC.forward(theta, gs[i], bs[i], act_bf16=True)
        got = f0[i].cpu().numpy()
        assert got.shape == ref.shape
        err = _rel(got, ref)
        far = float(np.mean(np.abs(got - ref) > 1e-4 * np.abs(ref).max()))
        print(f"network start {shape} image {i}: rel L2 {err:.1e}, pixels off by > 1e-4: {far:.2%}", flush=True)
        assert err <= 2e-4, (i, err)
        assert far <= 0.01, (i, far)
        assert np.all(got >= 0)
    net.close()


def test_loss_and_gradient_match_oracle(torch_dev):
    from paper_1210_2258_amd import CnnNet
    torch = torch_dev
    theta = _params(2)
    gs, bs, ts = _batch(3, 48, 80, seed=2)
    net = CnnNet(theta)
    loss, grad = net.loss_grad([_dev(torch, g) for g in gs], bs, [_dev(torch, t) for t in ts])
    ref_loss, ref_grad = OC.loss_and_grad(theta, gs, bs, ts)
    assert abs(loss - ref_loss) <= 1e-6 * ref_loss, (loss, ref_loss)
    assert _rel(grad, ref_grad) <= 1e-4, _rel(grad, ref_grad)
    # every layer's weights and biases separately
    o = 0
    for co, ci in OC.SHAPES:
        nw = co * ci * OC.K * OC.K
        assert _rel(grad[o:o + nw], ref_grad[o:o + nw]) <= 1e-4
        assert _rel(grad[o + nw:o + nw + co], ref_grad[o + nw:o + nw + co]) <= 1e-4
        o += nw + co
    net.close()


def test_gradient_is_deterministic(torch_dev):
    from paper_1210_2258_amd import CnnNet
    torch = torch_dev
    gs, bs, ts = _batch(2, 64, 64, seed=3)
    g_d, t_d = [_dev(torch, g) for g in gs], [_dev(torch, t) for t in ts]
    net = CnnNet(_params(3))
    l1, g1 = net.loss_grad(g_d, bs, t_d)
    l2, g2 = net.loss_grad(g_d, bs, t_d)
    assert l1 == l2 and np.array_equal(g1, g2)
    net.close()


def test_adam_steps_match_oracle(torch_dev):
    """Two Adam steps on one batch.  Where the gradient component is well
    away from zero the update is a smooth function of the gradients and must
    agree closely; near-zero components may differ by the sign of noise."""
    from paper_1210_2258_amd import CnnNet
    torch = torch_dev
    theta = _params(4)
    gs, bs, ts = _batch(2, 48, 48, seed=4)
    g_d, t_d = [_dev(torch, g) for g in gs], [_dev(torch, t) for t in ts]
    lr = 1e-3
    net = CnnNet(theta)
    for _ in range(2):
        net.train_step(g_d, bs, t_d, lr)
    got = net.params().astype(np.float64)
    net.close()

    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    small = np.zeros(th.size, bool)
    for t in (1, 2):
        _, gr = OC.loss_and_grad(th.astype(np.float32), gs, bs, ts)
        small |= np.abs(gr) < 1e-3 * np.sqrt(np.mean(gr * gr))
        th, m, v = OC.adam(th, m, v, gr, t, lr)
    err = np.abs(got - th)
    assert small.mean() < 0.1
    assert np.all(err[~small] <= 1e-6 * np.abs(th[~small]) + 1e-2 * lr), err[~small].max()
    assert np.all(err <= 4 * lr + 1e-6 * np.abs(th))


def test_training_lowers_the_loss(torch_dev):
    from paper_1210_2258_amd import CnnNet
    torch = torch_dev
    gs, bs, ts = _batch(4, 64, 64, seed=5)
    g_d, t_d = [_dev(torch, g) for g in gs], [_dev(torch, t) for t in ts]
    net = CnnNet(OC.init_params(5))
    first = net.train_step(g_d, bs, t_d, 3e-3)
    for _ in range(40):
        last = net.train_step(g_d, bs, t_d, 3e-3)
    net.close()
    assert np.isfinite(last) and last < 0.7 * first, (first, last)


def test_rejects_bad_arguments(torch_dev):
    import paper_1210_2258_amd as m
    torch = torch_dev
    with pytest.raises(ValueError):
        m.CnnNet(np.zeros(10, np.float32))
    net = m.CnnNet(_params(6))
    g = torch.ones((40, 48), device="cuda")
    with pytest.raises(m.SgpError) as e:
        net.infer([g], [1.0])
    assert e.value.code == -1
    with pytest.raises(ValueError):
        net.infer([g, torch.ones((48, 48), device="cuda")], [1.0, 1.0])
    net.close()
