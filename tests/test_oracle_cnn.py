"""Pins of the warm-start network oracle: direct-sum convolution, finite
differences of the loss, bf16 rounding of known values, Adam's first step."""
import numpy as np

from oracle import cnn as C


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(0)
    inp = rng.normal(size=(2, 6, 7))
    w = rng.normal(size=(3, 2, 5, 5))
    b = rng.normal(size=3)
    assert np.allclose(C.conv(inp, w, b), C.conv_direct(inp, w, b), atol=1e-12)


def test_conv_backward_is_adjoint():
    rng = np.random.default_rng(1)
    inp = rng.normal(size=(3, 8, 6))
    w = rng.normal(size=(2, 3, 5, 5))
    dout = rng.normal(size=(2, 8, 6))
    din, dw, db = C.conv_bwd(inp, w, dout)
    # <conv(inp) - bias, dout> is bilinear: its derivatives are the backward outputs
    base = np.sum((C.conv(inp, w, np.zeros(2))) * dout)
    assert np.isclose(np.sum(din * inp), base)
    assert np.isclose(np.sum(dw * w), base)
    assert np.allclose(db, dout.sum(axis=(1, 2)))


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(2)
    theta = C.init_params(3).astype(np.float64) * 0.5
    g = rng.poisson(20, (8, 8)).astype(float)
    tgt = rng.uniform(0, 30, (8, 8))
    L, grad = C.loss_and_grad(theta, [g], [3.0], [tgt], bf16=False)
    idx = rng.choice(theta.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        lp, _ = C.loss_and_grad(theta + e, [g], [3.0], [tgt], bf16=False)
        lm, _ = C.loss_and_grad(theta - e, [g], [3.0], [tgt], bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(grad[i])) + 1e-10, (i, fd, grad[i])


def test_bf16_rounding_known_values():
    one = np.float32(1.0)
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 2 ** -7 + 2 ** -8, 1 + 2 ** -7 + 2 ** -9, -3.0], dtype=np.float32)
    exp = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -3.0], dtype=np.float32)
    assert np.array_equal(C.bf16_round(vals), exp)
    assert C.bf16_round(one) == one


def test_adam_first_step_is_signed_lr():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = C.adam(theta, np.zeros(3), np.zeros(3), g, 1, 0.01)
    assert np.allclose(t1, theta - 0.01 * np.sign(g), atol=1e-7)


def test_forward_is_periodic_translation_equivariant():
    rng = np.random.default_rng(4)
    theta = C.init_params(5)
    g = rng.poisson(30, (16, 16)).astype(float)
    f0, _ = C.forward(theta, g, 5.0)
    f1, _ = C.forward(theta, np.roll(g, (3, -5), axis=(0, 1)), 5.0)
    assert np.allclose(np.roll(f0, (3, -5), axis=(0, 1)), f1)
