"""Pins of the warm-start network oracle: direct-sum convolution, finite
differences of the loss, bf16 rounding of known values, Adam's first step."""
import numpy as np
import pytest

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


def _single_tap_params(bias1):
    """Layer 1 passes x through its centre tap (weight 1) plus bias1 on every
    channel; layers 2-4 keep only the centre tap of input channel 0 (weight
    1, bias 0)."""
    theta = np.zeros(C.n_params(), np.float32)
    o = 0
    for li, (co, ci) in enumerate(C.SHAPES):
        w = np.zeros((co, ci, C.K, C.K), np.float32)
        w[:, 0, 2, 2] = 1.0
        theta[o:o + w.size] = w.ravel()
        o += w.size
        theta[o:o + co] = bias1 if li == 0 else 0.0
        o += co
    return theta


@pytest.mark.parametrize("bias1,expect", [(2.0 ** -8, 1.0), (3 * 2.0 ** -8, 1.0 + 2.0 ** -6),
                                          (2.0 ** -9, 1.0), (5 * 2.0 ** -9, 1.0 + 2.0 ** -7)])
def test_bf16_activation_rounding_known_values(bias1, expect):
    """A constant image gives x = 1 and a first-layer pre-activation of
    1 + bias1: 1 + 2^-8 and 1 + 3 2^-8 are ties (bfloat16 spacing 2^-7 at 1)
    and go to the even neighbour, 1 + 2^-9 rounds down and 1 + 5 2^-9 up.
    The later layers pass the rounded value on unchanged (it is already a
    bfloat16 value), and the output layer is not rounded."""
    g = np.full((16, 16), 7.0)
    f0, c = C.forward(_single_tap_params(bias1), g, 0.0, act_bf16=True)
    for a in c["acts"][1:4]:
        assert np.all(a[0] == expect)
    f_plain, c2 = C.forward(_single_tap_params(bias1), g, 0.0)
    assert np.all(c2["acts"][1][0] == 1.0 + bias1)
    assert np.all(c["o"] == expect)                 # o = a3 through the centre tap


def test_bf16_activations_are_bfloat16_values():
    rng = np.random.default_rng(4)
    theta = C.init_params(2)
    g = rng.poisson(30.0, (32, 48)).astype(np.float64)
    _, c = C.forward(theta, g, 5.0, act_bf16=True)
    for a in c["acts"][1:4]:
        assert np.array_equal(C.bf16_round(a.astype(np.float32)).astype(np.float64), a)
    o = c["o"].astype(np.float32)
    assert not np.array_equal(C.bf16_round(o), o)   # the output layer keeps full precision
