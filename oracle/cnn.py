"""Plain float64 CPU oracle of the warm-start network (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by tests/ and bench.py's cpu leg; shares
no code with the HIP kernels.

The network maps an observed image g (background b) to a start image f0 for
SGP (Sect. 3.1 of the paper admits any caller-supplied positive start; the
network itself is not part of the paper):

    s  = max(mean(g - b), 1e-3)                  per-image scale
    x  = (g - b) / s
    a1 = relu(conv(x;  W1, b1))      1 -> 16 channels
    a2 = relu(conv(a1; W2, b2))     16 -> 16
    a3 = relu(conv(a2; W3, b3))     16 -> 16
    o  = conv(a3; W4, b4)           16 -> 1
    y  = softplus(o),   f0 = s * y

conv is a 5x5 cross-correlation with periodic padding,
    out[co](y, x) = bias[co] + sum_{ci,ky,kx} W[co, ci, ky, kx] in[ci]((y+ky-2) mod H, (x+kx-2) mod W),
and every convolution weight (not the biases) is rounded to bfloat16 (round
to nearest even) before use.  For inference the hidden activations a1..a3
are also stored as bfloat16 (forward(..., act_bf16=True)); training keeps
them in float32.
The training loss on a batch is the mean over pixels of
(sqrt(y + eps) - sqrt(t + eps))^2 with t = f_target / s, eps = 1e-3.
Adam (beta1 0.9, beta2 0.999, eps 1e-8) updates float32 master weights.
"""
from __future__ import annotations

import numpy as np

SHAPES = [(16, 1), (16, 16), (16, 16), (1, 16)]  # (cout, cin) of the four layers
K = 5
EPS_LOSS = 1e-3


def n_params():
    return sum(co * ci * K * K + co for co, ci in SHAPES)


def unpack(theta):
    """Flat parameter vector -> [(W, bias)] (layout: W1, b1, W2, b2, ...)."""
    out, o = [], 0
    for co, ci in SHAPES:
        w = theta[o:o + co * ci * K * K].reshape(co, ci, K, K)
        o += co * ci * K * K
        b = theta[o:o + co]
        o += co
        out.append((w, b))
    return out


def bf16_round(a):
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def init_params(seed=0):
    """He-style seeded initialisation of the float32 master weights."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (co, ci) in enumerate(SHAPES):
        std = np.sqrt(2.0 / (ci * K * K))
        w = rng.normal(0.0, std, (co, ci, K, K))
        b = np.zeros(co) if li < 3 else np.full(co, 0.0)
        parts += [w.ravel(), b]
    return np.concatenate(parts).astype(np.float32)


def conv(inp, w, b):
    """inp [C, H, W], w [CO, C, 5, 5] -> [CO, H, W] (periodic 5x5 correlation)."""
    C, H, W = inp.shape
    out = np.zeros((w.shape[0], H, W))
    for ky in range(K):
        for kx in range(K):
            sh = np.roll(np.roll(inp, -(ky - 2), axis=1), -(kx - 2), axis=2)  # in(y+ky-2, x+kx-2)
            out += np.einsum("oc,chw->ohw", w[:, :, ky, kx], sh)
    return out + b[:, None, None]


def conv_direct(inp, w, b):
    """Direct definition of conv (tests only)."""
    C, H, W = inp.shape
    CO = w.shape[0]
    out = np.zeros((CO, H, W))
    for co in range(CO):
        for y in range(H):
            for x in range(W):
                s = b[co]
                for ci in range(C):
                    for ky in range(K):
                        for kx in range(K):
                            s += w[co, ci, ky, kx] * inp[ci, (y + ky - 2) % H, (x + kx - 2) % W]
                out[co, y, x] = s
    return out


def conv_bwd(inp, w, dout):
    """Gradients of conv: (d inp, d w, d b) given d out."""
    C, H, W = inp.shape
    dw = np.zeros_like(w, dtype=np.float64)
    din = np.zeros((C, H, W))
    for ky in range(K):
        for kx in range(K):
            sh = np.roll(np.roll(inp, -(ky - 2), axis=1), -(kx - 2), axis=2)
            dw[:, :, ky, kx] = np.einsum("ohw,chw->oc", dout, sh)
            t = np.einsum("oc,ohw->chw", w[:, :, ky, kx], dout)
            din += np.roll(np.roll(t, ky - 2, axis=1), kx - 2, axis=2)
    return din, dw, dout.sum(axis=(1, 2))


def softplus(o):
    return np.where(o > 20, o, np.log1p(np.exp(np.minimum(o, 20))))


def sigmoid(o):
    return 1.0 / (1.0 + np.exp(-o))


def scale_of(g, b):
    return max(float(np.mean(np.asarray(g, np.float64) - b)), 1e-3)


def forward(theta, g, b, bf16=True, act_bf16=False):
    """Returns (f0, cache) for one image.  bf16=False skips the weight
    rounding (only for finite-difference checks of the gradient formula).
    act_bf16=True also stores the three hidden activations as bfloat16, as
    the inference path does: each one, after its ReLU, is rounded to float32
    and then to the nearest bfloat16 (ties to even); the output layer is not
    rounded."""
    rnd = bf16_round if bf16 else (lambda a: a)
    layers = [(rnd(w).astype(np.float64), bb.astype(np.float64)) for w, bb in unpack(theta)]
    s = scale_of(g, b)
    x = ((np.asarray(g, np.float64) - b) / s)[None]
    acts = [x]
    h = x
    for li, (w, bb) in enumerate(layers):
        pre = conv(h, w, bb)
        h = np.maximum(pre, 0.0) if li < 3 else pre
        if act_bf16 and li < 3:
            h = bf16_round(h.astype(np.float32)).astype(np.float64)
        acts.append(h)
    o = acts[-1][0]
    y = softplus(o)
    return s * y, dict(s=s, acts=acts, o=o, y=y, layers=layers)


def loss_and_grad(theta, gs, bs, targets, bf16=True):
    """Mean loss over a batch and its gradient w.r.t. the (bf16-rounded)
    weights, returned as a flat float64 vector in the parameter layout."""
    tot_px = sum(np.asarray(g).size for g in gs)
    loss = 0.0
    grads = [(np.zeros(w.shape), np.zeros(bb.shape)) for w, bb in unpack(theta)]
    for g, b, tgt in zip(gs, bs, targets):
        f0, c = forward(theta, g, b, bf16)
        s, y, o = c["s"], c["y"], c["o"]
        t = np.asarray(tgt, np.float64) / s
        r = np.sqrt(y + EPS_LOSS) - np.sqrt(t + EPS_LOSS)
        loss += float(np.sum(r * r))
        dy = r / np.sqrt(y + EPS_LOSS) / tot_px
        d = (dy * sigmoid(o))[None]
        for li in range(3, -1, -1):
            w, bb = c["layers"][li]
            din, dw, db = conv_bwd(c["acts"][li], w, d)
            grads[li][0][...] += dw
            grads[li][1][...] += db
            if li > 0:
                d = din * (c["acts"][li] > 0)
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return loss / tot_px, flat


def adam(theta, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v) in float64."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
