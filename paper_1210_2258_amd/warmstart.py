"""Learned warm start for SGP: network start images and the batched solve
that uses them.

The network (include/sgpcnn.h) predicts a start image from the observed
image; SGP accepts any non-negative start (Sect. 3.1 of the paper) and the
solver keeps the flat start whenever the predicted one has the larger KL
divergence (SGP_INIT_WARM).  Weights trained by ``train_warmstart`` ship
next to this module as ``warmstart_weights.npy``.
"""
from __future__ import annotations

import os
from collections import defaultdict

import numpy as np

from ._lib import INIT_WARM, KIND_SGP, CnnNet, batch_deconv

WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_weights.npy")


LAYERS = ((16, 1), (16, 16), (16, 16), (1, 16))   # (output, input) channels; 5x5 kernels


def initial_params(seed: int = 0) -> np.ndarray:
    """Seeded starting weights for training: He-normal weights (std
    sqrt(2 / fan-in)), zero biases, in the layout of include/sgpcnn.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci in LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (ci * 25)), co * ci * 25))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def load_net(path: str | None = None) -> CnnNet:
    """Network with the shipped (or given) weights; raises if they are missing."""
    path = path or WEIGHTS_PATH
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: train it with paper_1210_2258_amd.train_warmstart")
    return CnnNet(np.load(path, allow_pickle=False))


def infer_many(net: CnnNet, gs, bs, stream=None):
    """Start images for images of any shapes (one network call per shape)."""
    groups = defaultdict(list)
    for i, g in enumerate(gs):
        groups[tuple(g.shape)].append(i)
    out = [None] * len(gs)
    # largest group first: the network's work buffers are sized once
    for shape, idx in sorted(groups.items(), key=lambda kv: -kv[0][0] * kv[0][1] * len(kv[1])):
        f0 = net.infer([gs[i] for i in idx], [bs[i] for i in idx], stream=stream)
        for i, t in zip(idx, f0):
            out[i] = t
    return out


def warm_batch_deconv(net: CnnNet, gs, psfs, bs, *, stream=None, **params):
    """Network starts for every image, then one batched SGP run that starts
    each problem from the better (in KL) of its network start and the flat
    image.  Returns (list of f, list of reports)."""
    f0s = infer_many(net, gs, bs, stream=stream)
    params.setdefault("init", INIT_WARM)
    return batch_deconv(gs, psfs, bs, kind=KIND_SGP, f0s=f0s, stream=stream, **params)
