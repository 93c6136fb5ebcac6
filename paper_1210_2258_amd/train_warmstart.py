"""Trains the warm-start network on the GPU with the library's own kernels.

Training pairs are seeded 128x128 star fields drawn like the heterogeneous
star-field batches the warm start serves (Gaussian PSF with sigma in [1, 4],
constant background in [5, 50], 100 stars on a square image whose side is
drawn from 128, 256, 512, 1024, here at the same star density on a 128x128
cut-out), and as targets the SGP reconstructions the library itself computes
for them from the flat start, stopped by the discrepancy rule.  Training
runs sgp_cnn_train_step (forward, backward and Adam kernels) on minibatches.

    python -m paper_1210_2258_amd.train_warmstart [--pairs 20000] [--epochs 40]
        [--batch 32] [--lr 1.5e-3] [--out paper_1210_2258_amd/warmstart_weights.npy]

Writes the float32 parameter vector (.npy) and a JSON record of the run
beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAIN_CFG = 40          # generator stream of the training pairs
SIDE = 128
SIZES = (128, 256, 512, 1024)


def training_image(i):
    """(g, psf, b) of training pair i (seeded, independent of every other)."""
    from synth import workloads as W
    r = W.rng_for(TRAIN_CFG, i, "size")
    sz = int(SIZES[r.integers(0, len(SIZES))])
    sigma = float(r.uniform(1.0, 4.0))
    b = float(r.uniform(5.0, 50.0))
    nstars = int(r.poisson(100.0 * (SIDE / sz) ** 2))
    w = W.star_field(TRAIN_CFG, i, SIDE, SIDE, max(nstars, 0), sigma, b)
    return w.g[0].astype(np.float32), w.psf[0].astype(np.float32), b


def _chunk(lo_hi):
    lo, hi = lo_hi
    out = [training_image(i) for i in range(lo, hi)]
    return (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]),
            np.array([o[2] for o in out], np.float32))


def make_inputs(n, workers):
    step = 256
    parts = [(lo, min(lo + step, n)) for lo in range(0, n, step)]
    import multiprocessing as mp
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_chunk, parts))
    return (np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res]),
            np.concatenate([r[2] for r in res]))


def make_targets(torch, m, g, psf, b, chunk, max_iter):
    """SGP from the flat start to the discrepancy stop, batched."""
    n = g.shape[0]
    tgt = torch.empty_like(g)
    iters = np.zeros(n, np.int32)
    reached = np.zeros(n, bool)
    for lo in range(0, n, chunk):
        hi = min(lo + chunk, n)
        fs = [tgt[i] for i in range(lo, hi)]
        _, reps = m.batch_deconv([g[i] for i in range(lo, hi)], [psf[i] for i in range(lo, hi)],
                                 [float(v) for v in b[lo:hi]], fs=fs, max_iter=max_iter,
                                 stop=m.STOP_DISCREPANCY)
        for j, r in enumerate(reps):
            iters[lo + j] = r["iters"]
            reached[lo + j] = r["reason"] == "discrepancy"
        print(f"targets {hi}/{n}: mean iterations {iters[lo:hi].mean():.1f}", flush=True)
    return tgt, iters, reached


def train(net, g, b, tgt, idx_train, idx_val, epochs, batch, lr0, lr_min, seed):
    rng = np.random.default_rng(seed)
    steps_per_epoch = len(idx_train) // batch
    total = steps_per_epoch * epochs
    hist = []
    step = 0
    for ep in range(epochs):
        perm = rng.permutation(idx_train)
        t0 = time.perf_counter()
        acc = 0.0
        for s in range(steps_per_epoch):
            sel = perm[s * batch:(s + 1) * batch]
            lr = lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * step / max(total - 1, 1)))
            acc += net.train_step([g[i] for i in sel], [float(b[i]) for i in sel], [tgt[i] for i in sel], lr)
            step += 1
        val = 0.0
        nvb = 0
        for s in range(0, len(idx_val), batch):
            sel = idx_val[s:s + batch]
            loss, _ = net.loss_grad([g[i] for i in sel], [float(b[i]) for i in sel], [tgt[i] for i in sel])
            val += loss * len(sel)
            nvb += len(sel)
        rec = {"epoch": ep + 1, "train_loss": acc / steps_per_epoch, "val_loss": val / max(nvb, 1),
               "seconds": time.perf_counter() - t0}
        hist.append(rec)
        print(json.dumps(rec), flush=True)
    return hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1.5e-3)
    ap.add_argument("--lr-min", type=float, default=5e-5)
    ap.add_argument("--val-frac", type=float, default=0.05)
    ap.add_argument("--max-iter", type=int, default=1500)
    ap.add_argument("--chunk", type=int, default=2048)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "warmstart_weights.npy"))
    a = ap.parse_args(argv)
    # inputs first: the worker processes fork before anything touches the GPU
    t0 = time.perf_counter()
    g_h, psf_h, b_h = make_inputs(a.pairs, a.workers)
    t_gen = time.perf_counter() - t0
    print(f"generated {a.pairs} inputs in {t_gen:.1f} s", flush=True)
    import torch

    import paper_1210_2258_amd as m
    from paper_1210_2258_amd.warmstart import initial_params
    if not torch.cuda.is_available():
        raise SystemExit("training needs a GPU")
    m.load()
    g = torch.from_numpy(g_h).cuda()
    psf = torch.from_numpy(psf_h).cuda()
    del psf_h
    t1 = time.perf_counter()
    tgt, iters, reached = make_targets(torch, m, g, psf, b_h, a.chunk, a.max_iter)
    torch.cuda.synchronize()
    t_sgp = time.perf_counter() - t1
    del psf
    keep = np.flatnonzero(reached)
    rng = np.random.default_rng(a.seed)
    keep = rng.permutation(keep)
    nval = int(len(keep) * a.val_frac)
    idx_val, idx_train = np.sort(keep[:nval]), keep[nval:]
    net = m.CnnNet(initial_params(a.seed))
    t2 = time.perf_counter()
    hist = train(net, g, b_h, tgt, idx_train, idx_val, a.epochs, a.batch, a.lr, a.lr_min, a.seed)
    t_train = time.perf_counter() - t2
    theta = net.params()
    net.close()
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.save(a.out, theta)
    rec = {"pairs": a.pairs, "pairs_reaching_discrepancy": int(reached.sum()),
           "train_pairs": int(len(idx_train)), "val_pairs": int(len(idx_val)),
           "sgp_iterations_mean": float(iters.mean()), "sgp_iterations_max": int(iters.max()),
           "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "lr_min": a.lr_min, "seed": a.seed,
           "generate_s": t_gen, "targets_s": t_sgp, "train_s": t_train, "history": hist,
           "command": "python -m paper_1210_2258_amd.train_warmstart " + " ".join(argv or sys.argv[1:])}
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k != "history"}), flush=True)


if __name__ == "__main__":
    main()
