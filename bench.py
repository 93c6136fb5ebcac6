"""Benchmark: SGP iterations per second on the 2048x2048 galaxy workload.

One "step" is one SGP iteration (scaling, projection, direction, forward
convolution, Armijo test, update, adjoint convolution, gradient and BB
steplength) over the whole image, through the stepping C ABI with the
iteration loop replayed as a HIP graph.  Inputs are resident in HBM before
the timed region starts.  Also reported: the time to reach the discrepancy
stop (call to return, setup included), the roofline of the dominant kernel
(from HIP events on the solver's stream), and the FP64 oracle timed on the
host's cores on a bounded sample.

The heterogeneous batch (512 star fields of 128..1024 pixels a side) is
deconvolved three ways with one stop rule (discrepancy, relative KL change
as a backstop): one image at a time from the flat start (plain SGP), in one
batched run from the flat start, and in one batched run from the learned
warm start (network inference included in its time).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SGP iter/s & time-to-discrepancy at 2048² FP32; warm-start+batch vs plain"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per pixel and launch (FP32 fields, complex64 half spectra,
# one HBM pass per 2D-FFT transpose), single image with a constant background:
#   row_dir  reads f, grad            writes spectrum              12 B/px
#   col_conv reads spectrum, K         writes spectrum              12 B/px
#   row_ad   reads spectrum, Af, g     writes Ad, Af', spectrum     24 B/px
#   col_corr reads spectrum, K         writes spectrum              12 B/px
#   row_grad reads spectrum, grad, f   writes grad, f               20 B/px
# (the A d pass also makes the update for lambda = 1; the update pass,
#   row_upd  reads Af, Ad, g           writes Af', spectrum         20 B/px
# runs only when another lambda is accepted; the gradient pass takes
# f + lam d, evaluating d again from f and grad)
BYTES_PER_PX = {"row_dir": 12, "col_conv": 12, "row_ad": 24, "row_upd": 20, "col_corr": 12,
                "row_grad": 20}
ITER_BYTES_PER_PX = sum(v for k, v in BYTES_PER_PX.items() if k != "row_upd")  # 80


def iter_bytes(p, NY, NX, ny, nx, boundary):
    """Algorithmic bytes of one SGP iteration in the usual case (lambda = 1
    accepted) for p images observed on ny x nx inside the NY x NX FFT domain:
    per FFT-domain pixel the direction pass reads f, grad (+ the weights
    M_R / alpha of a boundary problem) and writes one spectrum; the forward
    column pass reads that spectrum once and K_j, writes p spectra; the A d
    pass reads spectrum j, and on S A_j f and g_j, writes on S A_j d and the
    new A_j f, and spectrum j; the adjoint column pass reads p spectra and K_j,
    writes one; the gradient pass reads the spectrum, grad, f (+ weights),
    writes grad and f."""
    F, Sx = NY * NX, ny * nx
    w = 4 if boundary else 0
    row_dir = (8 + w + 4) * F
    col_conv = (4 + 8 * p) * F
    row_ad = p * (8 * F + 16 * Sx)
    col_corr = (4 + 8 * p) * F
    row_grad = (16 + w + 4) * F
    return row_dir + col_conv + row_ad + col_corr + row_grad


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--cpu-iters", type=int, default=8)
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--no-batch", action="store_true", help="skip the heterogeneous batch legs")
    ap.add_argument("--no-ttd", action="store_true", help="skip the time-to-discrepancy runs")
    ap.add_argument("--batch-images", type=int, default=512)
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-image RL / OSEM / SGP comparison")
    ap.add_argument("--no-mosaic", action="store_true", help="skip the mosaic leg")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-iteration rates of the multi-image and boundary workloads")
    ap.add_argument("--no-mall", action="store_true", help="skip the 4 x 2048^2 batch beyond the Infinity Cache")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep tile variant 0 instead of timing the tile variants per FFT length")
    ap.add_argument("--tiles", type=int, nargs=2, metavar=("ROW", "COL"),
                    help="tile variants of the main image size, set instead of tuned (as in profiled runs)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the Fourier re-binning size sweep 256..2048 (RL and SGP, GPU and oracle)")
    return ap.parse_args()


def _c4_item(i):
    from synth import workloads as W
    w = W.config4(n_images=1, purpose_base=i)[0]
    return w.g[0], w.psf[0], float(w.b[0])


def make_batch_inputs(n):
    """The 512-image star-field batch, generated in worker processes that
    fork before anything touches the GPU."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4), mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_c4_item, range(n), chunksize=8))


def tune(m, g, psf, b, iters, record):
    """Autotuner of the FFT tile schedule on one problem of this size; the
    choice stays in the library's table for the runs that follow."""
    r, c, ms = m.autotune(g, psf, b, iters=iters)
    record["x".join(map(str, g.shape))] = {"rows_variant": r, "cols_variant": c,
                                           "ms_per_iter": {f"{k[0]}{k[1]}": v for k, v in ms.items()}}


def batch_legs(torch, m, items, tiles=None):
    """Plain (one image at a time, flat start), flat batch and warm batch,
    each timed from call to return with the inputs resident."""
    import numpy as np
    from paper_1210_2258_amd import warmstart as WS
    gs = [torch.from_numpy(g).cuda() for g, _, _ in items]
    ps = [torch.from_numpy(p).cuda() for _, p, _ in items]
    bs = [b for _, _, b in items]
    kw = dict(max_iter=3000, stop=m.STOP_DISCREPANCY | m.STOP_CONV, tol=1e-7)
    net = WS.load_net()
    seen = {}
    for i, g in enumerate(gs):
        seen.setdefault(tuple(g.shape), i)
    if tiles is not None:  # tile schedule of every size in the batch, before any timed leg
        for i in seen.values():
            tune(m, gs[i], ps[i], bs[i], 128, tiles)
    # warm-up: workspaces of every shape and group size, network buffers
    for i in seen.values():
        m.sgp_deconv(gs[i], ps[i], bs[i], max_iter=2)
    m.batch_deconv(gs, ps, bs, max_iter=1)
    WS.infer_many(net, gs, bs)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    plain = [m.sgp_deconv(gs[i], ps[i], bs[i], **kw)[1] for i in range(len(gs))]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, flat = m.batch_deconv(gs, ps, bs, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _, warm = WS.warm_batch_deconv(net, gs, ps, bs, **kw)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    WS.infer_many(net, gs, bs)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    net.close()

    def summary(reps, secs):
        it = np.array([r["iters"] for r in reps])
        return {"seconds": secs, "iterations": int(it.sum()), "max_iterations": int(it.max()),
                "reached_discrepancy": int(sum(r["reason"] == "discrepancy" for r in reps)),
                "stopped_by_kl_change": int(sum(r["reason"] == "convergence" for r in reps)),
                "mean_kl": float(np.mean([r["kl"] for r in reps])),
                "mean_discrepancy": float(np.mean([r["discrepancy"] for r in reps]))}
    out = {"images": len(gs), "pixels": int(sum(g.numel() for g in gs)),
           "stop": "discrepancy <= 1, else relative KL change <= 1e-7, else 3000 iterations",
           "plain": summary(plain, t1 - t0), "flat_batch": summary(flat, t2 - t1),
           "warm_batch": summary(warm, t3 - t2), "network_inference_s": t4 - t3,
           "warm_used_flat_fallback": int(sum(r["used_fallback"] for r in warm)),
           "kl_ratio_warm_over_plain": float(np.mean([w["kl"] / p["kl"] for w, p in zip(warm, plain)]))}
    out["speedup_warm_batch_vs_plain"] = out["plain"]["seconds"] / out["warm_batch"]["seconds"]
    out["speedup_warm_batch_vs_flat_batch"] = out["flat_batch"]["seconds"] / out["warm_batch"]["seconds"]
    return out


def time_to_discrepancy(torch, m, g, psf, b):
    """SGP and RL to the discrepancy stop, call to return, setup included."""
    f_out = torch.empty_like(g)
    m.sgp_deconv(g, psf, b, f=f_out, max_iter=10, stop=m.STOP_FIXED)  # warm the plan cache
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    f_out, drep = m.sgp_deconv(g, psf, b, f=f_out, max_iter=5000, stop=m.STOP_DISCREPANCY)
    torch.cuda.synchronize()
    ttd = time.perf_counter() - t2
    t3 = time.perf_counter()
    f_rl, rrep = m.rl_deconv(g, psf, b, max_iter=20000, stop=m.STOP_DISCREPANCY)
    torch.cuda.synchronize()
    ttd_rl = time.perf_counter() - t3
    return ({"time_to_discrepancy_s": ttd, "iters_to_discrepancy": drep["iters"],
             "discrepancy_final": drep["discrepancy"], "kl_final": drep["kl"],
             "rl_time_to_discrepancy_s": ttd_rl, "rl_iters_to_discrepancy": rrep["iters"]}, f_out)


def multi_image_legs(torch, m, w):
    """Multiple-image RL (Eq. multipleRL), its linear relaxation with the
    Armijo line search (Eq. RL2), OSEM (Algorithm 2) and SGP on the
    3 x 1024^2 interferometric workload, each to the discrepancy stop, call to
    return with the inputs resident (the comparison of the paper's Tables 5-8
    on synthetic data)."""
    g = torch.from_numpy(w.g).cuda()
    psf = torch.from_numpy(w.psf).cuda()
    out = {"workload": f"{w.g.shape[0]} x {w.g.shape[1]}x{w.g.shape[2]} fringe-PSF images of one object, b = 20",
           "stop": "discrepancy <= 1 (cap 20000 iterations)"}
    legs = (("rl", m.rl_multi_deconv, {}), ("rl_linear", m.rl_multi_deconv, {"rl_line_search": 1}),
            ("osem", m.osem_deconv, {}), ("sgp", m.sgp_multi_deconv, {}))
    for name, fn, kw in legs:
        fn(g, psf, w.b, max_iter=2, **kw)  # workspace of this shape and kind
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rep = fn(g, psf, w.b, max_iter=20000, stop=m.STOP_DISCREPANCY, **kw)
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "iterations": rep["iters"], "reason": rep["reason"],
                     "kl": rep["kl"], "discrepancy": rep["discrepancy"]}
    out["speedup_sgp_vs_rl"] = out["rl"]["seconds"] / out["sgp"]["seconds"]
    out["speedup_osem_vs_rl"] = out["rl"]["seconds"] / out["osem"]["seconds"]
    out["speedup_rl_linear_vs_rl"] = out["rl"]["seconds"] / out["rl_linear"]["seconds"]
    return out


def mosaic_leg(torch, m, w, g, psf, f_full, tiles=None):
    """The 2048^2 galaxy field as a mosaic of four 1024^2 cores seen through
    windows with 128-pixel margins on 1280^2 domains (one batch of boundary
    problems), SGP to the discrepancy stop of every window; compared with the
    full-image reconstruction f_full."""
    N, core, margin = 1280, 1024, 128
    c0 = (psf.shape[0] - N) // 2
    psf_N = psf[c0:c0 + N, c0:c0 + N].contiguous()
    if tiles is not None:  # tile schedule of the 1280 domain, on a corner window (core + one margin)
        win = core + margin
        gw = g[:win, :win].contiguous()
        r, c, ms = m.autotune(gw, psf_N, float(w.b[0]), domain=(N, N, (N - win) // 2, (N - win) // 2), iters=64)
        tiles[f"{N}x{N} boundary"] = {"rows_variant": r, "cols_variant": c,
                                      "ms_per_iter": {f"{k[0]}{k[1]}": v for k, v in ms.items()}}
    m.mosaic_deconv(g, psf_N, float(w.b[0]), core, margin, max_iter=2)  # workspaces
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f, rep = m.mosaic_deconv(g, psf_N, float(w.b[0]), core, margin, max_iter=5000, stop=m.STOP_DISCREPANCY)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    diff = float(torch.linalg.vector_norm(f - f_full) / torch.linalg.vector_norm(f_full))
    return {"tiles": 4, "core": core, "margin": margin, "fft_domain": N, "seconds": secs,
            "iterations_longest_tile": rep["iters"], "max_tile_discrepancy": rep["discrepancy"],
            "rel_l2_vs_full_image": diff}


def beyond_mall_leg(torch, m, g, psf, b, n=4, iters=40):
    """n copies of the 2048^2 problem in one batched run (about 130 MB of
    fields and spectra per image, so n = 4 exceeds the 256 MB Infinity Cache):
    per-iteration time from two fixed-count runs (their difference cancels
    the setup), as pixel throughput and as a fraction of the HBM roofline at
    80 B/px."""
    gs, ps, bs = [g] * n, [psf] * n, [b] * n
    fs = [torch.empty_like(g) for _ in range(n)]
    m.batch_deconv(gs, ps, bs, fs=fs, max_iter=2)  # workspaces
    t = []
    for k in (iters, 2 * iters):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, reps = m.batch_deconv(gs, ps, bs, fs=fs, max_iter=k, stop=m.STOP_FIXED)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
        assert all(r["iters"] == k for r in reps)
    per_iter = (t[1] - t[0]) / iters
    npx = n * g.numel()
    gbs = ITER_BYTES_PER_PX * npx / per_iter / 1e9
    return {"images": n, "image": list(g.shape), "ms_per_iteration": 1e3 * per_iter,
            "ms_per_image_iteration": 1e3 * per_iter / n, "pixel_iterations_per_s": npx / per_iter,
            "iteration_GBs_at_80_B_per_px": gbs, "frac": gbs / HBM_PEAK_GBS}


def rebin_sweep(torch, m, with_oracle):
    """Sizes 256..2048 made by Fourier re-binning of the 256^2 galaxy field;
    RL and SGP run at every size for the iteration counts the discrepancy rule
    gives at 256^2 (the procedure of the paper's third experiment).  Reports
    GPU seconds per run (call to return, setup included), the SGP-over-RL
    speedup ("Alg") and, with the oracle, its seconds per run on one host core
    extrapolated from two timed iterations ("Par" = oracle / GPU)."""
    from synth import workloads as W
    series = W.rebin_series(W.rebin_base(size=256, total=1e6))
    out = {"object": "galaxy field drawn at 256^2 (1e6 counts, Airy PSF with first zero at 4 px, b = 50), "
                     "re-binned by 2x steps to 2048^2", "sizes": {}}
    counts = {}
    for n, g_h, psf_h in series:
        g = torch.from_numpy(g_h).cuda()
        psf = torch.from_numpy(psf_h).cuda()
        row = {}
        for name, fn in (("rl", m.rl_deconv), ("sgp", m.sgp_deconv)):
            if name not in counts:  # fixed from the 256^2 case by the discrepancy rule
                _, r = fn(g, psf, 50.0, max_iter=20000, stop=m.STOP_DISCREPANCY)
                counts[name] = max(r["iters"], 1)
            fn(g, psf, 50.0, max_iter=2)  # workspace of this size
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r = fn(g, psf, 50.0, max_iter=counts[name])
            torch.cuda.synchronize()
            row[name] = {"iterations": counts[name], "gpu_seconds": time.perf_counter() - t0, "kl": r["kl"]}
        row["alg_speedup_sgp_vs_rl"] = row["rl"]["gpu_seconds"] / row["sgp"]["gpu_seconds"]
        if with_oracle:
            from oracle import sgp as O
            P = O.Problem(g_h, psf_h, 50.0)
            f0 = P.start("flat")
            for name in ("rl", "sgp"):
                t0 = time.perf_counter()
                if name == "rl":
                    P.rl(f0, 0)
                else:
                    P.sgp(f0, O.Params(max_iter=0))
                t1 = time.perf_counter()
                if name == "rl":
                    P.rl(f0, 2)
                else:
                    P.sgp(f0, O.Params(max_iter=2))
                t2 = time.perf_counter()
                per_it = max((t2 - t1) - (t1 - t0), 1e-9) / 2
                est = (t1 - t0) + per_it * counts[name]
                row[name]["oracle_seconds_estimated"] = est
                row[name]["par_speedup"] = est / row[name]["gpu_seconds"]
        out["sizes"][str(n)] = row
    return out


COUNTER_FILE = os.path.join(ROOT, "profiles", "sgp_2048_hbm_counters.md")
KERNEL_SOURCES = ("common.hpp", "fft.hpp", "reduce.hpp", "finalize.hpp", "kernels.hpp", "pix.hpp",
                  "inst.hip", "dispatch.hip")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1210_2258_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, npx):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None when the
    kernel sources changed since the counters were taken."""
    try:
        txt = open(COUNTER_FILE).read()
        rec = json.loads(txt.split("```json")[1].split("```")[0])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("pixels") != npx:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes"]


def oracle_rate(w, iters, workers=None):
    """The FP64 oracle on the host: (setup seconds, seconds per SGP iteration)
    from runs with 0 and `iters` iterations (setup cancels).  workers: None
    runs numpy.fft (one thread), n runs the same transforms through scipy.fft
    with n threads (the elementwise work stays on one thread)."""
    from oracle import sgp as O
    O.FFT_WORKERS = workers
    try:
        P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
        f0 = P.start("flat")
        t0 = time.perf_counter()
        P.sgp(f0, O.Params(max_iter=0))
        t1 = time.perf_counter()
        P.sgp(f0, O.Params(max_iter=iters))
        t2 = time.perf_counter()
    finally:
        O.FFT_WORKERS = None
    return t1 - t0, max((t2 - t1) - (t1 - t0), 1e-9) / iters


def cpu_baseline(w, iters, gpu_iters_to_disc=None):
    """The FP64 oracle on the host cores, on the 2048^2 workload: SGP
    iterations per second on one core (numpy.fft) and with the transforms on
    every core (scipy.fft workers = os.cpu_count())."""
    cores = os.cpu_count() or 1
    t_0 = time.perf_counter()
    setup1, per1 = oracle_rate(w, iters)
    setupn, pern = oracle_rate(w, iters, workers=cores)
    spent = time.perf_counter() - t_0
    out = {"value": 1.0 / per1, "unit": "iter/s", "cores": 1, "kind": "oracle",
           "sample": f"{iters} SGP iterations of the {w.g.shape[-2]}x{w.g.shape[-1]} workload, "
                     f"oracle setup time subtracted ({spent:.1f} s of CPU work for both legs); "
                     f"host has {cores} logical CPUs",
           "all_cores": {"value": 1.0 / pern, "unit": "iter/s", "cores": cores,
                         "fft": f"scipy.fft, workers={cores}"}}
    if gpu_iters_to_disc:
        out["time_to_discrepancy_s_estimated"] = {
            "one_core": setup1 + per1 * gpu_iters_to_disc, "all_cores": setupn + pern * gpu_iters_to_disc,
            "iterations": gpu_iters_to_disc,
            "how": "oracle setup + s/iteration x the iteration count the GPU run needed"}
    return out


def config_rates(torch, m, steps, warmup, with_oracle, tune_tiles=True):
    """SGP iterations per second on the multi-image (3 x 1024^2) and the
    boundary-corrected (1024^2 window in a 1280^2 domain) workloads, each
    with its bytes model and fraction of the HBM roofline, under the tile
    schedule the autotuner picks on that problem; with the oracle, its
    seconds per iteration on the same input (2 timed iterations, one core)."""
    from synth import workloads as W
    out = {}
    for name, w in (("multi_3x1024", W.config2()), ("boundary_1280", W.config3())):
        g = torch.from_numpy(w.g).cuda()
        psf = torch.from_numpy(w.psf).cuda()
        p, ny, nx = w.g.shape
        if w.domain is not None:
            NY, NX = w.domain[0], w.domain[1]
        else:
            NY, NX = ny, nx
        tiles = None
        if tune_tiles:
            r, c, ms = m.autotune(g, psf, w.b, domain=w.domain, iters=96)
            tiles = {"rows_variant": r, "cols_variant": c,
                     "ms_per_iter": {f"{k[0]}{k[1]}": v for k, v in ms.items()}}
        S = m.Solver(m.KIND_SGP, g, psf, w.b, domain=w.domain, max_iter=steps + warmup + 10)
        S.prepare(steps)
        S.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rep = S.report()
        S.close()
        assert rep["iters"] == steps + warmup, rep["iters"]
        nb = iter_bytes(p, NY, NX, ny, nx, w.domain is not None)
        row = {"images": p, "window": [ny, nx], "fft_domain": [NY, NX], "iter_per_s": 1.0 / dt,
               "ms_per_iteration": 1e3 * dt, "bytes_per_iteration": nb,
               "achieved_GBs": nb / dt / 1e9, "frac": nb / dt / 1e9 / HBM_PEAK_GBS}
        if tiles is not None:
            row["tile_schedule"] = tiles
        if with_oracle:
            _, per = oracle_rate(w, 2)
            row["oracle_s_per_iteration_one_core"] = per
        out[name] = row
    return out


def note(msg):
    """One progress line per finished leg, on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    batch_items = None if args.no_batch else make_batch_inputs(args.batch_images)
    import numpy as np
    import torch

    import paper_1210_2258_amd as m
    from synth import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    m.load()
    w = W.config1(size=args.size)
    ny, nx = w.g.shape[-2:]
    npx = ny * nx
    g = torch.from_numpy(w.g[0]).cuda()
    psf = torch.from_numpy(w.psf[0]).cuda()
    b = float(w.b[0])
    torch.cuda.synchronize()

    if args.copy_calib:
        # a plain copy of known size (an elementwise multiply by one, so the
        # dispatch has a name of its own): FETCH_SIZE / WRITE_SIZE of this
        # dispatch give the counters' scale for the solver kernels
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    tiles = {}
    if args.tiles:
        m.set_tile_schedule(nx, args.tiles[0], m.get_tile_schedule(nx)[1])
        m.set_tile_schedule(ny, m.get_tile_schedule(ny)[0], args.tiles[1])
        tiles[f"{ny}x{nx}"] = {"rows_variant": args.tiles[0], "cols_variant": args.tiles[1],
                               "ms_per_iter": None, "set_by": "--tiles"}
    elif not args.no_autotune:
        tune(m, g, psf, b, 96, tiles)
        note(f"tile autotune done: {tiles}")

    # ---- throughput: W warm-up iterations, then exactly K timed iterations
    # (the graphs the timed call replays are captured before it)
    total = args.warmup + args.steps
    S = m.Solver(m.KIND_SGP, g, psf, b, max_iter=total + 10)
    S.prepare(args.steps)
    S.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = S.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = S.report()
    assert not done and rep["iters"] == total, (done, rep["iters"], total)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    its = args.steps / elapsed

    # ---- per-kernel durations (HIP events around each launch, no graph)
    S.set_timing(True)
    S.step(8)
    tm = S.timing()
    S.close()
    kern = {k: (ms / c if c else 0.0, c, ms) for k, (ms, c) in tm.items() if c}
    dom = max((k for k in kern if k in BYTES_PER_PX), key=lambda k: kern[k][2])
    avg_ms = kern[dom][0]
    achieved = BYTES_PER_PX[dom] * npx / (avg_ms * 1e-3) / 1e9
    iter_ms_events = sum(v[2] for v in kern.values()) / 8
    iter_roofline = ITER_BYTES_PER_PX * npx / (ms_per_step * 1e-3) / 1e9
    note(f"throughput {its:.0f} iter/s, per-kernel timing done")

    out_ttd = {}
    f_full = None
    if not args.no_ttd:
        out_ttd, f_full = time_to_discrepancy(torch, m, g, psf, b)
        note("time to discrepancy done")
    traffic = counter_traffic(dom, npx)
    
    out = {
        "metric": METRIC,
        "value": its,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"c1 galaxy field {ny}x{nx}: 20 Sersic profiles + 500 stars, 1e8 counts, "
                               "Airy (first zero 4 px) + 1% Gaussian halo PSF, b = 50, single-image SGP "
                               "with RL scaling, FP64 reductions",
                   "image": [ny, nx], "images_per_step": 1, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                     "avg_ms": avg_ms, "bytes_per_launch": BYTES_PER_PX[dom] * npx},
        "iteration_roofline": {"bytes_per_iter": ITER_BYTES_PER_PX * npx, "achieved_GBs": iter_roofline,
                               "frac": iter_roofline / HBM_PEAK_GBS},
        "kernels_ms": {k: v[0] for k, v in kern.items()},
        "iteration_ms_events": iter_ms_events,
        **out_ttd,
    }
    if batch_items is not None:
        out["batch_512"] = batch_legs(torch, m, batch_items, None if args.no_autotune else tiles)
        note("batch legs done")
    if tiles:
        out["tile_schedule"] = tiles
    if not args.no_multi:
        out["multi_image_3x1024"] = multi_image_legs(torch, m, W.config2())
        note("multi-image legs done")
    if not args.no_mosaic and f_full is not None:
        out["mosaic_2048"] = mosaic_leg(torch, m, w, g, psf, f_full, None if args.no_autotune else tiles)
        note("mosaic leg done")
    if not args.no_mall and args.size == 2048:
        out["beyond_mall_4x2048"] = beyond_mall_leg(torch, m, g, psf, b)
        note("beyond-MALL leg done")
    if not args.no_sweep:
        out["rebin_sweep"] = rebin_sweep(torch, m, with_oracle=not args.no_cpu)
        note("rebin sweep done")
    if not args.no_configs:
        out["configs"] = config_rates(torch, m, 100, 10, not args.no_cpu, tune_tiles=not args.no_autotune)
        note("config rates done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_iters, out_ttd.get("iters_to_discrepancy"))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
