"""How far FP32 storage alone moves an SGP run (CPU, oracle only).

The oracle's own iteration is re-run with f and d rounded to float32 after
every update (everything else FP64).  The distance to the exact FP64 run is
the floor any FP32-field implementation faces; the fixed iteration counts of
the GPU parity tests are chosen below the point where it reaches the
tolerances (KL 1e-6, f 1e-4)."""
import numpy as np
import pytest

from oracle import sgp as O
from synth import workloads as W


def _r32(a):
    return a.astype(np.float32).astype(np.float64)


def _sgp_fp32_fields(P, f0, n, L1, L2):
    prm = O.Params(max_iter=n)
    f = _r32(f0)
    J, G = P.kl(f), P.grad(f)
    alpha, tau, Q = prm.alpha0, prm.tau1, []
    hist = []
    for k in range(n):
        D = P.scaling(f, L1, L2)
        d = _r32(np.maximum(0.0, f - alpha * D * G) - f)
        gd = float(np.sum(G * d))
        lam = 1.0
        while P.kl(f + lam * d) > J + prm.beta * lam * gd:
            lam *= prm.theta
        fn = _r32(f + lam * d)
        Jn, Gn = P.kl(fn), P.grad(fn)
        s, z = fn - f, Gn - G
        Dn = P.scaling(fn, L1, L2)
        m = Dn > 0
        sums = (np.sum(s[m] ** 2 / Dn[m] ** 2), np.sum(s[m] * z[m] / Dn[m]),
                np.sum(s[m] * z[m] * Dn[m]), np.sum(z[m] ** 2 * Dn[m] ** 2))
        _, _, _, _, alpha, tau, Q, _ = O.steplength_update(alpha, tau, Q, k, *sums, prm)
        f, J, G = fn, Jn, Gn
        hist.append(J)
    return f, np.array(hist)


@pytest.mark.parametrize("make,k_ok,k_bad", [(lambda: W.small_single(64, 80), 10, 30)])
def test_fp32_storage_floor(make, k_ok, k_bad):
    w = make()
    P = O.Problem(w.g, w.psf, w.b)
    f0 = P.start("flat")
    fo, io = P.sgp(f0, O.Params(max_iter=k_bad))
    f32, h32 = _sgp_fp32_fields(P, f0, k_bad, io["L1"], io["L2"])
    ho = np.array(io["history"][1:])
    rel = np.abs(h32 / ho - 1)
    assert rel[k_ok - 1] < 1e-7          # well inside the KL bar at the parity count
    assert rel[k_bad - 1] > 1e-6         # FP32 storage alone breaks the KL bar later
