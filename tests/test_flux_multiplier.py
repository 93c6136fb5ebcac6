"""The device's search for the flux-projection multiplier (the constraint set
{f >= 0, sum f = c} of Sect. 2, projected in the D^-1 metric), run on the
host through the library's own finalisers, against the oracle's exact
breakpoint scan; and its report when the Newton passes the solver allows per
iteration end before the root."""
import numpy as np

import paper_1210_2258_amd as m
from oracle import sgp as O

SGP_W_FLUX_UNCONVERGED = 4


def test_matches_breakpoint_scan():
    rng = np.random.default_rng(7)
    for n, extra in ((50, 3.0), (400, 10.0), (1000, 0.5)):
        z = rng.normal(0.5, 1.0, n)
        D = rng.uniform(0.1, 2.0, n)
        D[rng.random(n) < 0.1] = 0.0  # pixels outside R: held at max(0, z)
        c = np.maximum(0.0, z[D == 0]).sum() + extra
        mu, steps, conv, rc = m.flux_multiplier(z, D, c, max_steps=64)
        assert conv and rc == 0
        x = np.where(D > 0, np.maximum(0.0, z - mu * D), np.maximum(0.0, z))
        xo = O.flux_projection(z, D, c)
        assert abs(x.sum() - c) <= 1e-12 * c
        assert np.allclose(x, xo, rtol=0, atol=1e-12)


def test_slow_newton_reported():
    # breakpoints t_i = i + 1 with weights D_i = 2^-i and a tiny flux: each
    # Newton step from the left passes only one breakpoint, so the root needs
    # 12 steps, more than the 8 the solver runs per iteration
    n = 12
    D = 0.5 ** np.arange(n)
    z = np.arange(1, n + 1) * D
    c = 1e-5
    mu8, steps8, conv8, rc8 = m.flux_multiplier(z, D, c, max_steps=8)
    assert steps8 == 8 and not conv8 and rc8 == SGP_W_FLUX_UNCONVERGED
    mu, steps, conv, rc = m.flux_multiplier(z, D, c, max_steps=32)
    assert conv and rc == 0 and steps == 12
    xo = O.flux_projection(z, D, c)
    x = np.maximum(0.0, z - mu * D)
    assert np.allclose(x, xo, rtol=0, atol=1e-15)
    # the unconverged multiplier lies left of the root: the projection's sum
    # exceeds c (what the warning reports)
    assert mu8 < mu and np.maximum(0.0, z - mu8 * D).sum() > c
