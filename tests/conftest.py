import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture
def one_step_at_depth():
    """Returns check(torch, w, depth, f_tol, kl_tol): the HIP path's SGP
    iteration number ``depth`` against one FP64 oracle iteration started from
    the HIP path's own state: iterate f_depth, the gradient it carries there,
    steplength alpha_depth and bounds L1, L2.  Whole trajectories part after some tens of iterations (the
    Barzilai-Borwein steplengths amplify FP32 rounding), while this compares
    the arithmetic of one iteration at any depth: the Armijo decision, the
    updated f and its KL, and the two Barzilai-Borwein values formed from
    the new gradient."""
    import numpy as np

    from oracle import sgp as O

    def check(torch, w, depth, f_tol, kl_tol):
        import paper_1210_2258_amd as m
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
        stacked = w.p > 1 or w.domain is not None
        g = dev(w.g if stacked else w.g[0])
        psf = dev(w.psf if stacked else w.psf[0])
        b = w.b if stacked else float(w.b[0])
        # two iterations past the one checked: the capped last iteration
        # does not form the next steplength
        S = m.Solver(m.KIND_SGP, g, psf, b, domain=w.domain, trace=True, max_iter=depth + 2)
        S.step(depth)
        torch.cuda.synchronize()
        fk = S.f.cpu().numpy().astype(np.float64)
        gk = S.gradient().cpu().numpy().astype(np.float64)
        S.step(1)
        torch.cuda.synchronize()
        f1 = S.f.cpu().numpy()
        rep = S.report()
        S.close()
        assert rep["iters"] == depth + 1
        tr = {k: v[depth] for k, v in rep["trace"].items()}
        P = O.Problem(w.g, w.psf, w.b, domain=w.domain)
        # the oracle's iteration from the GPU's own state: f_k, the gradient it
        # carries there (start gradient plus every step's change, in FP32),
        # alpha_k and the bounds
        fo, io = P.sgp(fk, O.Params(max_iter=1, alpha0=float(tr["alpha"])),
                       bounds=(rep["L1"], rep["L2"]), grad0=gk)
        L = io["log"][0]
        assert int(tr["backtracks"]) == L["backtracks"], (tr["backtracks"], L["backtracks"])
        rel = float(np.linalg.norm(f1.astype(np.float64) - fo) / np.linalg.norm(fo))
        assert rel <= f_tol, rel
        assert abs(rep["kl"] - io["kl"]) <= kl_tol * io["kl"], (rep["kl"], io["kl"])
        # alpha1 = a / c1 and alpha2 = c2 / e are ratios of inner products of
        # the step s, the gradient change z and D.  z comes from FP32
        # transforms, whose error is absolute (~1e-7 of the largest entry of
        # z, not relative per pixel), so each sum's error bound is 1e-6
        # max|z| (10x that) times the sum of the absolute values of its other
        # factors; relative to the sum it grows with the cancellation.  The
        # bar is that bound plus twice the measured relative difference of
        # the two steps (which enters a quadratically), at least 1e-3.
        s_ = fo - fk
        e_s = float(np.linalg.norm(f1.astype(np.float64) - fk - s_) / np.linalg.norm(s_))
        z_ = P.grad(fo) - P.grad(fk)
        D = P.scaling(fo, rep["L1"], rep["L2"])
        msk = D > 0
        s_, z_, D = s_[msk], z_[msk], D[msk]
        ez = 1e-6 * np.abs(z_).max()
        c1 = np.sum(s_ * z_ / D)
        c2, e = np.sum(s_ * z_ * D), np.sum(z_ * z_ * D * D)
        b1 = ez * np.sum(np.abs(s_ / D)) / abs(c1)
        b2 = ez * np.sum(np.abs(s_ * D)) / abs(c2) + 2 * ez * np.sum(np.abs(z_) * D * D) / e
        for key, bnd in (("a1", b1), ("a2", b2)):
            tol = max(1e-3, 2 * e_s + bnd)
            print(f"depth {depth} {key}: rel diff {abs(tr[key] / L[key] - 1):.1e}, step diff {e_s:.1e}, "
                  f"bar {tol:.1e}", flush=True)
            assert abs(tr[key] - L[key]) <= tol * abs(L[key]), (key, tr[key], L[key], tol)
        return rel

    return check
