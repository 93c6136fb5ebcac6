"""SGP (Algorithm 1) with the rounding of an FP32 implementation, on the CPU.

Test infrastructure: a model of where a single-precision implementation
rounds, used to tell how soon FP32 arithmetic by itself moves an SGP run
away from the exact FP64 one.  It follows the order of operations the GPU
path uses (the oracle is left untouched):

* fields (f, grad, A_j f, A_j d, the direction) are float32;
* every 2D transform runs in single precision (scipy.fft on complex64), and
  the transfer functions are computed the same way from the float32
  unit-volume PSF;
* the pointwise terms are float32: the residual change
  -g lam A_j d / (y y_new) fed to the adjoint, the KL terms
  g h((y - g) / g) and the Armijo terms (y - g) x + g h(x), x = lam A_j d / y,
  with h(x) = x - log1p(x) (series for |x| < 1/2);
* the gradient is carried as grad + z, z = -M_R sum_j A_j^T(delta rho_j);
* sums (KL, grad^T d, the Armijo differences, the four BB sums) are float64,
  as are the scalar rules (Armijo test, Eqs. (BB1), (BB2), (alphadef)),
  which come from the oracle's steplength rule.

It is not bit-identical to the GPU (its FFTs round in another order); it
shows the size of the FP32 effect, not its exact pattern.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from oracle import sgp as O

f32 = np.float32
c64 = np.complex64   # the complex type of the transforms (float32 pairs)


def _fft2(x):
    return scipy.fft.fft2(x.astype(c64))


def _ifft2(x):
    return scipy.fft.ifft2(x.astype(c64))


def _h(x):
    """h(x) = x - log1p(x) in float32 (series in u = x / (2 + x) for |x| < 1/2)."""
    x = x.astype(f32)
    out = np.empty_like(x)
    sm = np.abs(x) < f32(0.5)
    xs = x[sm]
    u = (xs / (f32(2) + xs)).astype(f32)
    u2 = (u * u).astype(f32)
    q = np.full_like(u, f32(1.0 / 19.0))
    for k in range(17, 2, -2):
        q = (f32(1.0 / k) + u2 * q).astype(f32)
    out[sm] = xs * u - f32(2) * u * u2 * q
    xl = x[~sm]
    out[~sm] = xl - np.log1p(xl).astype(f32)
    return out


def _kl_terms(g, y):
    """float32 KL terms, summed in float64."""
    t = np.where(g > 0, g * _h(((y - g) / np.where(g > 0, g, f32(1))).astype(f32)), y).astype(f32)
    return float(np.sum(t, dtype=np.float64))


def _armijo(g, y, t):
    x = (t / y).astype(f32)
    return float(np.sum(((y - g) * x).astype(np.float64) + (g * _h(x)).astype(np.float64)))


class Fp32Problem:
    """The problem of an oracle ``Problem`` (same inputs, normalisation and
    masks), its operators evaluated in single precision."""

    def __init__(self, P: O.Problem):
        self.P = P
        self.p = P.p
        K32 = (P.K).astype(f32)
        self.Khat = np.stack([_fft2(np.fft.ifftshift(K32[j])) for j in range(P.p)]).astype(c64)
        if P.boundary:
            MS = P.MS.astype(f32)
            alpha = np.stack([np.real(_ifft2(np.conj(self.Khat[j]) * _fft2(MS))).astype(f32)
                              for j in range(P.p)])
            R = np.all(alpha.astype(np.float64) >= 1e-3, axis=0)
            s = alpha.astype(np.float64).sum(axis=0)
            self.invw = np.where(R, 1.0 / np.where(R, s, 1.0), 0.0).astype(f32)
        else:
            self.invw = np.full((P.NY, P.NX), f32(1.0 / P.p), dtype=f32)
        self.g = P.g.astype(f32)
        self.b = P.b.astype(f32)
        self.S = P.S

    def A(self, j, x):
        return np.real(_ifft2(self.Khat[j] * _fft2(x))).astype(f32)[self.S]

    def AT_sum(self, rhos):
        """M_R o sum_j A_j^T rho_j, the sum taken in Fourier space."""
        P = self.P
        acc = np.zeros((P.NY, P.NX), c64)
        for j in range(self.p):
            e = np.zeros((P.NY, P.NX), f32)
            e[self.S] = rhos[j]
            acc += np.conj(self.Khat[j]) * _fft2(e)
        v = np.real(_ifft2(acc)).astype(f32)
        return np.where(self.invw > 0, v, f32(0))


def sgp_fp32(P: O.Problem, n_iter: int, prm: O.Params | None = None):
    """n_iter SGP iterations from the flat start; returns (f, KL history
    J_0..J_n, per-iteration log of alpha and backtracks)."""
    prm = prm or O.Params(max_iter=n_iter)
    E = Fp32Problem(P)
    p = E.p
    f = (f32(P.start("flat").max()) * (E.invw > 0)).astype(f32)
    Af = [E.A(j, f) for j in range(p)]
    ys = [np.maximum(Af[j] + E.b[j], f32(1e-30)) for j in range(p)]
    J = sum(_kl_terms(E.g[j], ys[j]) for j in range(p))
    rho = [((E.g[j] - ys[j]) / ys[j]).astype(f32) for j in range(p)]
    v = E.AT_sum(rho)
    grad = (-v).astype(f32)
    yr = np.where(E.invw > 0, f * (f32(1) + E.invw * v), f32(0)).astype(f32)
    MS = np.zeros(f.shape, bool)
    MS[E.S] = True
    pos = yr[(yr > 0) & MS].astype(np.float64)
    ymin, ymax = pos.min(), pos.max()
    L1, L2 = (ymin / 10, ymax * 10) if ymax / ymin < 50 else (ymin, ymax)
    L1f, L2f = f32(L1), f32(L2)
    alpha, tau, Q = prm.alpha0, prm.tau1, []
    hist, log = [J], []
    lam_tab = [prm.theta ** m for m in range(prm.max_backtracks + 1)]
    for k in range(n_iter):
        al = f32(alpha)
        D = (E.invw * np.minimum(L2f, np.maximum(L1f, f))).astype(f32)
        z = (f.astype(np.float64) - (al * D).astype(np.float64) * grad).astype(f32)  # one fused multiply-add
        d = (np.maximum(f32(0), z) - f).astype(f32)
        gd = float(np.sum(grad.astype(np.float64) * d))
        Ad = [E.A(j, d) for j in range(p)]
        ys = [np.maximum(Af[j] + E.b[j], f32(1e-30)) for j in range(p)]
        nback = None
        for m, lam in enumerate(lam_tab):
            dJ = sum(_armijo(E.g[j], ys[j], (f32(lam) * Ad[j]).astype(f32)) for j in range(p))
            if dJ <= prm.beta * lam * gd:
                nback = m
                break
        if nback is None:
            break
        lam = lam_tab[nback]
        lamf = f32(lam)
        Afn, drho, Jn = [], [], 0.0
        for j in range(p):
            step = (lamf * Ad[j]).astype(f32)
            afn = (Af[j] + step).astype(f32)
            yn = np.maximum(afn + E.b[j], f32(1e-30))
            Jn += _kl_terms(E.g[j], yn)
            g = E.g[j]
            drho.append(np.where(g > 0, (-g * step / (ys[j] * yn)).astype(f32), f32(0)))
            Afn.append(afn)
        v = E.AT_sum(drho)
        zf = np.where(E.invw > 0, -v, f32(0)).astype(f32)
        grad_n = (grad + zf).astype(f32)
        fn = (f.astype(np.float64) + np.float64(lamf) * d).astype(f32)   # one fused multiply-add
        s = lam * d.astype(np.float64)
        zz = zf.astype(np.float64)
        Dn = (E.invw * np.minimum(L2f, np.maximum(L1f, fn))).astype(f32).astype(np.float64)
        msk = Dn > 0
        sd = s[msk] / Dn[msk]
        sums = (float(np.sum(sd * sd)), float(np.sum(sd * zz[msk])),
                float(np.sum(s[msk] * zz[msk] * Dn[msk])), float(np.sum(zz[msk] ** 2 * Dn[msk] ** 2)))
        a1, a2, _, _, alpha_n, tau, Q, _ = O.steplength_update(alpha, tau, Q, k, *sums, prm)
        log.append(dict(alpha=alpha, backtracks=nback, a1=a1, a2=a2))
        f, grad, Af, J, alpha = fn, grad_n, Afn, Jn, alpha_n
        hist.append(J)
    return f, np.array(hist), log


def kl_gap_crossing(h, ho, bar=1e-6):
    """First iteration k >= 1 with |h[k] / ho[k] - 1| > bar (None if never)."""
    n = min(len(h), len(ho))
    rel = np.abs(np.asarray(h[:n]) / np.asarray(ho[:n]) - 1.0)
    idx = np.nonzero(rel[1:] > bar)[0]
    return int(idx[0]) + 1 if idx.size else None
