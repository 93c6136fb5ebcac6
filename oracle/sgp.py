"""Plain float64 CPU oracle for SGP / Richardson-Lucy Poisson deconvolution.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code,
table or helper with the HIP library and imports nothing from it.

It follows Prato, Cavicchioli, Zanni, Boccacci, Bertero, "Efficient
deconvolution methods for astronomical imaging: algorithms and IDL-GPU codes"
(A&A 539, A133, 2012; arXiv:1210.2258):

* imaging model and RL iteration ............ Sect. 1, Eq. (RL)
* KL divergence ............................. Sect. 1, Eq. (divergence)
* SGP ....................................... Sect. 2.1, Algorithm 1
* scaled BB rules, safeguards, alternation .. Sect. 2.1, Eqs. (BB1), (BB2), (alphadef)
* RL scaling matrix ......................... Sect. 2.1, Eq. (Dk)
* single-image gradient ..................... Sect. 2.2, Eq. (KLgrad)
* multiple images ........................... Sect. 2.3, Eqs. (multipleKL), (multipleRL), (multiplegradient)
* boundary effect correction ................ Sect. 2.4, Eqs. (projection), (backprojection),
                                              (gradientboundary), (Rdef), (boundaryRL), (Dkbound)
* OSEM (ordered subsets over the images) ..... Sect. 2.3, Algorithm 2, Eq. (OSEMstep);
                                              Sect. 2.4, Eq. (boundaryOSEM)
* mosaic of boundary-corrected subdomains ..... Sect. 4.1 (second experiment): overlapping
                                              windows, each reconstructed with Sect. 2.4,
                                              non-overlapping cores stitched
* start, parameters, adaptive bounds ........ Sect. 3.1, 3.2
* stopping rules ............................ Sect. 3.3, Eqs. (convergence), (discrepancy)
* flux-constrained projection ............... Sect. 2 intro (constraint set named, algorithm
                                              not given); derived here from the KKT conditions
* relaxed RL ................................ Sect. 1, Eq. (RL1) (multiplicative relaxation)
* linearly relaxed RL ....................... Sect. 1, Eq. (RL2) with the Armijo rule

Every array is float64.  Inputs given in float32 are promoted.  The iteration
is written step by step in the paper's order and notation; library primitives
(``numpy.fft``, ``numpy.sort``) are the only building blocks.

Readings of points the paper leaves open (each is a named parameter or a
documented choice, shared with the HIP library by specification, not by code):

* which D in the BB rules: the scaling of the new iterate, D_{k+1}=D(f^{(k+1)});
* the first ``n_bb2_only`` (20) steplengths use the min-rule of Eq. (alphadef)
  without touching tau; alternation starts afterwards;
* the memory of alpha^(2) values holds only the values computed so far;
* "10 alpha_{k-1}" is the steplength used in the step just taken;
* the RL step of Sect. 3.2 only sets (L1, L2); SGP starts from f^(0); its
  min / max are taken over S (equal to R unless boundary-corrected);
* a term with g = 0 contributes y to the KL sum;
* boundary weights alpha_j = K_j (correlated with) M_S, i.e. A_j^T 1 before M_R;
* multi-image scaling D = clip(f, L1, L2) / p;
* flat start = mean_j sum_S (g_j - b_j) / |S|, put on R only;
* discrepancy stop at the first k with 2 J / (p |S|) <= b_D; KL summed over S;
* reconstruction-error stop (Sect. 3.3, needs the true object): rho^(k) is
  taken for k = 0, 1, ... as each iterate is formed; at the first k with
  rho^(k) > rho^(k-1) the run returns f^(k-1), the minimum (for SGP this
  rule is tested after the discrepancy and convergence rules of the same
  iterate; for RL and OSEM before them, since the error is known before the
  iterate's KL);
* backtracking capped at ``max_backtracks``; d = 0 stops as stationary;
* BB sums taken over pixels with D > 0 (D^{-1} is undefined off R);
* relaxed RL for several images or a boundary problem: Eq. (RL1) is written
  for one image with A^T 1 = 1; the factor it raises to the power a is taken
  as the RL factor q = (M_R / alpha) o sum_j A_j^T (g_j / (A_j f + b_j)) of
  Eqs. (multipleRL), (boundaryRL), so the step is f o q^a (RL for a = 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

STOP_FIXED = 1
STOP_CONV = 2
STOP_DISCREPANCY = 4
STOP_RMSE = 8

REASON_MAXITER = 0
REASON_CONV = 1
REASON_DISCREPANCY = 2
REASON_RMSE = 3
REASON_STATIONARY = 4
REASON_ARMIJO = 5


# Threads of the 2D transforms.  None: numpy.fft (one thread, what every pin
# runs); an integer n: scipy.fft with n workers, the same discrete Fourier
# transform, used only to time the oracle on several host cores.
FFT_WORKERS = None


def _fft2(x):
    if FFT_WORKERS:
        import scipy.fft
        return scipy.fft.fft2(x, workers=FFT_WORKERS)
    return np.fft.fft2(x)


def _ifft2(x):
    if FFT_WORKERS:
        import scipy.fft
        return scipy.fft.ifft2(x, workers=FFT_WORKERS)
    return np.fft.ifft2(x)


@dataclass
class Params:
    """Sect. 3.2 defaults (beta, theta, alpha0, tau1, alpha_max, M_alpha,
    alpha_min) plus the Sect. 3.3 stopping controls."""
    max_iter: int = 1000
    stop: int = STOP_FIXED
    tol: float = 1e-4
    disc_target: float = 1.0
    beta: float = 1e-4
    theta: float = 0.4
    alpha0: float = 1.3
    alpha_min: float = 1e-5
    alpha_max: float = 1e5
    tau1: float = 0.5
    m_alpha: int = 3
    n_bb2_only: int = 20
    auto_bounds: bool = True
    L1: float = 1e-10
    L2: float = 1e10
    flux_constraint: bool = False
    flux: float = -1.0
    max_backtracks: int = 40
    f_true: np.ndarray | None = None
    rl_alpha: float = 1.0   # exponent of Eq. (RL1); 1 is RL
    rl_lambda_cap: float = 10.0  # Eq. (RL2) line search: largest step tried (with the nonnegativity bound)


def _as_stack(a, p=None):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 2:
        a = a[None]
    return a


class Problem:
    """p images g_j observed on S (ny x nx), PSFs K_j on Sbar (NY x NX),
    backgrounds b_j on S.  Without ``domain`` the problem is periodic and
    Sbar = S.  With ``domain=(NY, NX, oy, ox)`` S sits at offset (oy, ox)
    inside Sbar (Sect. 2.4)."""

    def __init__(self, g, psf, b, domain=None, sigma_R=1e-3):
        g = _as_stack(g)
        self.p, self.ny, self.nx = g.shape
        psf = _as_stack(psf)
        if domain is None:
            self.NY, self.NX, self.oy, self.ox = self.ny, self.nx, 0, 0
            self.boundary = False
        else:
            self.NY, self.NX, self.oy, self.ox = (int(v) for v in domain)
            self.boundary = True
        if psf.shape != (self.p, self.NY, self.NX):
            raise ValueError("PSF stack must be [p, NY, NX]")
        b = np.asarray(b, dtype=np.float64)
        if b.ndim == 0:
            b = np.full((self.p, self.ny, self.nx), float(b))
        elif b.ndim == 1:
            b = b[:, None, None] * np.ones((1, self.ny, self.nx))
        elif b.ndim == 2:
            b = b[None] * np.ones((self.p, 1, 1))
        self.g, self.b = g, b
        self.S = (slice(self.oy, self.oy + self.ny), slice(self.ox, self.ox + self.nx))
        # Sect. 2.2-2.4: every PSF normalised to unit volume (over Sbar)
        K = psf / psf.sum(axis=(1, 2), keepdims=True)
        # PSF centre at (NY//2, NX//2) is moved to the origin before the FFT
        self.K = K
        self.Khat = np.fft.fft2(np.fft.ifftshift(K, axes=(1, 2)), axes=(1, 2))
        self.MS = np.zeros((self.NY, self.NX))
        self.MS[self.S] = 1.0
        if self.boundary:
            # weights of Sect. 2.4: alpha_j(n) = sum_m K_j(m-n) M_S(m)
            self.alpha_j = np.stack([self._corr(j, self.MS) for j in range(self.p)])
            # Eq. (Rdef): R = {n : alpha_j(n) >= sigma for all j}
            self.MR = np.all(self.alpha_j >= sigma_R, axis=0).astype(np.float64)
        else:
            self.alpha_j = np.ones((self.p, self.NY, self.NX))
            self.MR = np.ones((self.NY, self.NX))
        self.alpha = self.alpha_j.sum(axis=0)
        # M_R / alpha, the quotient being zero outside R (Eqs. boundaryRL, Dkbound);
        # 1/p for periodic multiple images (scaling f/p of Sect. 2.3)
        self.invw = np.where(self.MR > 0, 1.0 / np.where(self.MR > 0, self.alpha, 1.0), 0.0)
        self.nS = self.ny * self.nx

    # ---------------------------------------------------------------- operators
    def _conv(self, j, x):
        return np.real(_ifft2(self.Khat[j] * _fft2(x)))

    def _corr(self, j, x):
        return np.real(_ifft2(np.conj(self.Khat[j]) * _fft2(x)))

    def embed(self, x_S):
        """Zero-pad an array on S into Sbar (the M_S o . of Eq. backprojection)."""
        out = np.zeros((self.NY, self.NX))
        out[self.S] = x_S
        return out

    def A(self, j, f):
        """Eq. (projection): (A_j f) = M_S o (K_j * (M_R o f)); returned on S."""
        return self._conv(j, self.MR * f)[self.S]

    def AT(self, j, y_S):
        """Eq. (backprojection): A_j^T y = M_R o (K_j correlated with M_S o y)."""
        return self.MR * self._corr(j, self.embed(y_S))

    def A_direct(self, j, f):
        """Brute-force O(N^2) periodic convolution, for tests only."""
        NY, NX = self.NY, self.NX
        K0 = np.fft.ifftshift(self.K[j])
        fm = self.MR * f
        out = np.zeros((NY, NX))
        ys, xs = np.nonzero(fm)
        for n_y, n_x in zip(ys, xs):
            out += fm[n_y, n_x] * np.roll(np.roll(K0, n_y, axis=0), n_x, axis=1)
        return out[self.S]

    # ------------------------------------------------------------- objective
    def y(self, j, f):
        return self.A(j, f) + self.b[j]

    def kl(self, f):
        """Eqs. (divergence) / (multipleKL), summed over S; g = 0 terms give y."""
        J = 0.0
        for j in range(self.p):
            y = self.y(j, f)
            g = self.g[j]
            if np.any((y <= 0) & (g > 0)):
                raise FloatingPointError("A f + b <= 0 where g > 0")
            pos = g > 0
            t = y - g
            t[pos] += g[pos] * np.log(g[pos] / y[pos])
            J += t.sum()
        return J

    def grad(self, f):
        """Eqs. (KLgrad), (multiplegradient), (gradientboundary):
        sum_j {A_j^T 1 - A_j^T (g_j / (A_j f + b_j))}."""
        G = np.zeros((self.NY, self.NX))
        for j in range(self.p):
            G += self.MR * self.alpha_j[j] - self.AT(j, self.g[j] / self.y(j, f))
        return G

    def discrepancy(self, J):
        """Eq. (discrepancy), N^2 read as the pixel count of one observed image."""
        return 2.0 * J / (self.p * self.nS)

    # ---------------------------------------------------------- RL family
    def rl_factor(self, f):
        """q = (M_R / alpha) o sum_j A_j^T (g_j / (A_j f + b_j)), the factor of
        Eqs. (RL), (multipleRL), (boundaryRL)."""
        s = np.zeros((self.NY, self.NX))
        for j in range(self.p):
            s += self.AT(j, self.g[j] / self.y(j, f))
        return self.invw * s

    def rl_step(self, f, rl_alpha=1.0):
        """Eqs. (RL), (multipleRL), (boundaryRL): f <- f o q; with
        rl_alpha != 1 the multiplicative relaxation of Eq. (RL1), f o q^a
        (f stays 0 off R, as in RL)."""
        q = self.rl_factor(f)
        if rl_alpha == 1.0:
            return f * q
        return np.where(self.invw > 0, f * q ** rl_alpha, 0.0)

    def start(self, kind="flat", user=None):
        """Sect. 3.1 initial points."""
        if kind == "zero":
            return np.zeros((self.NY, self.NX))
        if kind == "data":
            return self.MR * self.embed(self.g[0])
        if kind == "user":
            return np.asarray(user, dtype=np.float64).copy()
        c = np.mean([(self.g[j] - self.b[j]).sum() for j in range(self.p)]) / self.nS
        if c <= 0:
            c = 1e-6 * max(self.g.mean(), 1e-30)
        return c * self.MR

    def bounds(self, f0):
        """Sect. 3.2: one RL step, min positive / max of the result.

        With boundary correction the extrema are taken over the observed
        window S: outside S the RL values rest on weights alpha_j that may be
        as small as sigma, a region the paper itself calls unreliable, and
        there the step is a ratio of two tiny numbers."""
        yr = self.rl_step(f0)
        pos = yr[(yr > 0) & (self.MS > 0)]
        ymin, ymax = pos.min(), pos.max()
        if ymax / ymin < 50:
            return ymin / 10.0, ymax * 10.0
        return ymin, ymax

    def rl(self, f0, n_iter, params: Params | None = None):
        """RL iteration (relaxed by Eq. (RL1) when rl_alpha differs from 1)
        with the Sect. 3.3 stopping rules."""
        prm = params or Params(max_iter=n_iter)
        f = f0.copy()
        J = self.kl(f)
        hist = [J]
        reason = REASON_MAXITER
        k = 0
        if (prm.stop & STOP_DISCREPANCY) and self.discrepancy(J) <= prm.disc_target:
            return f, dict(iters=0, kl=J, history=hist, reason=REASON_DISCREPANCY)
        rho = rel_error(f, prm.f_true) if rmse_active(prm) else None
        while k < n_iter:
            f_new = self.rl_step(f, prm.rl_alpha)
            # Sect. 3.3: the error of an iterate is known as soon as it is
            # formed; once it grows, the previous iterate (the minimum) is
            # returned
            if rho is not None:
                rho_new = rel_error(f_new, prm.f_true)
                if rho_new > rho:
                    reason = REASON_RMSE
                    break
                rho = rho_new
            f = f_new
            Jn = self.kl(f)
            k += 1
            hist.append(Jn)
            if (prm.stop & STOP_DISCREPANCY) and self.discrepancy(Jn) <= prm.disc_target:
                reason = REASON_DISCREPANCY
                J = Jn
                break
            if (prm.stop & STOP_CONV) and converged(Jn, J, prm.tol):
                reason = REASON_CONV
                J = Jn
                break
            J = Jn
        return f, dict(iters=k, kl=J, history=hist, reason=reason)

    def rl_linear(self, f0, n_iter, params: Params | None = None):
        """Linear relaxation of RL, Eq. (RL2): f <- f + lam d along the RL
        direction d = -(M_R / w) o f o grad J (the RL step minus f), with
        lam >= 1 chosen by the Armijo rule (Sect. 1 names a line search along
        this direction by the Armijo rule; the rule and its test are those of
        Algorithm 1, steps 4-5).  Reading: the largest step tried is
        lam_max = min(rl_lambda_cap, min over d_i < 0 of f_i / (-d_i)), the
        largest keeping f >= 0; candidates lam_max, theta lam_max, ... while
        above 1, then lam = 1, the RL step itself, taken when no larger
        candidate passes (it never increases J).  A step taken at the
        nonnegativity bound sets the pixels that bound it to exactly 0, as
        exact arithmetic does (rounding would leave them at a tiny positive
        or negative fraction of their value, alive or clipped by chance, and
        a live one would bound every later step).  With the same stopping
        rules as rl()."""
        prm = params or Params(max_iter=n_iter)
        f = f0.copy()
        J = self.kl(f)
        hist = [J]
        lams = []
        k = 0
        reason = REASON_MAXITER
        if (prm.stop & STOP_DISCREPANCY) and self.discrepancy(J) <= prm.disc_target:
            return f, dict(iters=0, kl=J, history=hist, lam=lams, reason=REASON_DISCREPANCY)
        rho = rel_error(f, prm.f_true) if rmse_active(prm) else None
        while k < n_iter:
            G = self.grad(f)
            d = -self.invw * f * G
            gd = float(np.sum(G * d))
            if gd == 0.0:
                reason = REASON_STATIONARY
                break
            neg = d < 0
            ratio = np.full(f.shape, np.inf)
            ratio[neg] = f[neg] / -d[neg]
            bound = float(ratio.min())
            lam_max = min(prm.rl_lambda_cap, bound)
            lam = lam_max
            while lam > 1.0:
                f_new = np.maximum(0.0, f + lam * d)
                if lam == bound:
                    f_new[ratio <= bound] = 0.0
                J_new = self.kl(f_new)
                if J_new <= J + prm.beta * lam * gd:
                    break
                lam *= prm.theta
            if lam <= 1.0:
                lam = 1.0
                f_new = np.maximum(0.0, f + d)
                J_new = self.kl(f_new)
            if rho is not None:  # Sect. 3.3, as in rl()
                rho_new = rel_error(f_new, prm.f_true)
                if rho_new > rho:
                    reason = REASON_RMSE
                    break
                rho = rho_new
            J_prev = J
            f, J = f_new, J_new
            k += 1
            hist.append(J)
            lams.append(lam)
            if (prm.stop & STOP_DISCREPANCY) and self.discrepancy(J) <= prm.disc_target:
                reason = REASON_DISCREPANCY
                break
            if (prm.stop & STOP_CONV) and converged(J, J_prev, prm.tol):
                reason = REASON_CONV
                break
        return f, dict(iters=k, kl=J, history=hist, lam=lams, reason=reason)

    # -------------------------------------------------------------- OSEM
    def osem_weight(self, j):
        """M_R / alpha_j, zero outside R (Eq. boundaryOSEM); for periodic
        problems alpha_j = A_j^T 1 = 1 and the weight is 1 (Eq. OSEMstep)."""
        return np.where(self.MR > 0, 1.0 / np.where(self.MR > 0, self.alpha_j[j], 1.0), 0.0)

    def osem_cycle(self, f):
        """Algorithm 2, steps 1-3: h^(0) = f, then for j = 1..p
        h^(j) = w_j o h^(j-1) o A_j^T (g_j / (A_j h^(j-1) + b_j)); returns h^(p)."""
        h = f.copy()
        for j in range(self.p):
            h = self.osem_weight(j) * h * self.AT(j, self.g[j] / self.y(j, h))
        return h

    def osem(self, f0, n_iter, params: Params | None = None):
        """OSEM cycles with the stopping rules of rl() (KL of each iterate f^(k))."""
        prm = params or Params(max_iter=n_iter)
        f = f0.copy()
        J = self.kl(f)
        hist = [J]
        k = 0
        if (prm.stop & STOP_DISCREPANCY) and self.discrepancy(J) <= prm.disc_target:
            return f, dict(iters=0, kl=J, history=hist, reason=REASON_DISCREPANCY)
        reason = REASON_MAXITER
        rho = rel_error(f, prm.f_true) if rmse_active(prm) else None
        while k < n_iter:
            f_new = self.osem_cycle(f)
            if rho is not None:  # Sect. 3.3, as in rl()
                rho_new = rel_error(f_new, prm.f_true)
                if rho_new > rho:
                    reason = REASON_RMSE
                    break
                rho = rho_new
            f = f_new
            Jn = self.kl(f)
            k += 1
            hist.append(Jn)
            if (prm.stop & STOP_DISCREPANCY) and self.discrepancy(Jn) <= prm.disc_target:
                reason, J = REASON_DISCREPANCY, Jn
                break
            if (prm.stop & STOP_CONV) and converged(Jn, J, prm.tol):
                reason, J = REASON_CONV, Jn
                break
            J = Jn
        return f, dict(iters=k, kl=J, history=hist, reason=reason)

    # --------------------------------------------------------------- SGP
    def scaling(self, f, L1, L2):
        """Eqs. (Dk), (Dkbound): D = (M_R / alpha) o min[L2, max{L1, f}]."""
        return self.invw * np.minimum(L2, np.maximum(L1, f))

    def bb_sums(self, f, f_new, G, G_new, L1, L2):
        """The four sums of Eqs. (BB1), (BB2) after the step f -> f_new:
        s = f_new - f, z = grad(f_new) - grad(f), D the scaling of the new
        iterate, over the pixels with D > 0.  Returns
        (s'D^-1 D^-1 s, s'D^-1 z, s'D z, z'D D z)."""
        s = f_new - f
        z = G_new - G
        Dn = self.scaling(f_new, L1, L2)
        m = Dn > 0
        sm, zm, Dm = s[m], z[m], Dn[m]
        a_num = float(np.sum(sm * sm / (Dm * Dm)))
        c1 = float(np.sum(sm * zm / Dm))
        c2 = float(np.sum(sm * zm * Dm))
        e_den = float(np.sum(zm * zm * Dm * Dm))
        return a_num, c1, c2, e_den

    def flux_value(self, prm: Params):
        if prm.flux >= 0:
            return prm.flux
        return np.mean([(self.g[j] - self.b[j]).sum() for j in range(self.p)])

    def project(self, z, D, prm: Params, c=None):
        """P_+ of Algorithm 1 step 2 (orthant), or, with the flux constraint,
        the D^{-1}-metric projection onto {x >= 0, sum x = c}."""
        if not prm.flux_constraint:
            return np.maximum(0.0, z)
        return flux_projection(z, D, c)

    def sgp(self, f0, params: Params | None = None, force_alpha=None,
            force_lambda=None, bounds=None, grad0=None):
        """Algorithm 1 with the Sect. 2.1 steplength rules and Sect. 3 policies.

        ``force_alpha`` / ``force_lambda`` pin alpha_k / lambda_k (tests only:
        the RL identity of Eq. (RL2) with lambda = 1).  ``bounds`` and
        ``grad0`` supply (L1, L2) and the gradient at f0 instead of computing
        them (tests only: one iteration re-run from another implementation's
        state).
        Returns (f, info) where info carries the per-iteration decision log."""
        prm = params or Params()
        c = self.flux_value(prm) if prm.flux_constraint else None
        f = f0.copy()
        if prm.flux_constraint:
            # the start is put on the constraint set {f >= 0, sum f = c}
            tot = f.sum()
            if tot > 0:
                f *= c / tot
        # Sect. 3.2: the bounds come from one RL step from the starting
        # point, the start on the constraint set when the flux is constrained
        if bounds is not None:
            L1, L2 = bounds
        elif prm.auto_bounds:
            L1, L2 = self.bounds(f)
        else:
            L1, L2 = prm.L1, prm.L2
        J = self.kl(f)
        G = self.grad(f)
        # a supplied gradient is carried as a sum of changes: each step adds
        # the exact change grad J(f_new) - grad J(f), which is also the z of
        # Eqs. (BB1), (BB2)
        Gx = None
        if grad0 is not None:
            Gx, G = G, np.asarray(grad0, dtype=np.float64).copy()
        alpha = prm.alpha0
        tau = prm.tau1
        Q: list[float] = []
        log = []
        hist = [J]
        reason = REASON_MAXITER
        k = 0
        if (prm.stop & STOP_DISCREPANCY) and self.discrepancy(J) <= prm.disc_target:
            return f, dict(iters=0, kl=J, history=hist, log=log, L1=L1, L2=L2,
                           reason=REASON_DISCREPANCY, alpha=alpha)
        rho = rel_error(f, prm.f_true) if rmse_active(prm) else None
        while k < prm.max_iter:
            if force_alpha is not None:
                alpha = force_alpha
            # steps 1-3: scaling, projection, direction
            D = self.scaling(f, L1, L2)
            yk = self.project(f - alpha * D * G, D, prm, c)
            d = yk - f
            gd = float(np.sum(G * d))
            if gd == 0.0:
                reason = REASON_STATIONARY
                break
            # steps 4-5: monotone Armijo backtracking
            lam = 1.0
            nback = 0
            armijo_ok = True
            if force_lambda is not None:
                lam = force_lambda
                f_new = f + lam * d
                J_new = self.kl(f_new)
            else:
                while True:
                    f_new = f + lam * d
                    J_new = self.kl(f_new)
                    if J_new <= J + prm.beta * lam * gd:
                        break
                    if nback >= prm.max_backtracks:
                        armijo_ok = False
                        break
                    lam *= prm.theta
                    nback += 1
            if not armijo_ok:
                reason = REASON_ARMIJO
                break
            # step 6: update
            G_new = self.grad(f_new)
            if Gx is not None:
                Gx, G_new = G_new, G + (G_new - Gx)
            a_num, c1, c2, e_den = self.bb_sums(f, f_new, G, G_new, L1, L2)
            a1, a2, br1, br2, alpha_next, tau, Q, alt = steplength_update(
                alpha, tau, Q, k, a_num, c1, c2, e_den, prm)
            log.append(dict(k=k, alpha=alpha, gd=gd, backtracks=nback, lam=lam,
                            J=J_new, a=a_num, c1=c1, c2=c2, e=e_den,
                            a1=a1, a2=a2, br1=br1, br2=br2, alt=alt, tau=tau,
                            alpha_next=alpha_next))
            J_prev, f_prev = J, f
            f, J, G, alpha = f_new, J_new, G_new, alpha_next
            k += 1
            hist.append(J)
            if (prm.stop & STOP_DISCREPANCY) and self.discrepancy(J) <= prm.disc_target:
                reason = REASON_DISCREPANCY
                break
            if (prm.stop & STOP_CONV) and converged(J, J_prev, prm.tol):
                reason = REASON_CONV
                break
            if rho is not None:
                # Sect. 3.3: stop when the reconstruction error has reached
                # its minimum, i.e. at its first increase, and return the
                # iterate of the minimum (the one before the step just taken)
                rho_new = rel_error(f, prm.f_true)
                if rho_new > rho:
                    reason = REASON_RMSE
                    f, J, k = f_prev, J_prev, k - 1
                    hist.pop()
                    log.pop()
                    break
                rho = rho_new
        return f, dict(iters=k, kl=J, history=hist, log=log, L1=L1, L2=L2,
                       reason=reason, alpha=alpha)


def converged(J_new, J_old, tol):
    """Eq. (convergence): |J(f^(k+1)) - J(f^(k))| <= tol J(f^(k))."""
    return abs(J_new - J_old) <= tol * J_old


def rel_error(f, f_true):
    """Sect. 3.3: relative reconstruction error rho = ||f - f~||_2 / ||f~||_2."""
    ft = np.asarray(f_true, dtype=np.float64)
    return float(np.linalg.norm(f - ft) / np.linalg.norm(ft))


def rmse_active(prm):
    """The reconstruction-error stop is on (it needs the true object)."""
    return bool(prm.stop & STOP_RMSE) and prm.f_true is not None


def steplength_update(alpha, tau, Q, k, a_num, c1, c2, e_den, prm: Params):
    """Sect. 2.1 steplength rule after iteration k (producing alpha_{k+1}).

    a_num = s^T D^-1 D^-1 s, c1 = s^T D^-1 z (Eq. BB1);
    c2 = s^T D z, e_den = z^T D D z (Eq. BB2).
    Safeguards: a non-positive denominator gives min{10 alpha, alpha_max},
    otherwise the BB value is clamped to [alpha_min, alpha_max].
    Eq. (alphadef): the memory Q keeps the last M_alpha values of alpha^(2);
    the first ``n_bb2_only`` steplengths take min Q, later ones alternate on
    alpha^(2)/alpha^(1) <= tau (tau <- 0.9 tau) else alpha^(1) (tau <- 1.1 tau).
    Returns (a1, a2, br1, br2, alpha_next, tau, Q, alt)."""
    if c1 <= 0:
        a1, br1 = min(10.0 * alpha, prm.alpha_max), 0
    else:
        a1, br1 = min(prm.alpha_max, max(prm.alpha_min, a_num / c1)), 1
    if c2 <= 0:
        a2, br2 = min(10.0 * alpha, prm.alpha_max), 0
    else:
        a2, br2 = min(prm.alpha_max, max(prm.alpha_min, c2 / e_den)), 1
    Q = (list(Q) + [a2])[-prm.m_alpha:]
    if k + 1 <= prm.n_bb2_only:
        return a1, a2, br1, br2, min(Q), tau, Q, 0
    if a2 / a1 <= tau:
        return a1, a2, br1, br2, min(Q), 0.9 * tau, Q, 1
    return a1, a2, br1, br2, a1, 1.1 * tau, Q, 2


def flux_projection(z, D, c):
    """argmin_{x >= 0, sum x = c} (x - z)^T D^{-1} (x - z).

    KKT: x_i = max(0, z_i - mu D_i) for one multiplier mu, where
    phi(mu) = sum_i max(0, z_i - mu D_i) - c = 0.  phi is piecewise linear and
    non-increasing with breakpoints t_i = z_i / D_i; the oracle sorts them and
    scans the pieces (brute force).  Pixels with D_i = 0 are held at
    max(0, z_i)."""
    z = np.asarray(z, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    act = D > 0
    zf, Df = z[act], D[act]
    fixed = np.maximum(0.0, z[~act]).sum()
    target = c - fixed
    t = zf / Df
    order = np.argsort(-t)          # descending breakpoints
    ts, zs, Ds = t[order], zf[order], Df[order]
    # with mu in [ts[i], ts[i-1]] the active set is the first i entries
    Sz = np.cumsum(zs)
    SD = np.cumsum(Ds)
    mu = None
    for i in range(1, ts.size + 1):
        m = (Sz[i - 1] - target) / SD[i - 1]
        lo = ts[i] if i < ts.size else -np.inf
        hi = ts[i - 1]
        if lo <= m <= hi:
            mu = m
            break
    if mu is None:
        raise ValueError("flux projection: no root (c must be positive)")
    x = np.maximum(0.0, z) * (~act)
    x[act] = np.maximum(0.0, zf - mu * Df)
    return x


# ------------------------------------------------------------------ mosaic
def mosaic_tiles(H, W, core, margin, N):
    """Subdomains of an H x W image: core tiles of core x core, each observed
    through a window extended by margin pixels towards its neighbours (clipped
    at the image edge) and placed at the centre of an N x N FFT domain.
    Returns [(core rows, core cols, window rows, window cols, (oy, ox))]."""
    tiles = []
    for i in range(H // core):
        for j in range(W // core):
            y0, y1 = max(0, i * core - margin), min(H, (i + 1) * core + margin)
            x0, x1 = max(0, j * core - margin), min(W, (j + 1) * core + margin)
            oy, ox = (N - (y1 - y0)) // 2, (N - (x1 - x0)) // 2
            tiles.append(((i * core, (i + 1) * core), (j * core, (j + 1) * core), (y0, y1), (x0, x1), (oy, ox)))
    return tiles


def mosaic(g, psf_N, b, core, margin, method="sgp", n_iter=100, params: Params | None = None):
    """Each window reconstructed as a boundary-corrected problem (Sect. 2.4) on
    the N x N domain of psf_N, then the cores stitched into an H x W image.
    method: "sgp" or "rl".  Returns (mosaic, list of per-tile info)."""
    g = np.asarray(g, dtype=np.float64)
    H, W = g.shape
    N = psf_N.shape[-1]
    out = np.zeros((H, W))
    infos = []
    for (cy, cx, wy, wx, (oy, ox)) in mosaic_tiles(H, W, core, margin, N):
        gw = g[wy[0]:wy[1], wx[0]:wx[1]]
        P = Problem(gw, psf_N, b, domain=(N, N, oy, ox))
        f0 = P.start("flat")
        if method == "rl":
            f, info = P.rl(f0, n_iter, params)
        else:
            f, info = P.sgp(f0, params or Params(max_iter=n_iter))
        ry, rx = oy + cy[0] - wy[0], ox + cx[0] - wx[0]
        out[cy[0]:cy[1], cx[0]:cx[1]] = f[ry:ry + core, rx:rx + core]
        infos.append(info)
    return out, infos
