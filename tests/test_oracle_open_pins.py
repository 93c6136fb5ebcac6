"""Pins of oracle parts that the first set of pins left open, each checked
against something other than the oracle's own formula, and each shown to
catch a plausible local mistake (the mistake is planted in the oracle, on
the CPU, by monkeypatching; the pin must then fail):

* the Barzilai-Borwein sums of Eqs. (BB1), (BB2): by their least-squares
  property, alpha1 = argmin ||(alpha D)^-1 s - z||, alpha2 =
  argmin ||s - alpha D z||, minimised numerically over alpha, with s, z and
  D of the new iterate built from two oracle iterates (reading: D is the
  scaling of the new iterate);
* Eq. (convergence): stop index and returned iterate of RL, OSEM and SGP
  against the history of an independent fixed-count run;
* the flat start of Sect. 3.1 for several images (mean over the images) and
  for a boundary problem (on R, divided by |S|), by hand;
* the bounds of Sect. 3.2 on a boundary problem (extrema over the observed
  window S), against a direct evaluation of the RL step;
* Eq. (discrepancy) with p = 3 images, against the separable closed form of a
  delta-PSF problem, and the discrepancy stop against a run's history."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import sgp as O
from synth import workloads as W


# ------------------------------------------------------------ BB sums
def pin_bb_sums():
    w = W.small_single(64, 80)
    P = O.Problem(w.g, w.psf, w.b)
    f0 = P.start("flat")
    L1, L2 = P.bounds(f0)
    for k in (0, 3, 5):
        fk, _ = P.sgp(f0, O.Params(max_iter=k))
        fk1, io = P.sgp(f0, O.Params(max_iter=k + 1))
        L = io["log"][k]
        assert L["br1"] == 1 and L["br2"] == 1      # both ratios are positive here
        s = fk1 - fk
        z = P.grad(fk1) - P.grad(fk)
        Dp = P.invw * np.clip(fk1, L1, L2)           # Eq. (Dk) at the new iterate
        msk = Dp > 0
        s, z, Dp = s[msk], z[msk], Dp[msk]
        r1 = minimize_scalar(lambda t: np.sum((s / (np.exp(t) * Dp) - z) ** 2),
                             bounds=(-20, 20), method="bounded", options={"xatol": 1e-12})
        r2 = minimize_scalar(lambda t: np.sum((s - np.exp(t) * Dp * z) ** 2),
                             bounds=(-20, 20), method="bounded", options={"xatol": 1e-12})
        a1_ls, a2_ls = np.exp(r1.x), np.exp(r2.x)
        assert abs(L["a"] / L["c1"] - a1_ls) <= 1e-6 * a1_ls, (k, L["a"] / L["c1"], a1_ls)
        assert abs(L["c2"] / L["e"] - a2_ls) <= 1e-6 * a2_ls, (k, L["c2"] / L["e"], a2_ls)


def _bb_swapped(self, f, f_new, G, G_new, L1, L2):      # D and D^-1 exchanged
    s, z, D = f_new - f, G_new - G, self.scaling(f_new, L1, L2)
    m = D > 0
    s, z, D = s[m], z[m], D[m]
    return float(np.sum(s * s * D * D)), float(np.sum(s * z * D)), float(np.sum(s * z / D)), float(np.sum(z * z / D / D))


def _bb_old_D(self, f, f_new, G, G_new, L1, L2):        # D of the old iterate
    s, z, D = f_new - f, G_new - G, self.scaling(f, L1, L2)
    m = D > 0
    s, z, D = s[m], z[m], D[m]
    return float(np.sum(s * s / D / D)), float(np.sum(s * z / D)), float(np.sum(s * z * D)), float(np.sum(z * z * D * D))


def _bb_one_power(self, f, f_new, G, G_new, L1, L2):    # a dropped power of D
    s, z, D = f_new - f, G_new - G, self.scaling(f_new, L1, L2)
    m = D > 0
    s, z, D = s[m], z[m], D[m]
    return float(np.sum(s * s / D)), float(np.sum(s * z / D)), float(np.sum(s * z * D)), float(np.sum(z * z * D))


def _bb_sign(self, f, f_new, G, G_new, L1, L2):         # s taken backwards
    s, z, D = f - f_new, G_new - G, self.scaling(f_new, L1, L2)
    m = D > 0
    s, z, D = s[m], z[m], D[m]
    return float(np.sum(s * s / D / D)), float(np.sum(s * z / D)), float(np.sum(s * z * D)), float(np.sum(z * z * D * D))


# ---------------------------------------------------- convergence stop
def _first_conv_index(hist, tol):
    for k in range(1, len(hist)):
        if abs(hist[k] - hist[k - 1]) <= tol * hist[k - 1]:
            return k
    return None


def pin_convergence():
    w1 = W.small_single(64, 80)
    w3 = W.small_multi(64, 64)
    for name, w, tol, nmax in (("rl", w1, 1e-3, 400), ("osem", w3, 1e-3, 200), ("sgp", w1, 1e-2, 100)):
        P = O.Problem(w.g, w.psf, w.b)
        f0 = P.start("flat")

        def run(n, stop):
            prm = O.Params(max_iter=n, stop=stop, tol=tol)
            if name == "rl":
                return P.rl(f0, n, prm)
            if name == "osem":
                return P.osem(f0, n, prm)
            return P.sgp(f0, prm)
        _, ref = run(nmax, O.STOP_FIXED)
        k = _first_conv_index(ref["history"], tol)
        assert k is not None and 1 < k < nmax, (name, k)
        fc, ic = run(nmax, O.STOP_CONV)
        assert ic["reason"] == O.REASON_CONV and ic["iters"] == k, (name, ic["iters"], k)
        fk, ik = run(k, O.STOP_FIXED)
        assert np.array_equal(fc, fk), name                    # the iterate that met the rule
        assert ic["kl"] == ref["history"][k] == ik["kl"], name


def _conv_no_abs(J_new, J_old, tol):
    return (J_new - J_old) <= tol * J_old


def _conv_reversed(J_new, J_old, tol):
    return abs(J_new - J_old) >= tol * J_old


class _ConvLate:
    """Answers each test with the previous test's outcome: the run stops one
    iteration after the rule was met."""
    def __init__(self):
        self.prev = False

    def __call__(self, J_new, J_old, tol):
        out, self.prev = self.prev, abs(J_new - J_old) <= tol * J_old
        return out


# ----------------------------------------------------------- starts
def pin_multi_flat_start():
    ny = nx = 8
    g = np.stack([np.full((ny, nx), 3.0), np.full((ny, nx), 5.0), np.full((ny, nx), 10.0)])
    psf = np.zeros((3, ny, nx))
    psf[:, ny // 2, nx // 2] = 1.0
    P = O.Problem(g, psf, np.array([1.0, 1.0, 2.0]))
    # mean over the images of the background-subtracted flux, per pixel:
    # ((3-1) + (5-1) + (10-2)) / 3 = 14/3
    assert np.allclose(P.start("flat"), 14.0 / 3.0, rtol=1e-15, atol=0)


def _boundary_box():
    """12x12 domain, 8x8 window at (2, 2), a 3x3 PSF (1 2 1)^T (1 2 1) / 16:
    alpha = K correlated with M_S is >= 1/16 on the window dilated by one
    pixel (rows and columns 1..10) and 0 elsewhere, so R is that 10x10 square."""
    NY = NX = 12
    psf = np.zeros((NY, NX))
    k1 = np.array([1.0, 2.0, 1.0]) / 4.0
    psf[5:8, 5:8] = np.outer(k1, k1)
    rng = np.random.default_rng(3)
    g = rng.poisson(50.0, (8, 8)).astype(np.float64)
    g[0, 0] = 10000.0            # a bright pixel in the window's corner
    return g, psf, 5.0, (NY, NX, 2, 2)


def pin_boundary_flat_start():
    g, psf, b, dom = _boundary_box()
    P = O.Problem(g, psf, b, domain=dom)
    R = np.zeros((12, 12), bool)
    R[1:11, 1:11] = True
    assert np.array_equal(P.MR > 0, R)
    c = (g - b).sum() / 64.0                  # divided by |S| = 64, not by |R| = 100
    f0 = P.start("flat")
    assert np.allclose(f0[R], c, rtol=1e-15, atol=0) and np.all(f0[~R] == 0.0)


def _rl_step_direct(g, psf, b, dom, f0):
    """One boundary RL step, Eq. (boundaryRL), by explicit sums over the 3x3
    PSF support (no transforms)."""
    NY, NX, oy, ox = dom
    ny, nx = g.shape
    ky, kx = np.nonzero(psf)
    S = np.zeros((NY, NX), bool)
    S[oy:oy + ny, ox:ox + nx] = True
    cy, cx = NY // 2, NX // 2
    alpha = np.zeros((NY, NX))
    for n_y in range(NY):
        for n_x in range(NX):
            for a, c in zip(ky, kx):
                m_y, m_x = n_y + (a - cy), n_x + (c - cx)
                if 0 <= m_y < NY and 0 <= m_x < NX and S[m_y, m_x]:
                    alpha[n_y, n_x] += psf[a, c]
    R = alpha >= 1e-3
    Af = np.zeros((NY, NX))
    for m_y in range(NY):
        for m_x in range(NX):
            for a, c in zip(ky, kx):
                n_y, n_x = m_y - (a - cy), m_x - (c - cx)
                if 0 <= n_y < NY and 0 <= n_x < NX and R[n_y, n_x]:
                    Af[m_y, m_x] += psf[a, c] * f0[n_y, n_x]
    ratio = np.zeros((NY, NX))
    ratio[S] = g.ravel() / (Af[S] + b)
    back = np.zeros((NY, NX))
    for n_y in range(NY):
        for n_x in range(NX):
            if not R[n_y, n_x]:
                continue
            for a, c in zip(ky, kx):
                m_y, m_x = n_y + (a - cy), n_x + (c - cx)
                if 0 <= m_y < NY and 0 <= m_x < NX:
                    back[n_y, n_x] += psf[a, c] * ratio[m_y, m_x]
    y = np.where(R, f0 * back / np.where(R, alpha, 1.0), 0.0)
    return y, S


def pin_boundary_bounds():
    g, psf, b, dom = _boundary_box()
    P = O.Problem(g, psf, b, domain=dom)
    f0 = P.start("flat")
    y, S = _rl_step_direct(g, psf, b, dom, f0)
    vals = y[S & (y > 0)]
    lo, hi = vals.min(), vals.max()
    exp = (lo / 10, hi * 10) if hi / lo < 50 else (lo, hi)
    L1, L2 = P.bounds(f0)
    assert np.allclose((L1, L2), exp, rtol=1e-12, atol=0), ((L1, L2), exp)
    # the bright corner makes the extrema over R differ from those over S
    assert y.max() > 1.5 * hi


def _start_sum_over_images(self, kind="flat", user=None):
    c = np.sum([(self.g[j] - self.b[j]).sum() for j in range(self.p)]) / self.nS
    return c * self.MR


def _start_over_R(self, kind="flat", user=None):
    c = np.mean([(self.g[j] - self.b[j]).sum() for j in range(self.p)]) / self.MR.sum()
    return c * self.MR


def _start_everywhere(self, kind="flat", user=None):
    c = np.mean([(self.g[j] - self.b[j]).sum() for j in range(self.p)]) / self.nS
    return c * np.ones((self.NY, self.NX))


def _bounds_over_R(self, f0):
    yr = self.rl_step(f0)
    pos = yr[yr > 0]
    ymin, ymax = pos.min(), pos.max()
    return (ymin / 10.0, ymax * 10.0) if ymax / ymin < 50 else (ymin, ymax)


# ------------------------------------------------------ discrepancy, p = 3
def pin_discrepancy_three_images():
    ny, nx = 8, 10
    rng = np.random.default_rng(11)
    f = rng.uniform(5.0, 50.0, (ny, nx))
    bs = np.array([2.0, 3.0, 4.0])
    g = np.stack([rng.poisson(f + bj).astype(np.float64) for bj in bs])
    g[0, 0, 0] = 0.0
    psf = np.zeros((3, ny, nx))
    psf[:, ny // 2, nx // 2] = 1.0                 # A_j = identity: J separable
    P = O.Problem(g, psf, bs)
    J = 0.0
    for j in range(3):
        y = f + bs[j]
        t = y - g[j]
        pos = g[j] > 0
        t[pos] += g[j][pos] * np.log(g[j][pos] / y[pos])
        J += t.sum()
    assert abs(P.kl(f) - J) <= 1e-12 * J
    assert abs(P.discrepancy(J) - 2.0 * J / (3 * ny * nx)) <= 1e-15 * J
    # the stop of a three-image SGP run at the first k with 2 J_k / (3 |S|) <= 1
    w = W.small_multi(64, 64)
    Pm = O.Problem(w.g, w.psf, w.b)
    f0 = Pm.start("flat")
    _, ref = Pm.sgp(f0, O.Params(max_iter=60))
    D = 2.0 * np.array(ref["history"]) / (3 * 64 * 64)
    k = int(np.argmax(D <= 1.0))
    assert D[k] <= 1.0 and k > 0 and np.all(D[:k] > 1.0)
    _, io = Pm.sgp(f0, O.Params(max_iter=60, stop=O.STOP_DISCREPANCY))
    assert io["iters"] == k and io["reason"] == O.REASON_DISCREPANCY


def _disc_one_image(self, J):
    return 2.0 * J / self.nS


PINS = {"bb_sums": pin_bb_sums, "convergence": pin_convergence, "multi_flat_start": pin_multi_flat_start,
        "boundary_flat_start": pin_boundary_flat_start, "boundary_bounds": pin_boundary_bounds,
        "discrepancy_three_images": pin_discrepancy_three_images}


@pytest.mark.parametrize("name", list(PINS))
def test_pin(name):
    PINS[name]()


# (pin, attribute of the oracle replaced, mutant)
MUTANTS = [
    ("bb_sums", (O.Problem, "bb_sums"), _bb_swapped),
    ("bb_sums", (O.Problem, "bb_sums"), _bb_old_D),
    ("bb_sums", (O.Problem, "bb_sums"), _bb_one_power),
    ("bb_sums", (O.Problem, "bb_sums"), _bb_sign),
    ("convergence", (O, "converged"), _conv_no_abs),
    ("convergence", (O, "converged"), _conv_reversed),
    ("convergence", (O, "converged"), "late"),
    ("multi_flat_start", (O.Problem, "start"), _start_sum_over_images),
    ("boundary_flat_start", (O.Problem, "start"), _start_over_R),
    ("boundary_flat_start", (O.Problem, "start"), _start_everywhere),
    ("boundary_bounds", (O.Problem, "bounds"), _bounds_over_R),
    ("discrepancy_three_images", (O.Problem, "discrepancy"), _disc_one_image),
]


@pytest.mark.parametrize("pin,target,mutant", MUTANTS,
                         ids=[f"{p}-{m if isinstance(m, str) else m.__name__}" for p, _, m in MUTANTS])
def test_pin_catches_mutant(monkeypatch, pin, target, mutant):
    owner, attr = target
    if mutant == "late":
        mutant = _ConvLate()
    monkeypatch.setattr(owner, attr, mutant)
    with pytest.raises(AssertionError):
        PINS[pin]()
