// Scalar control of the solvers, run on device by the thread that finalises a
// reduction.  Each function follows one step of the method:
//   fin_dir      Algorithm 1, steps 2-3: grad^T d and the stationarity test
//   fin_armijo   Algorithm 1, steps 4-5: first lambda = theta^m passing
//                J(f + lambda d) <= J(f) + beta lambda grad^T d
//   fin_update   Algorithm 1, step 6 and the stopping rules of Sect. 3.3
//   fin_bb       Sect. 2.1: Eqs. (BB1), (BB2), safeguards and Eq. (alphadef)
//   fin_bounds   Sect. 3.2: (L1, L2) from one RL step
//   fin_rl       Eq. (RL): stopping rules evaluated on J(f^(k))
#pragma once
#include "common.hpp"

namespace sgp {

__host__ __device__ inline double* trace_row(DevState* st, int k) {
  if (!st->trace_on || !st->trace || k < 0 || k > st->max_iter) return nullptr;
  return st->trace + (size_t)k * kTraceCols;
}

__host__ __device__ inline void fin_dir(DevState* st, double gd) {
  st->gd = gd;
  double* tr = trace_row(st, st->k);
  if (tr) {
    tr[TR_K] = st->k;
    tr[TR_ALPHA] = st->alpha;
    tr[TR_GD] = gd;
    tr[TR_FLUXMU] = st->mu;
  }
  if (!__builtin_isfinite(gd)) {
    st->done = 1;
    st->reason = REASON_NUMERIC;
  } else if (gd == 0.0) {
    st->done = 1;
    st->reason = REASON_STATIONARY;
  }
}

// dJ[m] = J(f + theta^(m0+m) d) - J(f) for m = 0..n-1.
__host__ __device__ inline void fin_armijo(DevState* st, const double* dJ, int m0, int n) {
  st->need_more = 0;
  st->spec_ok = 0;
  for (int m = 0; m < n; ++m) {
    const int mm = m0 + m;
    if (mm > st->max_backtracks) break;
    const double lam = st->lam_tab[mm];
    // (+infinity: a candidate outside the domain of J, which fails the test)
    if (__builtin_isnan(dJ[m])) {
      st->done = 1;
      st->reason = REASON_NUMERIC;
      return;
    }
    // (the linear relaxation of RL takes its last candidate, lambda = 1,
    // the RL step, without the test)
    if (dJ[m] <= st->beta * lam * st->gd || (st->rl2 && mm == st->max_backtracks)) {
      st->lam = lam;
      st->nback = mm;
      st->f_pending = 1;
      st->spec_ok = mm == 0;  // lambda = theta^0 = 1: the A d pass already made this update
      return;
    }
  }
  if (m0 + n <= st->max_backtracks) {
    st->need_more = 1;
  } else {
    st->done = 1;
    st->reason = REASON_ARMIJO;
  }
}

// Whether fin_armijo(st, dJ, m0, n) would ask for further candidates, without
// touching the state (every workgroup of the Armijo kernel takes the test).
__host__ __device__ inline bool armijo_needs_more(const DevState* st, const double* dJ, int m0, int n) {
  for (int m = 0; m < n; ++m) {
    const int mm = m0 + m;
    if (mm > st->max_backtracks) break;
    if (__builtin_isnan(dJ[m])) return false;
    if (dJ[m] <= st->beta * st->lam_tab[mm] * st->gd) return false;
    if (st->rl2 && mm == st->max_backtracks) return false;
  }
  return m0 + n <= st->max_backtracks;
}

__host__ __device__ inline void fin_update(DevState* st, double Jn) {
  const int k = st->k;
  double* tr = trace_row(st, k);
  if (tr) {
    tr[TR_BACK] = st->nback;
    tr[TR_LAM] = st->lam;
    tr[TR_J] = Jn;
  }
  st->Jprev = st->J;
  st->J = Jn;
  st->k = k + 1;
  st->total_back += st->nback;
  if (!__builtin_isfinite(Jn)) {
    st->done = 1;
    st->reason = REASON_NUMERIC;
  } else if ((st->stop & STOP_DISCREPANCY) && st->norm_disc * Jn <= st->disc_target) {
    st->done = 1;
    st->reason = REASON_DISCREPANCY;
  } else if ((st->stop & STOP_CONV) && fabs(Jn - st->Jprev) <= st->tol * st->Jprev) {
    st->done = 1;
    st->reason = REASON_CONV;
  } else if (st->k >= st->max_iter && !(st->stop & STOP_RMSE)) {
    // (with the reconstruction-error stop the last iterate is tested first:
    // fin_rmse ends the run)
    st->done = 1;
    st->reason = REASON_MAXITER;
  }
}

struct BBInfo {
  double a1, a2, next;
  int br1, br2, alt;
};

// Steplength rule after a completed iteration (st->k iterations done).
// a = s'D^-2 s, c1 = s'D^-1 z, c2 = s'D z, e = z'D^2 z.  Updates tau and the
// memory Q; returns alpha^(1), alpha^(2), the next steplength and branches.
__host__ __device__ inline BBInfo bb_rule(DevState* st, double a, double c1, double c2, double e) {
  const double alpha = st->alpha;
  BBInfo r;
  if (c1 <= 0) { r.a1 = fmin(10.0 * alpha, st->alpha_max); r.br1 = 0; }
  else { r.a1 = fmin(st->alpha_max, fmax(st->alpha_min, a / c1)); r.br1 = 1; }
  if (c2 <= 0) { r.a2 = fmin(10.0 * alpha, st->alpha_max); r.br2 = 0; }
  else { r.a2 = fmin(st->alpha_max, fmax(st->alpha_min, c2 / e)); r.br2 = 1; }
  // memory of the last m_alpha values of alpha^(2)
  if (st->nQ < st->m_alpha) {
    st->Q[st->nQ++] = r.a2;
  } else {
    for (int i = 1; i < st->m_alpha; ++i) st->Q[i - 1] = st->Q[i];
    st->Q[st->m_alpha - 1] = r.a2;
  }
  double qmin = st->Q[0];
  for (int i = 1; i < st->nQ; ++i) qmin = fmin(qmin, st->Q[i]);
  const int kdone = st->k;  // iterations completed, i.e. k + 1 of the step just taken
  if (kdone <= st->n_bb2_only) { r.next = qmin; r.alt = 0; }
  else if (r.a2 / r.a1 <= st->tau) { r.next = qmin; st->tau *= 0.9; r.alt = 1; }
  else { r.next = r.a1; st->tau *= 1.1; r.alt = 2; }
  return r;
}

__host__ __device__ inline void fin_bb(DevState* st, double a, double c1, double c2, double e) {
  if (st->rl2) {  // Eq. (RL2): the RL direction, no steplength rule
    st->alpha = 1.0;
    if (st->k >= st->k_stop) st->pause = 1;
    return;
  }
  const BBInfo r = bb_rule(st, a, c1, c2, e);
  double* tr = trace_row(st, st->k - 1);
  if (tr) {
    tr[TR_A] = a; tr[TR_C1] = c1; tr[TR_C2] = c2; tr[TR_E] = e;
    tr[TR_A1] = r.a1; tr[TR_A2] = r.a2; tr[TR_BR1] = r.br1; tr[TR_BR2] = r.br2;
    tr[TR_ALT] = r.alt; tr[TR_TAU] = st->tau; tr[TR_ALPHA_NEXT] = r.next;
  }
  if (!__builtin_isfinite(r.next)) {
    st->done = 1;
    st->reason = REASON_NUMERIC;
  }
  st->alpha = r.next;
  if (st->k >= st->k_stop) st->pause = 1;
}

__host__ __device__ inline void fin_bounds(DevState* st, double ymin, double ymax) {
  st->ymin = ymin;
  st->ymax = ymax;
  if (st->auto_bounds) {
    if (ymax / ymin < 50.0) { st->L1 = ymin / 10.0; st->L2 = ymax * 10.0; }
    else { st->L1 = ymin; st->L2 = ymax; }
  } else {
    st->L1 = st->L1p;
    st->L2 = st->L2p;
  }
  st->alpha = st->alpha0;
  st->tau = st->tau1;
  st->nQ = 0;
  st->k = 0;
  st->total_back = 0;
  st->nback = 0;
  st->lam = 1.0;
  double lam = 1.0;
  for (int m = 0; m < kMaxCand; ++m) {  // the backtracking sequence lambda <- theta lambda
    st->lam_tab[m] = lam;
    lam *= st->theta;
  }
  if (!__builtin_isfinite(st->J)) {
    st->done = 1;
    st->reason = REASON_NUMERIC;
  } else if ((st->stop & STOP_DISCREPANCY) && st->norm_disc * st->J <= st->disc_target) {
    st->done = 1;
    st->reason = REASON_DISCREPANCY;
  } else if (st->max_iter <= 0) {
    st->done = 1;
    st->reason = REASON_MAXITER;
  }
}

// RL: J(f^(k)) has just been formed; decide whether f^(k) is returned, or
// whether a stepping call pauses before the next update (J is then not
// committed, so the resumed call re-forms it with the same previous value).
__host__ __device__ inline void fin_rl(DevState* st, double J) {
  const int k = st->k;
  double* tr = trace_row(st, k);
  if (tr) {
    tr[TR_K] = k;
    tr[TR_J] = J;
  }
  const double Jprev = st->J;
  if (!__builtin_isfinite(J)) {
    st->done = 1;
    st->reason = REASON_NUMERIC;
  } else if ((st->stop & STOP_DISCREPANCY) && st->norm_disc * J <= st->disc_target) {
    st->done = 1;
    st->reason = REASON_DISCREPANCY;
  } else if ((st->stop & STOP_CONV) && k > 0 && fabs(J - Jprev) <= st->tol * Jprev) {
    st->done = 1;
    st->reason = REASON_CONV;
  } else if (k >= st->max_iter) {
    st->done = 1;
    st->reason = REASON_MAXITER;
  } else if (k >= st->k_stop) {
    st->pause = 1;
    return;
  } else {
    st->k = k + 1;
  }
  st->Jprev = Jprev;
  st->J = J;
}

// Sect. 3.3, reconstruction error: t = {sum (f - f~)^2, sum f~^2} of the
// iterate just formed.  At setup (first) rho^(0) is recorded.  Afterwards an
// increase over the previous value ends the run, and the previous iterate
// (kept by PIX_FCOPY) is returned: its iteration count is one less, and its
// KL is the one held before the step (SGP: Jprev; RL / OSEM have not yet
// formed the KL of the new iterate, so J already belongs to the previous).
__host__ __device__ inline void fin_rmse(DevState* st, const double* t, bool first, bool sgp) {
  const double rho = t[1] > 0.0 ? sqrt(t[0] / t[1]) : sqrt(t[0]);
  st->rms_k = st->k;
  if (first) {
    st->rms_prev = rho;
    return;
  }
  if (!__builtin_isfinite(rho)) {
    st->done = 1;
    st->reason = REASON_NUMERIC;
  } else if (rho > st->rms_prev) {
    st->done = 1;
    st->reason = REASON_RMSE;
    st->rms_back = 1;
    st->k -= 1;
    if (sgp) st->J = st->Jprev;
  } else {
    st->rms_prev = rho;
    if (sgp && st->k >= st->max_iter) {  // the cap, deferred by fin_update
      st->done = 1;
      st->reason = REASON_MAXITER;
    }
  }
}

// Eq. (RL2) line search: t = min over d_i < 0 of f_i / (-d_i), the largest
// step keeping f + lam d >= 0 (infinite when no d_i < 0).  Candidates
// lam_max = min(t, cap), theta lam_max, ... while above 1, then 1; the
// Armijo test runs over them in that order (max_backtracks = index of the
// final 1, which fin_armijo accepts without the test).
__host__ __device__ inline void fin_rl2max(DevState* st, double t) {
  st->lam_bound = t;
  double lam = fmin(st->lam_cap, t);
  int m = 0;
  while (lam > 1.0 && m < kMaxCand - 1) {
    st->lam_tab[m++] = lam;
    lam *= st->theta;
  }
  st->lam_tab[m] = 1.0;
  if (m + 1 < kMaxCand) st->lam_tab[m + 1] = st->theta;  // read by the A d pass, never used
  st->max_backtracks = m;
}

// Flux projection (constraint set {x >= 0, sum x = c} of Sect. 2, projection
// in the D^-1 metric): x_i = max(0, z_i - mu D_i), with mu the root of the
// convex, decreasing, piecewise linear phi(mu) = sum_i max(0, z_i - mu D_i) - c.
// Newton steps from the left of the root stay left of it and end at the
// exact root once the active set stops changing:
//   mu <- (sum_{active} z_i - c') / sum_{active} D_i.
// t = {sum_{D>0} z, sum_{D>0} D, min_{D>0} z/D, sum_{D=0} max(0, z), #(D>0)}
__host__ __device__ inline void fin_flux_init(DevState* st, const double* t) {
  st->flux_fixed = t[3];
  const double c = st->flux_c - t[3];
  const double mu = (t[0] - c) / t[1];
  st->mu = mu;
  st->flux_cnt = t[4];
  st->flux_done = (mu <= t[2]) ? 1 : 0;  // every pixel active at mu: exact root
  if (!__builtin_isfinite(mu)) {
    st->done = 1;
    st->reason = REASON_NUMERIC;
  }
}

// t = {sum_{active} z, sum_{active} D, #active} with active = {z - mu D > 0}
// at the current mu.  An unchanged active set means the step returns the
// current mu: the root.
// last: this is the last Newton pass of the iteration; if mu has still not
// converged, the direction is projected with a mu left of the root (sum of
// the projection above c), which is counted in flux_unconv and reported.
__host__ __device__ inline void fin_flux_newton(DevState* st, const double* t, bool last = false) {
  if (!(t[1] > 0.0)) {  // nothing active: c' <= 0, the projection is x = 0 on D > 0
    st->flux_done = 1;
    return;
  }
  const double mu = (t[0] - (st->flux_c - st->flux_fixed)) / t[1];
  if (t[2] == st->flux_cnt) st->flux_done = 1;
  st->flux_cnt = t[2];
  st->mu = mu;
  if (!__builtin_isfinite(mu)) {
    st->done = 1;
    st->reason = REASON_NUMERIC;
  } else if (last && !st->flux_done) {
    st->flux_unconv += 1;
  }
}

}  // namespace sgp
