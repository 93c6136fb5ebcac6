// Pointwise (non-FFT) kernels: validation, PSF normalisation sums, start
// image, boundary weights, and the rare extra Armijo candidates.
#pragma once
#include "common.hpp"
#include "finalize.hpp"
#include "reduce.hpp"
#include "kernels.hpp"

namespace sgp {

constexpr int kArmCand = 8;  // candidates per Armijo pass: theta^2 .. theta^9, then 8 at a time

__host__ __device__ constexpr int pix_nslots(int op) {
  return op == PIX_VALIDATE ? 3 : op == PIX_PSFSUM ? 3 : op == PIX_FLATSUM ? 2 :
         op == PIX_ARMIJO ? kArmCand :
         op == PIX_FLUX_INIT ? 5 : op == PIX_FLUX_NEWTON ? 3 : op == PIX_FSUM ? 1 :
         op == PIX_RMSE ? 2 : op == PIX_RL2MAX ? 1 : 0;
}

struct PixKinds {
  int op;
  __device__ int operator()(int s) const {
    if (op == PIX_VALIDATE) return s == 1 ? RED_SUM : RED_MIN;  // min g, #non-finite, min b
    if (op == PIX_PSFSUM) return s == 1 ? RED_MIN : RED_SUM;    // sum, min, #non-finite
    if (op == PIX_FLUX_INIT) return s == 2 ? RED_MIN : RED_SUM;
    if (op == PIX_RL2MAX) return RED_MIN;
    return RED_SUM;
  }
};

// Candidates theta^10 .. theta^max_backtracks, kArmCand at a time, taken by
// the one workgroup that finished the first pass (practically never needed:
// it takes more than nine backtracks).  Every thread of the workgroup calls it.
__device__ void armijo_tail(const Args& a, DevState* st) {
  constexpr int NW = kPixThreads / 64;
  __shared__ double sh[kArmCand][NW];
  __shared__ int go;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long nS = (long long)a.ny * a.nx;
  const float* af = (st->k & 1) ? a.Af2 : a.Af;  // A f of this iteration
  for (int m0 = 2 + kArmCand; m0 <= st->max_backtracks; m0 += kArmCand) {
    const int n = min(kArmCand, st->max_backtracks + 1 - m0);
    double acc[kArmCand];
#pragma unroll
    for (int m = 0; m < kArmCand; ++m) acc[m] = 0.0;
    for (long long i = tid; i < a.p * nS; i += kPixThreads) {
      const int j = (int)(i / nS);
      const float adv = a.Ad[i];
      const float g = a.g[i];
      const float yv = fmaxf(af[i] + (a.bmap ? a.bmap[i] : pick_b(a, j)), 1e-30f);
#pragma unroll
      for (int m = 0; m < kArmCand; ++m)
        if (m < n) acc[m] += armijo_term(g, yv, (float)st->lam_tab[m0 + m] * adv);
    }
#pragma unroll
    for (int m = 0; m < kArmCand; ++m) {
      const double v = wave_reduce<kPixThreads>(RED_SUM, acc[m]);
      if (lane == 0) sh[m][wave] = v;
    }
    __syncthreads();
    if (tid == 0) {
      double t[kArmCand];
      for (int m = 0; m < kArmCand; ++m) {
        double v = sh[m][0];
        for (int w = 1; w < NW; ++w) v += sh[m][w];
        t[m] = v;
      }
      fin_armijo(st, t, m0, n);
      go = st->need_more;
    }
    __syncthreads();
    if (!go) return;
  }
}

template <int OP>
__global__ __launch_bounds__(kPixThreads) void pix_kernel(Args a_in) {
  const Args a = batch_view(a_in);
  constexpr int NS = pix_nslots(OP);
  DevState* st = a.st;
  if constexpr (OP == PIX_RMSE) {
    // once per formed iterate: also right after the update that completed a
    // stepping call's last iteration (the solver has paused by then), never
    // again for the same iteration count
    if (a.iter && (st->done || st->rms_k == st->k)) return;
  } else if constexpr (OP == PIX_RL2ZERO) {
    // before the update of f, which is also taken after a stop (f_pending),
    // and only for a step at the nonnegativity bound
    if (a.iter && ((st->done && !st->f_pending) || st->pause)) return;
    if (!(st->lam >= st->lam_bound)) return;
  } else {
    if (a.iter && (st->done || st->pause)) return;
  }
  if constexpr (OP == PIX_ARMIJO) {
    // Armijo test of lambda = 1 and theta (sums of ROW_AD) taken by every
    // workgroup; the first commits the outcome unless more candidates are
    // needed, which is rare.
    __shared__ int more;
    double t2[2];
    sum_partials<kPixThreads, 2>(RowKinds{ROW_AD}, a.part, a.fin_nblk, t2);
    if (threadIdx.x == 0) {
      more = armijo_needs_more(st, t2, 0, 2);
      if (!more && blockIdx.x == 0) fin_armijo(st, t2, 0, 2);
    }
    __syncthreads();
    if (!more) return;
  }
  if constexpr (OP == PIX_FLUX_NEWTON) {
    if (st->flux_done) return;
  }
  const long long nS = (long long)a.ny * a.nx;
  const long long nF = (long long)a.NY * a.NX;
  const long long stride = (long long)gridDim.x * kPixThreads;
  const long long i0 = (long long)blockIdx.x * kPixThreads + threadIdx.x;
  double acc[NS > 0 ? NS : 1];
  PixKinds kinds{OP};
#pragma unroll
  for (int s = 0; s < (NS > 0 ? NS : 1); ++s) acc[s] = red_identity(kinds(s));

  if constexpr (OP == PIX_VALIDATE) {
    for (long long i = i0; i < a.p * nS; i += stride) {
      const float g = a.g[i];
      if (!__builtin_isfinite(g)) acc[1] += 1.0;
      else acc[0] = fmin(acc[0], (double)g);
      if (a.bmap) {
        const float b = a.bmap[i];
        if (!__builtin_isfinite(b)) acc[1] += 1.0;
        else acc[2] = fmin(acc[2], (double)b);
      }
    }
  } else if constexpr (OP == PIX_PSFSUM) {
    const float* K = a.psf + (long long)a.jsel * nF;
    for (long long i = i0; i < nF; i += stride) {
      const float k = K[i];
      if (!__builtin_isfinite(k)) acc[2] += 1.0;
      else {
        acc[0] += k;
        acc[1] = fmin(acc[1], (double)k);
      }
    }
  } else if constexpr (OP == PIX_FLATSUM) {
    for (long long i = i0; i < a.p * nS; i += stride) {
      const int j = (int)(i / nS);
      const float b = a.bmap ? a.bmap[i] : pick_b(a, j);
      acc[0] += (double)a.g[i] - (double)b;
      acc[1] += (double)a.g[i];
    }
  } else if constexpr (OP == PIX_INITF) {
    for (long long i = i0; i < nF; i += stride) {
      const float w = a.invw ? a.invw[i] : a.invw_s;
      const float mr = w > 0.f ? 1.f : 0.f;
      float v = 0.f;
      const int mode = a.jsel;  // start option chosen by the host for this launch
      if (mode == INIT_FLAT) {
        v = mr * (float)st->cflat;
      } else if (mode == INIT_DATA) {
        const int y = (int)(i / a.NX), x = (int)(i % a.NX);
        const bool in = (unsigned)(y - a.oy) < (unsigned)a.ny && (unsigned)(x - a.ox) < (unsigned)a.nx;
        v = in ? mr * a.g[(long long)(y - a.oy) * a.nx + (x - a.ox)] : 0.f;
      } else if (mode == INIT_USER) {
        v = fmaxf(0.f, a.src[i]);
      }
      a.f[i] = v;
    }
  } else if constexpr (OP == PIX_CHOOSE) {
    // Sect. 3.1: a caller-supplied start, kept only if its KL is not larger
    // than that of the flat start
    if (st->J > st->J_alt) {
      for (long long i = i0; i < nF; i += stride) {
        const float w = a.invw ? a.invw[i] : a.invw_s;
        a.f[i] = w > 0.f ? (float)st->cflat : 0.f;
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) st->used_fallback = 1;
    }
  } else if constexpr (OP == PIX_INVW) {
    // Eq. (Rdef): R = {alpha_j >= sigma for all j}; invw = M_R / sum_j alpha_j
    for (long long i = i0; i < nF; i += stride) {
      bool inR = true;
      double sum = 0.0;
      for (int j = 0; j < a.p; ++j) {
        const float al = a.aux[(long long)j * nF + i];
        inR = inR && ((double)al >= st->sigma_R);
        sum += al;
      }
      a.d[i] = inR ? (float)(1.0 / sum) : 0.f;  // a.d points at the invw buffer for this launch
    }
  } else if constexpr (OP == PIX_INVWJ) {
    // Eq. (boundaryOSEM): M_R / alpha_j per image, R as for PIX_INVW
    for (long long i = i0; i < nF; i += stride) {
      bool inR = true;
      for (int j = 0; j < a.p; ++j) inR = inR && ((double)a.aux[(long long)j * nF + i] >= st->sigma_R);
      for (int j = 0; j < a.p; ++j) {
        const float al = a.aux[(long long)j * nF + i];
        a.d[(long long)j * nF + i] = inR ? (float)(1.0 / (double)al) : 0.f;  // a.d: the weight buffer
      }
    }
  } else if constexpr (OP == PIX_ARMIJO) {
    constexpr int m0 = 2;
    const int n = st->max_backtracks + 1 - m0;  // candidates theta^m0 .. theta^max_backtracks
    const float* af = (st->k & 1) ? a.Af2 : a.Af;  // A f of this iteration
    for (long long i = i0; i < a.p * nS; i += stride) {
      const int j = (int)(i / nS);
      const float adv = a.Ad[i];
      const float g = a.g[i];
      const float yv = fmaxf(af[i] + (a.bmap ? a.bmap[i] : pick_b(a, j)), 1e-30f);
#pragma unroll
      for (int m = 0; m < NS; ++m) {
        if (m < n) acc[m] += armijo_term(g, yv, (float)st->lam_tab[m0 + m] * adv);
      }
    }
  }

  if constexpr (OP == PIX_FLUX_INIT || OP == PIX_FLUX_NEWTON) {
    // z = f - alpha D grad with D = invw clip(f, L1, L2), as in the direction kernel
    const float alpha = (float)st->alpha, L1 = (float)st->L1, L2 = (float)st->L2;
    const double mu = st->mu;
    for (long long i = i0; i < nF; i += stride) {
      const float f = a.f[i];
      const float w = a.invw ? a.invw[i] : a.invw_s;
      const float D = w * fminf(L2, fmaxf(L1, f));
      const float z = f - alpha * D * a.grad[i];
      if constexpr (OP == PIX_FLUX_INIT) {
        if (D > 0.f) {
          acc[0] += z;
          acc[1] += D;
          acc[2] = fmin(acc[2], (double)z / (double)D);
          acc[4] += 1.0;
        } else {
          acc[3] += fmaxf(0.f, z);
        }
      } else {
        if (D > 0.f && (double)z - mu * (double)D > 0.0) {
          acc[0] += z;
          acc[1] += D;
          acc[2] += 1.0;
        }
      }
    }
  } else if constexpr (OP == PIX_FSUM) {
    for (long long i = i0; i < nF; i += stride) acc[0] += a.f[i];
  } else if constexpr (OP == PIX_RL2MAX) {
    // d of the direction pass (the same function: alpha = 1, L1 = 0,
    // L2 huge make it the RL step minus f)
    const RowScal sc = row_scalars<ROW_DIR>(st, 0);
    for (long long i = i0; i < nF; i += stride) {
      const float f = a.f[i];
      const float w = a.invw ? a.invw[i] : a.invw_s;
      const float dv = dir_value(f, a.grad[i], w, sc);
      if (dv < 0.f) acc[0] = fmin(acc[0], (double)f / -(double)dv);
    }
  } else if constexpr (OP == PIX_RL2ZERO) {
    // the pixels whose ratio f / -d attains the bound (the same d and the
    // same double division as PIX_RL2MAX) become exactly 0, as f + lam d is
    // in exact arithmetic; the update then keeps them there (d = 0)
    const RowScal sc = row_scalars<ROW_DIR>(st, 0);
    const double bound = st->lam_bound;
    for (long long i = i0; i < nF; i += stride) {
      const float f = a.f[i];
      const float w = a.invw ? a.invw[i] : a.invw_s;
      const float dv = dir_value(f, a.grad[i], w, sc);
      if (dv < 0.f && (double)f / -(double)dv <= bound) a.f[i] = 0.f;
    }
  } else if constexpr (OP == PIX_FCOPY) {
    for (long long i = i0; i < nF; i += stride) a.d[i] = a.f[i];
  } else if constexpr (OP == PIX_RMSE) {
    for (long long i = i0; i < nF; i += stride) {
      const double t = a.ftrue[i];
      const double e = (double)a.f[i] - t;
      acc[0] += e * e;
      acc[1] += t * t;
    }
  } else if constexpr (OP == PIX_FSCALE) {
    const double s = st->fsum > 0.0 ? st->flux_c / st->fsum : 1.0;
    for (long long i = i0; i < nF; i += stride) a.f[i] = (float)((double)a.f[i] * s);
  }

  __shared__ int arm_tail;
  if constexpr (OP == PIX_ARMIJO) {
    if (threadIdx.x == 0) arm_tail = 0;
  }
  if constexpr (NS > 0) {
    double tot[NS];
    // the Armijo kernel keeps ROW_AD's partials (Armijo sums, KL) intact:
    // slower workgroups may still be reading them
    double* part = OP == PIX_ARMIJO ? a.part + 3 * a.fin_nblk : a.part;
    if (grid_reduce<kPixThreads, NS>(acc, kinds, part, a.counter, a.nblk, blockIdx.x, tot)) {
      if constexpr (OP == PIX_VALIDATE) {
        if (tot[0] < 0.0 || tot[1] > 0.0) st->flags |= FLAG_BAD_DATA;
        if (tot[2] < 0.0) st->flags |= FLAG_BAD_BG;
      } else if constexpr (OP == PIX_PSFSUM) {
        if (!(tot[0] > 0.0) || tot[1] < 0.0 || tot[2] > 0.0) st->flags |= FLAG_BAD_PSF;
        else st->psf_scale[a.jsel] = 1.0 / (tot[0] * (double)a.NY * (double)a.NX);
      } else if constexpr (OP == PIX_FLATSUM) {
        // Sect. 3.1: background-subtracted (mean) flux divided by the pixel count
        double c = tot[0] / ((double)a.p * (double)nS);
        if (!(c > 0.0)) c = 1e-6 * fmax(tot[1] / ((double)a.p * (double)nS), 1e-30);
        st->cflat = c;
        // default flux of the constraint: (mean) background-subtracted flux
        if (!(st->flux >= 0.0)) st->flux_c = tot[0] / (double)a.p;
      } else if constexpr (OP == PIX_ARMIJO) {
        fin_armijo(st, tot, 2, kArmCand);
        arm_tail = st->need_more;
      } else if constexpr (OP == PIX_FLUX_INIT) {
        fin_flux_init(st, tot);
      } else if constexpr (OP == PIX_FLUX_NEWTON) {
        fin_flux_newton(st, tot, (a.flag & 1) != 0);
      } else if constexpr (OP == PIX_FSUM) {
        st->fsum = tot[0];
      } else if constexpr (OP == PIX_RMSE) {
        fin_rmse(st, tot, !a.iter, a.jsel == 1);
      } else if constexpr (OP == PIX_RL2MAX) {
        fin_rl2max(st, tot[0]);
      }
    }
  }
  if constexpr (OP == PIX_ARMIJO) {
    __syncthreads();
    if (arm_tail) armijo_tail(a, st);  // the last workgroup only
  }
}

// Second stage of the reduction of a row iteration kernel (row_deferred_fin):
// one workgroup per item sums the partials in a fixed order and runs the
// kernel's finaliser.
constexpr int kFinThreads = 256;
template <int OP>
__global__ __launch_bounds__(kFinThreads) void row_fin_kernel(Args a_in) {
  const Args a = batch_view(a_in);
  DevState* st = a.st;
  // the gradient pass before this launch has applied the accepted step
  if (OP == ROW_GRAD && a.iter && threadIdx.x == 0) st->f_pending = 0;
  if (a.iter && (st->done || st->pause)) return;
  constexpr int NS = row_nslots(OP);
  double tot[NS];
  sum_partials<kFinThreads, NS>(RowKinds{OP}, a.part + (long long)row_slot0(OP) * a.nblk, a.nblk, tot);
  if (threadIdx.x == 0) row_finalize<OP>(st, a, tot);
}

// Starts a stepping call of n iterations.
__global__ void resume_kernel(DevState* st, int n, int nitems) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nitems) {
    st[i].pause = 0;
    st[i].k_stop = st[i].k + n;
  }
}

// Clears n counters (a fill kernel rather than a memset node, so that the
// calls that may run under a caller's graph capture record kernels only).
__global__ void zero_kernel(unsigned* c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0u;
}


}  // namespace sgp
