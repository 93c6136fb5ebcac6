// Device kernels of the SGP / RL deconvolution path.
//
// Spectrum layout ("row-blocked"): the half spectrum of a real NY x NX field
// after the row transforms, or of a 2D transform, is stored as NY x NX/2
// complex values.  Packed column 0 holds (DC, Nyquist) of each real row, both
// real.  Element (y, kx) lives at ((y / 8) * (NX/2) + kx) * 8 + (y % 8), so a
// row kernel that owns 8 rows writes one contiguous block, and a column kernel
// that owns C columns reads 8*C contiguous values per block of rows.
//
// Row kernels own 8 rows (4 pairs).  Two real rows a, b travel through one
// complex FFT as z = a + i b; the half spectra are separated with
// A[k] = (Z[k] + conj Z[L-k]) / 2, B[k] = (Z[k] - conj Z[L-k]) / (2 i).
// Pointwise work of the solver runs between the inverse and forward row
// transforms, so every field is read and written once per kernel.
//
// Column kernels own C packed columns: forward FFT along y, multiplication by
// the transfer function (already divided by NY*NX), inverse FFT.  Column 0
// carries two real sequences (DC and Nyquist columns) and is split with the
// same even/odd rule before multiplying by its two transfer functions.
#pragma once
#include "common.hpp"
#include "fft.hpp"
#include "finalize.hpp"
#include "reduce.hpp"

namespace sgp {

__device__ __forceinline__ long long sidx(int y, int kx, int NXh) {
  return ((long long)(y >> 3) * NXh + kx) * 8 + (y & 7);
}

// View of the arguments for the item of grid-z slice blockIdx.z of a batched
// launch (the slice map lets a launch cover only the items still running).
__device__ __forceinline__ Args batch_view(const Args& in) {
  Args a = in;
  if (in.nbatch > 0) {
    const int b = in.zmap ? in.zmap[blockIdx.z] : (int)blockIdx.z;
    a.g = in.gtab[b];
    a.f = in.ftab[b];
    a.psf = in.psftab[b];
    a.src = in.srctab ? in.srctab[b] : in.src;
    a.bvec = in.bvec + b;  // one image per item
    a.grad += b * in.item_field;
    a.d += b * in.item_field;
    if (a.invw) a.invw += b * in.item_field;      // boundary items
    if (a.aux) a.aux += b * in.item_field * in.p;
    a.Af += b * in.item_obs;
    if (a.Af2) a.Af2 += b * in.item_obs;
    if (a.Ad) a.Ad += b * in.item_obs;
    a.spec += b * in.item_spec;
    a.khat += b * in.item_spec;
    a.knyq += b * in.item_nyq;
    a.part += b * in.item_part;
    a.counter += b;
    a.st += b;
  }
  return a;
}

// ------------------------------------------------------------- op traits
__host__ __device__ constexpr bool row_has_inv(int op) {
  return op == ROW_STORE || op == ROW_RATIO || op == ROW_RLUPD || op == ROW_SETUPGRAD ||
         op == ROW_AD || op == ROW_GRAD;
}
__host__ __device__ constexpr bool row_has_fwd(int op) {
  return op == ROW_PSF || op == ROW_MASKS || op == ROW_FIELD || op == ROW_RATIO ||
         op == ROW_RLUPD || op == ROW_DIR || op == ROW_AD || op == ROW_UPD;
}
__host__ __device__ constexpr int row_nslots(int op) {
  return op == ROW_RATIO ? 1 : op == ROW_SETUPGRAD ? 2 : op == ROW_DIR ? 1 :
         op == ROW_AD ? 3 : op == ROW_UPD ? 1 : op == ROW_GRAD ? 4 : 0;
}
// First partials slot of a row op.  The KL sum of the update lands in slot
// 2 whichever pass made the update (the A d pass for lambda = 1, whose slots
// 0, 1 hold the Armijo sums; the update pass otherwise).
__host__ __device__ constexpr int row_slot0(int op) { return op == ROW_UPD ? 2 : 0; }
// Iteration kernels whose reduction is finished by a separate one-workgroup
// launch (row_fin_kernel) instead of the last workgroup: the last-workgroup
// pattern needs a device-scope release in every workgroup, which writes back
// the whole L2 of its XCD before the workgroup may retire.
__host__ __device__ constexpr bool row_deferred_fin(int op) {
  return op == ROW_DIR || op == ROW_AD || op == ROW_UPD || op == ROW_GRAD;
}
// image index of the spectrum read / written
__host__ __device__ constexpr bool row_per_image(int op) {
  return op == ROW_PSF || op == ROW_STORE || op == ROW_RATIO || op == ROW_AD || op == ROW_UPD;
}

// Constant background of image j.  The values live in device memory: an
// array inside Args indexed by j would put the kernel's copy of Args in
// scratch memory.
__device__ __forceinline__ float pick_b(const Args& a, int j) { return a.bvec[j]; }

// Non-temporal store, for outputs that no kernel reads before they leave
// the cache (measured at 2048^2: the A d stores gain from it; the spectrum
// stores and the other field stores lose).
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }

struct Pix {
  const Args& a;
  int j;
  __device__ Pix(const Args& a_, int j_) : a(a_), j(j_) {}
  __device__ bool inS(int y, int x) const {
    return (unsigned)(y - a.oy) < (unsigned)a.ny && (unsigned)(x - a.ox) < (unsigned)a.nx;
  }
  __device__ long long s_of(int y, int x) const {
    return (long long)j * a.ny * a.nx + (long long)(y - a.oy) * a.nx + (x - a.ox);
  }
  __device__ float bg(long long s) const { return a.bmap ? a.bmap[s] : pick_b(a, j); }
  __device__ float w(long long pix) const { return a.invw ? a.invw[pix] : a.invw_s; }
};

// h(x) = x - log1p(x) for x > -1 without cancellation.  For |x| < 1/2, with
// u = x / (2 + x): log1p(x) = 2 atanh(u) and x - 2u = x u, so
// h(x) = x u - 2 u^3 (1/3 + u^2/5 + u^4/7 + ...); |u| <= 1/3, and the
// series stops at u^16 / 19 (truncation below 1e-10 relative).  Elsewhere
// x - log1p(x) (relative error below 3e-7 there since |log1p(x)| < 4 h(x)
// for |x| >= 1/2).
__device__ __forceinline__ float h_x(float x) {
  if (fabsf(x) < 0.5f) {
    const float u = x * __builtin_amdgcn_rcpf(2.f + x);
    const float u2 = u * u;
    float q = 1.f / 19.f;
#pragma unroll
    for (int k = 17; k >= 3; k -= 2) q = 1.f / (float)k + u2 * q;
    return x * u - 2.f * u * u2 * q;
  }
  return x - log1pf(x);
}

// 1 / d and n / d for the pointwise stages: the hardware reciprocal (about
// one ulp) refined by one Newton step on the residual, r' = r + r (1 - d r)
// and q' = q + r (n - d q) with q = n r, four instructions instead of the
// ten of an IEEE division, within an ulp of the rounded quotient.  Only for
// normal d (the hardware reciprocal flushes subnormals): every denominator
// passed here is a count (>= 1) or a model value clamped at 1e-30.
__device__ __forceinline__ float qrcp(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return fmaf(fmaf(-d, r, 1.f), r, r);
}
__device__ __forceinline__ float qdiv(float n, float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  const float q = n * r;
  return fmaf(fmaf(-d, q, n), r, q);
}

// KL term g ln(g / y) + y - g of Eq. (divergence) (y when g = 0), written as
// g h((y - g) / g).
__device__ __forceinline__ double kl_term(float g, float y) {
  return g > 0.f ? (double)(g * h_x(qdiv(y - g, g))) : (double)y;
}

// J(f + lam d) - J(f) contribution of one pixel with y = A f + b, t = lam A d:
// t - g log1p(t / y) = (y - g) x + g h(x) with x = t / y.  The exact model
// value y + t is positive for every lam <= 1 (f + lam d >= 0); when a step
// many orders of magnitude above y makes it round to <= 0 (x <= -1) where
// g > 0, the candidate lies outside the domain of J.  Such a pixel adds the
// barrier g 1e30 (+infinity once g > 3.4e8), so the candidate fails the
// Armijo test and the search goes on to a shorter step; where g = 0 the
// term stays t.  (h(-1) = +infinity is capped at 1e30 so that 0 h stays 0;
// x = NaN keeps the first product NaN, and the NaN h of x = +infinity passes
// the cap, so both are still reported as numeric failures.)
__device__ __forceinline__ double armijo_x(float g, float y, float x) {
  const float h = h_x(fmaxf(x, -1.f));
  return (double)((y - g) * x) + (double)(g * (h > 1e30f ? 1e30f : h));
}
__device__ __forceinline__ double armijo_term(float g, float y, float t) {
  return armijo_x(g, y, qdiv(t, y));
}

// Solver scalars a row kernel uses, read once per workgroup (the kernel's
// global stores could otherwise force them to be re-read at every pixel).
struct RowScal {
  float alpha, L1, L2, lam, lam0, lam1, rl_a;
  double lamd, mu, psf_scale;
  int flux;
};

template <int OP>
__device__ __forceinline__ RowScal row_scalars(const DevState* st, int j) {
  RowScal c{};
  if constexpr (OP == ROW_PSF) c.psf_scale = st->psf_scale[j];
  if constexpr (OP == ROW_DIR || OP == ROW_GRAD) {
    c.L1 = (float)st->L1;
    c.L2 = (float)st->L2;
  }
  if constexpr (OP == ROW_DIR || OP == ROW_GRAD) {
    c.alpha = (float)st->alpha;
    c.flux = st->flux_constraint;
    c.mu = st->mu;
  }
  if constexpr (OP == ROW_AD) {
    c.lam0 = (float)st->lam_tab[0];
    c.lam1 = (float)st->lam_tab[1];
  }
  if constexpr (OP == ROW_UPD) c.lam = (float)st->lam;
  if constexpr (OP == ROW_GRAD) {
    c.lamd = st->lam;
    c.lam = (float)st->lam;
  }
  if constexpr (OP == ROW_RLUPD) c.rl_a = (float)st->rl_alpha;
  return c;
}

// Direction of Algorithm 1 steps 2-3 at one pixel: D = w clip(f, L1, L2)
// (Eq. (Dk)), y = P(f - alpha D grad) onto f >= 0 (with the flux constraint
// onto {f >= 0, sum f = c}: max(0, z - mu D)), d = y - f.  The direction
// kernel uses it, and the gradient pass takes f + lam d with it instead of
// storing d; the products are fused explicitly, so both evaluate the same
// arithmetic and get the same d.
__device__ __forceinline__ float dir_value(float f, float gr, float w, const RowScal& sc) {
  const float D = w * fminf(sc.L2, fmaxf(sc.L1, f));
  const float z = fmaf(-(sc.alpha * D), gr, f);
  const float y = sc.flux && D > 0.f ? (float)fmax(0.0, fma(-sc.mu, (double)D, (double)z)) : fmaxf(0.f, z);
  return y - f;
}

// Units per load chunk: the largest divisor of nu not above cap (8; 4 in
// the gradient pass and 2 in the A d pass, which with more would exceed 128
// registers and spill; the A d pass measured faster so, with the register
// handoff, than with chunks of 4 through LDS).
__host__ __device__ constexpr int row_chunk(int nu, int cap = 8) {
  int c = nu < cap ? nu : cap;
  while (nu % c) --c;
  return c;
}

// Row ops that keep the data between their transforms and the pointwise
// stage in registers.  The ratio pass would then spill.
__host__ __device__ constexpr bool row_regs_ok(int op) {
  return op != ROW_RATIO;
}

// Global inputs of one pixel of the pointwise stage, loaded ahead of the
// pixel's arithmetic and stores so that a thread has all its loads in flight
// at once.
struct RowIn {
  float c[6];
};

template <int OP>
__device__ __forceinline__ RowIn row_load(const Args& a, int j, int y, int x) {
  Pix P(a, j);
  const long long pix = (long long)y * a.NX + x;
  RowIn in{};
  if constexpr (OP == ROW_PSF) {
    // K0 = ifftshift(K): K0[y][x] = K[(y + NY/2) % NY][(x + NX/2) % NX]
    const int ys = (y + a.NY / 2) % a.NY, xs = (x + a.NX / 2) % a.NX;
    in.c[0] = a.psf[(long long)j * a.NY * a.NX + (long long)ys * a.NX + xs];
  } else if constexpr (OP == ROW_FIELD) {
    in.c[0] = a.src[pix];
  } else if constexpr (OP == ROW_RATIO) {
    if (P.inS(y, x)) {
      const long long s = P.s_of(y, x);
      in.c[0] = a.g[s];
      in.c[1] = P.bg(s);
    }
  } else if constexpr (OP == ROW_RLUPD || OP == ROW_SETUPGRAD) {
    in.c[0] = P.w(pix);
    in.c[1] = a.f[pix];
  } else if constexpr (OP == ROW_DIR) {
    in.c[0] = a.f[pix];
    in.c[1] = a.grad[pix];
    in.c[2] = P.w(pix);
  } else if constexpr (OP == ROW_AD) {
    if (P.inS(y, x)) {
      const long long s = P.s_of(y, x);
      in.c[0] = a.g[s];
      in.c[1] = a.Af[s];  // A f of this iteration (see the buffer swap in row_kernel)
      in.c[2] = P.bg(s);
    }
  } else if constexpr (OP == ROW_UPD) {
    if (P.inS(y, x)) {
      const long long s = P.s_of(y, x);
      in.c[2] = a.Af[s];
      in.c[3] = a.Ad[s];
      in.c[4] = a.g[s];
      in.c[5] = P.bg(s);
    }
  } else if constexpr (OP == ROW_GRAD) {
    in.c[0] = P.w(pix);
    in.c[1] = a.grad[pix];
    in.c[3] = a.f[pix];
  }
  return in;
}

// One pixel of the pointwise stage.  v: result of the inverse transform at
// this pixel (conv / corr value); in: the pixel's loaded inputs; returns the
// value fed to the forward transform.  acc: per-thread FP64 accumulators.
template <int OP, int NS>
__device__ __forceinline__ float row_point(const Args& a, const RowScal& sc, int j, int y, int x, float v,
                                           const RowIn& in, double (&acc)[NS > 0 ? NS : 1]) {
  Pix P(a, j);
  const long long pix = (long long)y * a.NX + x;
  if constexpr (OP == ROW_PSF) {
    // scaled by 1 / (sum NY NX)
    return (float)((double)in.c[0] * sc.psf_scale);
  } else if constexpr (OP == ROW_MASKS) {
    return P.inS(y, x) ? 1.f : 0.f;
  } else if constexpr (OP == ROW_STORE) {
    a.aux[(long long)j * a.NY * a.NX + pix] = v;
    return 0.f;
  } else if constexpr (OP == ROW_FIELD) {
    return in.c[0];
  } else if constexpr (OP == ROW_RATIO) {
    if (!P.inS(y, x)) return 0.f;
    const long long s = P.s_of(y, x);
    if (a.flag & 1) a.Af[s] = v;
    const float g = in.c[0];
    const float yv = fmaxf(v + in.c[1], 1e-30f);
    acc[0] += kl_term(g, yv);
    return qdiv(g - yv, yv);
  } else if constexpr (OP == ROW_RLUPD) {
    // RL factor q = 1 + (M_R / alpha) v in residual form; relaxed RL
    // (Eq. (RL1)) raises it to the power rl_a
    const float w = in.c[0];
    const float f = in.c[1];
    const float q = 1.f + w * v;
    float fn = w > 0.f ? fmaxf(0.f, f * q) : 0.f;
    // q^a = 2^(a log2 q) on the hardware log2 / exp2 (about 1 ulp each;
    // q = 0 gives 0)
    if (sc.rl_a != 1.f && w > 0.f)
      fn = f * __builtin_amdgcn_exp2f(sc.rl_a * __builtin_amdgcn_logf(fmaxf(q, 0.f)));
    a.f[pix] = fn;
    return fn;
  } else if constexpr (OP == ROW_SETUPGRAD) {
    const float w = in.c[0];
    const float mr = w > 0.f ? 1.f : 0.f;
    a.grad[pix] = -mr * v;
    const float yr = w > 0.f ? in.c[1] * (1.f + w * v) : 0.f;  // one RL step from f0
    // bounds from the observed window S (equal to R for periodic problems)
    if (yr > 0.f && P.inS(y, x)) {
      acc[0] = fmin(acc[0], (double)yr);
      acc[1] = fmax(acc[1], (double)yr);
    }
    return 0.f;
  } else if constexpr (OP == ROW_DIR) {
    const float gr = in.c[1];
    const float dd = dir_value(in.c[0], gr, in.c[2], sc);
    acc[0] += (double)gr * (double)dd;
    return dd;
  } else if constexpr (OP == ROW_AD) {
    // A_j d, the Armijo sums for lambda = 1, theta, and the update of
    // Algorithm 1 step 6 for lambda = 1 (the usual outcome; ROW_UPD redoes it
    // for another lambda): A_j f + A_j d into the other A f buffer, its KL,
    // and delta rho_j = -g A_j d / (y_old y_new) for the adjoint
    if (!P.inS(y, x)) return 0.f;
    const long long s = P.s_of(y, x);
    st_nt(&a.Ad[s], v);
    const float g = in.c[0];
    const float afo = in.c[1];
    const float bgv = in.c[2];
    const float yv = fmaxf(afo + bgv, 1e-30f);
    // one reciprocal of y serves both candidates and delta rho
    const float ryv = qrcp(yv);
    const float step = sc.lam0 * v;  // lambda = 1
    const float x0 = step * ryv;
    acc[0] += armijo_x(g, yv, x0);
    acc[1] += armijo_x(g, yv, (sc.lam1 * v) * ryv);
    const float afn = afo + step;
    a.Af2[s] = afn;
    const float yn = fmaxf(afn + bgv, 1e-30f);
    acc[2] += kl_term(g, yn);
    return g > 0.f ? qdiv(-g * x0, yn) : 0.f;
  } else if constexpr (OP == ROW_UPD) {
    // A_j f += lam A_j d (f += lam d is taken by the gradient pass, which
    // reads f and d anyway); feeds delta rho_j = g/y_new - g/y_old
    // = -g lam A_j d / (y_old y_new) to the transform (no cancellation), so
    // the adjoint directly yields z = grad_new - grad_old
    const float lam = sc.lam;
    if (!P.inS(y, x)) return 0.f;
    const long long s = P.s_of(y, x);
    const float bgv = in.c[5];
    const float afo = in.c[2];
    const float step = lam * in.c[3];
    const float afn = afo + step;
    a.Af2[s] = afn;  // the other A f buffer (see the buffer swap in row_kernel)
    const float g = in.c[4];
    const float yo = fmaxf(afo + bgv, 1e-30f);
    const float yn = fmaxf(afn + bgv, 1e-30f);
    acc[0] += kl_term(g, yn);
    return g > 0.f ? qdiv(-g * step * qrcp(yo), yn) : 0.f;
  } else if constexpr (OP == ROW_GRAD) {
    // v = sum_j A_j^T delta rho_j, so z = grad_new - grad_old = -M_R v; the
    // step of Algorithm 1 step 6, f_new = f + lam d, is taken here, with d
    // evaluated again from the f and grad of the direction kernel
    const float w = in.c[0];
    const float dv = dir_value(in.c[3], in.c[1], w, sc);
    const float zf = w > 0.f ? -v : 0.f;
    a.grad[pix] = in.c[1] + zf;
    // (f + lam d >= 0 holds exactly for lam <= 1; the clamp only guards the
    // rounding of the longer steps of the linear relaxation of RL)
    const float fn = fmaxf(0.f, in.c[3] + sc.lam * dv);
    a.f[pix] = fn;
    const double s = sc.lamd * (double)dv;
    const double z = (double)zf;
    const double D = (double)(w * fminf(sc.L2, fmaxf(sc.L1, fn)));
    if (D > 0) {
      const double sd = s / D;  // (D may be subnormal when L1 is: an IEEE division)
      acc[0] += sd * sd;
      acc[1] += sd * z;
      acc[2] += s * z * D;
      acc[3] += z * z * D * D;
    }
    return 0.f;
  } else {
    return 0.f;
  }
}

template <int OP>
__device__ __forceinline__ void row_finalize(DevState* st, const Args& a, const double* t) {
  if constexpr (OP == ROW_RATIO) {
    if (a.iter) fin_rl(st, t[0]);
    else if (a.flag & 2) st->J_alt = t[0];
    else st->J = t[0];
  } else if constexpr (OP == ROW_SETUPGRAD) {
    fin_bounds(st, t[0], t[1]);
  } else if constexpr (OP == ROW_DIR) {
    fin_dir(st, t[0]);
  } else if constexpr (OP == ROW_AD) {
    fin_armijo(st, t, 0, 2);
  } else if constexpr (OP == ROW_UPD) {
    fin_update(st, t[0]);
  } else if constexpr (OP == ROW_GRAD) {
    fin_bb(st, t[0], t[1], t[2], t[3]);
  }
}

struct RowKinds {
  int op;
  __device__ int operator()(int s) const {
    if (op == ROW_SETUPGRAD) return s == 0 ? RED_MIN : RED_MAX;
    return RED_SUM;
  }
};

// Second reduction stage of a row iteration kernel run by one workgroup of
// NT threads at the start of the following launch (a.fin_op).
template <int NT>
__device__ void deferred_fin(const Args& a, DevState* st) {
  if (a.fin_op - 1 == ROW_DIR) {
    double t[1];
    sum_partials<NT, 1>(RowKinds{ROW_DIR}, a.part, a.fin_nblk, t);
    if (threadIdx.x == 0) row_finalize<ROW_DIR>(st, a, t);
  } else if (a.fin_op - 1 == ROW_UPD) {
    double t[1];
    sum_partials<NT, 1>(RowKinds{ROW_UPD}, a.part + (long long)row_slot0(ROW_UPD) * a.fin_nblk, a.fin_nblk, t);
    if (threadIdx.x == 0) row_finalize<ROW_UPD>(st, a, t);
  } else if (a.fin_op - 1 == ROW_GRAD) {
    double t[4];
    sum_partials<NT, 4>(RowKinds{ROW_GRAD}, a.part, a.fin_nblk, t);
    if (threadIdx.x == 0) row_finalize<ROW_GRAD>(st, a, t);
  }
}

// Workgroup index -> work index such that the g workgroups sharing one
// 128-byte spectrum line (an 8-row block, or two columns of one) land on the
// same XCD: the hardware deals linear workgroup ids round-robin over the 8
// XCDs, so consecutive work indices are taken from one XCD's share.
__device__ __forceinline__ int xcd_remap(int w, int n, int g) {
#ifndef SGP_NO_XCD_REMAP
  if ((n & 7) == 0 && ((n >> 3) % g) == 0) return (w & 7) * (n >> 3) + (w >> 3);
#endif
  return w;
}

// ------------------------------------------------------------------ rows
// RP row pairs (2 RP rows) per workgroup; 4 / RP workgroups share a block.
// Tile variant V: bit 0 the workgroup shape, bit 1 the transform plan
// (FftPlan<L, V >> 1>, the length's alternative points per thread and
// radices).  Shape 0 takes as many row pairs as fit 1024 threads (at most
// the 8-row block); shape 1 half as many, when that still fills a wavefront
// (otherwise it equals shape 0).  The pointwise work is the same in all; the
// autotuner picks one variant per row length.
#ifndef SGP_ROW_THREADS
#define SGP_ROW_THREADS 1024
#endif
template <int L, int V = 0> struct RowCfg {
  using P = FftPlan<L, (V >> 1)>;
  static constexpr int TF = P::TF;
  static constexpr int RP0 = SGP_ROW_THREADS / TF;
  // row pairs per workgroup: a power of two (workgroups tile the 8-row blocks)
  static constexpr int RPD = RP0 >= kRP ? kRP : RP0 >= 2 ? 2 : 1;
  static constexpr int RP = ((V & 1) && RPD >= 2 && (RPD / 2) * TF >= 64) ? RPD / 2 : RPD;
  static constexpr int NT = RP * TF;
};

template <int L, int OP, int V = 0>
__global__ __launch_bounds__((RowCfg<L, V>::NT)) void row_kernel(Args a_in) {
  Args a = batch_view(a_in);
  using P = typename RowCfg<L, V>::P;
  constexpr int TF = P::TF;
  constexpr int RP = RowCfg<L, V>::RP;
  constexpr int NT = RowCfg<L, V>::NT;
  constexpr int HALF = L / 2;
  constexpr int NS = row_nslots(OP);
  __shared__ float2 buf[RP][L];
  __shared__ float2 twl[L];  // twiddles staged in LDS in pass order
  DevState* st = a.st;
  // the gradient pass also runs after a stop when an accepted step still
  // has to be applied to f; the update pass only when lambda is not 1
  if (a.iter && ((st->done && !(OP == ROW_GRAD && st->f_pending)) || st->pause)) return;
  if constexpr (OP == ROW_UPD) {
    if (a.iter && st->spec_ok) return;
  }
  if constexpr (OP == ROW_AD || OP == ROW_UPD) {
    // A f alternates between two buffers: iteration k reads Af (k even) or
    // Af2 (k odd) and writes the other; from here on a.Af is the one read
    if (st->k & 1) {
      float* t = a.Af;
      a.Af = a.Af2;
      a.Af2 = t;
    }
  }
  const int tid = threadIdx.x;
  const int j = blockIdx.y + a.j0;
  const int wg = xcd_remap(blockIdx.x, gridDim.x, kRP / RP);
  const int y0 = wg * 2 * RP;  // first row of this workgroup
  const long long sstride = spec_elems(a.NY, a.NX);
  // (A, B) of rows y0 + 2q, y0 + 2q + 1 at column k: float4 index 4k + q + (y0 % 8) / 2
  float2* spec = a.spec + (row_per_image(OP) ? j : 0) * sstride + (long long)(y0 >> 3) * HALF * kTile + (y0 & 7);

  const float2* tw = twl;
  // the twiddles are loaded with the kernel's first data and written to LDS
  // before the barrier that precedes the first pass reading them
  TwStage<P, NT> tws;
  double acc[NS > 0 ? NS : 1];
  {
    RowKinds kinds{OP};
#pragma unroll
    for (int s = 0; s < (NS > 0 ? NS : 1); ++s) acc[s] = red_identity(kinds(s));
  }

  // with up to 8 points per thread the data passes between the transforms
  // and the pointwise stage in registers: thread tid owns pixels
  // x = lt + TF e (e < E) of row pair qt, the points its first / last FFT
  // pass reads / writes
  constexpr bool XR = P::E <= 8 && row_regs_ok(OP);
  const int qt = tid / TF, lt = tid % TF;
  float2 xr[P::E];
  if constexpr (row_has_inv(OP)) {
    const float4* S4 = reinterpret_cast<const float4*>(spec);
    // every spectrum load, then the twiddle loads, are in flight before the
    // first LDS write
    constexpr int NL = (HALF * RP + NT - 1) / NT;
    float4 sp[NL];
#pragma unroll
    for (int e = 0; e < NL; ++e) {
      const int u = tid + e * NT;
      if (u < HALF * RP) sp[e] = S4[4 * (u / RP) + u % RP];  // (A, B) of rows y0 + 2q, y0 + 2q + 1 at column k
    }
    tws.load(a.tw_row, tid);
#pragma unroll
    for (int e = 0; e < NL; ++e) {
      const int u = tid + e * NT;
      if (u >= HALF * RP) break;
      const int q = u % RP, k = u / RP;
      const float4 ab = sp[e];
      if (k == 0) {
        buf[q][lds_idx<L>(0)] = make_float2(ab.x, -ab.z);       // conj(A0 + i B0)
        buf[q][lds_idx<L>(HALF)] = make_float2(ab.y, -ab.w);    // conj(AN + i BN)
      } else {
        buf[q][lds_idx<L>(k)] = make_float2(ab.x - ab.w, -(ab.y + ab.z));      // conj(A + iB)
        buf[q][lds_idx<L>(L - k)] = make_float2(ab.x + ab.w, -(-ab.y + ab.z)); // conj(conj A + i conj B)
      }
    }
    tws.store(twl, tid);
    __syncthreads();
    if constexpr (XR) fft_lds_x<P, false, true>(buf[qt], lt, tw, xr);
    else fft_lds<P>(buf[qt], lt, tw);
  } else if constexpr (row_has_fwd(OP)) {
    tws.load(a.tw_row, tid);  // in flight with the pointwise loads
  }

  // pointwise stage in chunks of CH units per thread: every load of a chunk
  // is issued before the chunk's arithmetic and stores
  {
    const RowScal sc = row_scalars<OP>(st, j);
    constexpr int NU = RP * L / NT;  // units (pixel pairs) per thread
    static_assert(NU * NT == RP * L, "threads must tile the rows");
    constexpr int CH = OP == ROW_GRAD ? row_chunk(NU, 4) : OP == ROW_AD ? row_chunk(NU, 2) : row_chunk(NU);
    static_assert(NU % CH == 0, "chunks must tile the units");
#pragma unroll
    for (int c0 = 0; c0 < NU; c0 += CH) {
      RowIn in[CH][2];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int u = tid + (c0 + c) * NT;
        const int q = XR ? qt : u / L, x = XR ? lt + TF * (c0 + c) : u % L;
        in[c][0] = row_load<OP>(a, j, y0 + 2 * q, x);
        in[c][1] = row_load<OP>(a, j, y0 + 2 * q + 1, x);
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int u = tid + (c0 + c) * NT;
        const int q = XR ? qt : u / L, x = XR ? lt + TF * (c0 + c) : u % L;
        const int ya = y0 + 2 * q;
        float2 v = make_float2(0.f, 0.f);
        if constexpr (row_has_inv(OP)) {
          const float2 w = XR ? xr[c0 + c] : buf[q][lds_idx<L>(x)];
          v = make_float2(w.x, -w.y);
        }
        const float ua = row_point<OP, NS>(a, sc, j, ya, x, v.x, in[c][0], acc);
        const float ub = row_point<OP, NS>(a, sc, j, ya + 1, x, v.y, in[c][1], acc);
        if constexpr (row_has_fwd(OP)) {
          if constexpr (XR) xr[c0 + c] = make_float2(ua, ub);
          else buf[q][lds_idx<L>(x)] = make_float2(ua, ub);
        }
      }
    }
  }

  if constexpr (row_has_fwd(OP)) {
    // (register-fed: the inverse transform's last pass ended its LDS reads
    // with a barrier, and a forward-only op has not used buf)
    if constexpr (!row_has_inv(OP)) tws.store(twl, tid);  // (read after the first pass's barrier)
    if constexpr (XR) {
      fft_lds_x<P, true, false>(buf[qt], lt, tw, xr);
    } else {
      __syncthreads();
      fft_lds<P>(buf[qt], lt, tw);
    }
    float4* O4 = reinterpret_cast<float4*>(spec);
#pragma unroll
    for (int u = tid; u < HALF * RP; u += NT) {
      const int q = u % RP, k = u / RP;
      const float2 zk = buf[q][lds_idx<L>(k)];
      float4 o;
      if (k == 0) {
        const float2 zn = buf[q][lds_idx<L>(HALF)];
        o = make_float4(zk.x, zn.x, zk.y, zn.y);
      } else {
        const float2 zm = buf[q][lds_idx<L>(L - k)];
        o = make_float4(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y),
                        0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
      }
      O4[4 * k + q] = o;
    }
  }

  // a ratio pass of one OSEM sub-step (flag bit 4) needs no KL sum
  bool reduce = NS > 0;
  if constexpr (OP == ROW_RATIO) reduce = !(a.flag & 4);
  if constexpr (NS > 0) if (reduce) {
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    if constexpr (row_deferred_fin(OP)) {
      block_partials<NT, NS>(acc, RowKinds{OP}, a.part + (long long)row_slot0(OP) * a.nblk, a.nblk, bid);
    } else {
      double tot[NS];
      if (grid_reduce<NT, NS>(acc, RowKinds{OP}, a.part, a.counter, a.nblk, bid, tot))
        row_finalize<OP>(st, a, tot);
    }
  }
}

// --------------------------------------------------------------- columns
// C columns per workgroup.  Tile variant V: bit 1 the transform plan as for
// the rows; bit 0 the shape: 0 as many columns as fit 256 threads (at least
// one) and 40 KB of column data; 1 twice as many when at most 512 threads
// (1024 for a one-column tile) and the doubled LDS tile still fit, else half
// as many when that still fills a wavefront (otherwise it equals shape 0).
template <int LY, int V = 0> struct ColCfg {
  using P = FftPlan<LY, (V >> 1)>;
  static constexpr int TF = P::TF;
  static constexpr int C1 = 256 / TF;
  static constexpr int C2 = 40960 / (LY * 8);
  static constexpr int CD = (C1 < C2 ? C1 : C2) < 1 ? 1 : (C1 < C2 ? C1 : C2);
  static constexpr bool DBL = 2 * CD <= C2 && 2 * CD * TF <= (CD == 1 ? 1024 : 512);
  static constexpr bool HLV = CD >= 2 && (CD / 2) * TF >= 64;
  static constexpr int C = !(V & 1) ? CD : DBL ? 2 * CD : HLV ? CD / 2 : CD;
  static constexpr int NT = C * TF;
};

template <int LY, int MODE, int CONJ, int V = 0>
__global__ __launch_bounds__((ColCfg<LY, V>::NT)) void col_kernel(Args a_in) {
  const Args a = batch_view(a_in);
  using PC = typename ColCfg<LY, V>::P;
  constexpr int TF = PC::TF;
  constexpr int C = ColCfg<LY, V>::C;
  constexpr int NT = ColCfg<LY, V>::NT;
  constexpr int E = LY * C / NT;  // units per thread
  __shared__ float2 buf[C][LY];
  __shared__ float2 twl[LY];  // twiddles staged in LDS in pass order
  DevState* st = a.st;
  if (a.iter && (st->done || st->pause)) return;
  // the first workgroup of each item finishes the preceding row kernel's
  // reduction; a stop it decides is seen by the launches that follow
  if (a.fin_op && blockIdx.x == 0 && blockIdx.y == 0) deferred_fin<NT>(a, st);
  const int NXh = a.NX / 2;
  const int kx0 = xcd_remap(blockIdx.x, gridDim.x, C >= 2 ? 1 : 2) * C;
  const int tid = threadIdx.x;
  const long long sstride = spec_elems(a.NY, a.NX);
  const int jin = (MODE == COL_FWD) ? blockIdx.y : 0;
  const float2* tw = twl;
  // twiddle loads issued first, written to LDS before the barrier that
  // precedes the first pass reading them, once the column data is in flight
  TwStage<PC, NT> tws;
  tws.load(a.tw_col, tid);

  // unit e of this thread -> (column c, row y) and its offset in the layout
  auto unit = [&](int e, int& c, int& y, long long& off) {
    const int u = tid + e * NT;
    const int yb = u / (8 * C), r = u % (8 * C);
    c = r >> 3;
    y = yb * 8 + (r & 7);
    off = ((long long)yb * NXh + kx0) * 8 + r;
  };
  auto load = [&](const float2* S) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      buf[c][lds_idx<LY>(y)] = (kx0 + c < NXh) ? S[off] : make_float2(0.f, 0.f);
    }
  };
  const bool has_col0 = (kx0 == 0);

  if constexpr (MODE == COL_FWD) {
    load(a.spec + jin * sstride);
    tws.store(twl, tid);
    __syncthreads();
    fft_lds<PC>(buf[tid / TF], tid % TF, tw);
    float2* K = a.khat + jin * sstride;
    float2* KN = a.knyq + (long long)jin * LY;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      if (kx0 + c >= NXh) continue;
      const float2 v = buf[c][lds_idx<LY>(y)];
      if (has_col0 && c == 0) {
        const float2 m = cconj(buf[0][lds_idx<LY>((LY - y) % LY)]);
        K[off] = cscale(cadd(v, m), 0.5f);                   // DC column transfer function
        KN[y] = cscale(mul_mi(csub(v, m)), 0.5f);            // Nyquist column transfer function
      } else {
        K[off] = v;
      }
    }
  } else if constexpr (MODE == COL_CONV) {
    const int jlo = a.j0, jhi = a.j0 + (a.jn ? a.jn : a.p);  // images to convolve
    load(a.spec);
    float2 kpre[E];  // transfer function of image jlo, fetched while the spectrum is transformed
    const float2* K0 = a.khat + jlo * sstride;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      kpre[e] = (kx0 + c < NXh) ? K0[off] : make_float2(0.f, 0.f);
    }
    tws.store(twl, tid);
    __syncthreads();
    fft_lds<PC>(buf[tid / TF], tid % TF, tw);
    float2 x0[E], x1[E];  // spectrum (or its even / odd parts for column 0)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      const float2 v = buf[c][lds_idx<LY>(y)];
      if (has_col0 && c == 0) {
        const float2 m = cconj(buf[0][lds_idx<LY>((LY - y) % LY)]);
        x0[e] = cscale(cadd(v, m), 0.5f);
        x1[e] = cscale(mul_mi(csub(v, m)), 0.5f);
      } else {
        x0[e] = v;
        x1[e] = make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
    for (int jo = jlo; jo < jhi; ++jo) {
      int lane = tid % TF;
      asm volatile("" : "+v"(lane));  // keeps per-pass address arithmetic inside the loop
      const float2* KN = a.knyq + (long long)jo * LY;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int c, y; long long off;
        unit(e, c, y, off);
        float2 pr = make_float2(0.f, 0.f);
        if (kx0 + c < NXh) {
          const float2 kv = kpre[e];
          if (has_col0 && c == 0) {
            const float2 kn = KN[y];
            const float2 p0 = CONJ ? cmulc(x0[e], kv) : cmul(x0[e], kv);
            const float2 p1 = CONJ ? cmulc(x1[e], kn) : cmul(x1[e], kn);
            pr = cadd(p0, mul_pi(p1));
          } else {
            pr = CONJ ? cmulc(x0[e], kv) : cmul(x0[e], kv);
          }
        }
        buf[c][lds_idx<LY>(y)] = cconj(pr);
      }
      if (jo + 1 < jhi) {  // the next image's transfer function, in flight during this transform
        const float2* K1 = a.khat + (jo + 1) * sstride;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int c, y; long long off;
          unit(e, c, y, off);
          kpre[e] = (kx0 + c < NXh) ? K1[off] : make_float2(0.f, 0.f);
        }
      }
      __syncthreads();
      fft_lds<PC>(buf[tid / TF], lane, tw);
      float2* O = a.spec + jo * sstride;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int c, y; long long off;
        unit(e, c, y, off);
        if (kx0 + c < NXh) O[off] = cconj(buf[c][lds_idx<LY>(y)]);
      }
      __syncthreads();
    }
  } else if constexpr ((MODE == COL_CORR1 || MODE == COL_CONV1) && C <= 2 && E <= 8) {
    // one or two columns per workgroup: thread tid works on column
    // kx0 + tid / TF and holds its rows lane + TF e (lane = tid % TF) in
    // registers from the load to the store, the points its first and last
    // FFT passes touch; only column 0 stages its forward transform in LDS,
    // for the mirrored points of its even / odd split
    if (kx0 >= NXh) return;  // uniform over the workgroup
    const int c = tid / TF, lane = tid % TF;
    const bool live = kx0 + c < NXh;  // uniform over the column's threads; all take the barriers
    auto runit = [&](int e, int& y, long long& off) {
      y = lane + TF * e;
      off = ((long long)(y >> 3) * NXh + kx0 + c) * 8 + (y & 7);
    };
    const int jo = MODE == COL_CONV1 ? a.j0 : 0;
    const float2* K = a.khat + jo * sstride;
    const float2* KN = a.knyq + (long long)jo * LY;
    float2 xr[E], kpre[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int y; long long off;
      runit(e, y, off);
      xr[e] = live ? a.spec[off] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int y; long long off;
      runit(e, y, off);
      kpre[e] = live ? K[off] : make_float2(0.f, 0.f);
    }
    tws.store(twl, tid);  // (read after the first pass's barrier)
    fft_lds_x<PC, true, true>(buf[c], lane, tw, xr);
    if (has_col0) {  // uniform over the workgroup
      if (c == 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int y; long long off;
          runit(e, y, off);
          buf[0][lds_idx<LY>(y)] = xr[e];
        }
      }
      __syncthreads();
      if (c == 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int y; long long off;
          runit(e, y, off);
          const float2 v = xr[e];
          const float2 m = cconj(buf[0][lds_idx<LY>((LY - y) % LY)]);
          const float2 ev = cscale(cadd(v, m), 0.5f);
          const float2 od = cscale(mul_mi(csub(v, m)), 0.5f);
          const float2 kn = KN[y];
          xr[e] = cconj(cadd(CONJ ? cmulc(ev, kpre[e]) : cmul(ev, kpre[e]), mul_pi(CONJ ? cmulc(od, kn) : cmul(od, kn))));
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) xr[e] = cconj(CONJ ? cmulc(xr[e], kpre[e]) : cmul(xr[e], kpre[e]));
      }
      __syncthreads();  // mirrored reads done before the next transform writes buf
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) xr[e] = cconj(CONJ ? cmulc(xr[e], kpre[e]) : cmul(xr[e], kpre[e]));
    }
    fft_lds_x<PC, true, true>(buf[c], lane, tw, xr);
    if (live) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int y; long long off;
        runit(e, y, off);
        a.spec[jo * sstride + off] = cconj(xr[e]);
      }
    }
  } else if constexpr (MODE == COL_CORR1 || MODE == COL_CONV1) {
    // one image jo: spec[0] -> spec[jo] = K_jo x (or conj K_jo x); the
    // adjoint of one image (COL_CORRSUM for p = 1) is the case jo = 0, CONJ
    const int jo = MODE == COL_CONV1 ? a.j0 : 0;
    load(a.spec);
    const float2* K = a.khat + jo * sstride;
    const float2* KN = a.knyq + (long long)jo * LY;
    float2 kpre[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      kpre[e] = (kx0 + c < NXh) ? K[off] : make_float2(0.f, 0.f);
    }
    tws.store(twl, tid);
    __syncthreads();
    fft_lds<PC>(buf[tid / TF], tid % TF, tw);
    float2 pr[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      const float2 v = buf[c][lds_idx<LY>(y)];
      if (has_col0 && c == 0) {
        const float2 m = cconj(buf[0][lds_idx<LY>((LY - y) % LY)]);
        const float2 ev = cscale(cadd(v, m), 0.5f);
        const float2 od = cscale(mul_mi(csub(v, m)), 0.5f);
        const float2 kn = KN[y];
        pr[e] = cadd(CONJ ? cmulc(ev, kpre[e]) : cmul(ev, kpre[e]), mul_pi(CONJ ? cmulc(od, kn) : cmul(od, kn)));
      } else {
        pr[e] = CONJ ? cmulc(v, kpre[e]) : cmul(v, kpre[e]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      buf[c][lds_idx<LY>(y)] = cconj(pr[e]);
    }
    __syncthreads();
    fft_lds<PC>(buf[tid / TF], tid % TF, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      if (kx0 + c < NXh) a.spec[jo * sstride + off] = cconj(buf[c][lds_idx<LY>(y)]);
    }
  } else {  // COL_CORRSUM
    const int jb = a.j0, je = a.j0 + (a.jn ? a.jn : a.p);
    float2 acc[E], sp[E];  // sp: spectrum of the image transformed next
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      acc[e] = make_float2(0.f, 0.f);
      sp[e] = (kx0 + c < NXh) ? a.spec[jb * sstride + off] : make_float2(0.f, 0.f);
    }
    for (int ji = jb; ji < je; ++ji) {
      int lane = tid % TF;
      asm volatile("" : "+v"(lane));  // keeps per-pass address arithmetic inside the loop
      const float2* K = a.khat + ji * sstride;
      const float2* KN = a.knyq + (long long)ji * LY;
      float2 kpre[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int c, y; long long off;
        unit(e, c, y, off);
        kpre[e] = (kx0 + c < NXh) ? K[off] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int c, y; long long off;
        unit(e, c, y, off);
        buf[c][lds_idx<LY>(y)] = sp[e];
      }
      if (ji == jb) tws.store(twl, tid);
      if (ji + 1 < je) {  // the next image's spectrum, in flight during this transform
#pragma unroll
        for (int e = 0; e < E; ++e) {
          int c, y; long long off;
          unit(e, c, y, off);
          sp[e] = (kx0 + c < NXh) ? a.spec[(ji + 1) * sstride + off] : make_float2(0.f, 0.f);
        }
      }
      __syncthreads();
      fft_lds<PC>(buf[tid / TF], lane, tw);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        int c, y; long long off;
        unit(e, c, y, off);
        if (kx0 + c >= NXh) continue;
        const float2 v = buf[c][lds_idx<LY>(y)];
        const float2 kv = kpre[e];
        if (has_col0 && c == 0) {
          const float2 m = cconj(buf[0][lds_idx<LY>((LY - y) % LY)]);
          const float2 ev = cscale(cadd(v, m), 0.5f);
          const float2 od = cscale(mul_mi(csub(v, m)), 0.5f);
          const float2 kn = KN[y];
          acc[e] = cadd(acc[e], cadd(cmulc(ev, kv), mul_pi(cmulc(od, kn))));
        } else {
          acc[e] = cadd(acc[e], cmulc(v, kv));
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      buf[c][lds_idx<LY>(y)] = cconj(acc[e]);
    }
    __syncthreads();
    fft_lds<PC>(buf[tid / TF], tid % TF, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      int c, y; long long off;
      unit(e, c, y, off);
      if (kx0 + c < NXh) a.spec[off] = cconj(buf[c][lds_idx<LY>(y)]);
    }
  }
}

}  // namespace sgp
