// Stockham FFTs staged in LDS for gfx950 (wave64).
//
// A length-L complex transform is split into radix-8/4/5 passes.  Pass p with
// radix R and stride Ns (product of the earlier radices) reads butterfly j's
// inputs at j + i*L/R, applies the twiddles W_{Ns R}^{i (j mod Ns)}, runs an
// R-point DFT in registers and writes the outputs at
// (j / Ns) * Ns * R + (j mod Ns) + i*Ns (the self-sorting Stockham order, so
// the result lands in natural order with no bit reversal).  Each pass stages
// its reads in registers, so one LDS buffer per transform is enough.
//
// Several transforms share a workgroup; thread t works on transform t / TF
// with lane t % TF.  Twiddles come from a per-length table
// tw[m] = exp(-2 pi i m / L) built once per plan in double precision and
// rounded to float, regrouped per pass when a workgroup stages it in LDS
// (TwStage).  Inverse transforms use conj(FFT(conj(x))).
#pragma once
#include <hip/hip_runtime.h>

namespace sgp {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // a * (-i)
__device__ __forceinline__ float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }  // a * (+i)

// LDS index map for length-L transforms.  For power-of-two lengths bits 5-7
// of the logical index are XORed into bits 0-4 (a bijection), which spreads
// the stride-8 and stride-64 Stockham writes over all banks while keeping
// runs of 32 consecutive indices conflict-free.  Other lengths use the
// identity.
template <int L>
__host__ __device__ constexpr int lds_idx(int o) {
  if constexpr ((L & (L - 1)) == 0) return o ^ (((o >> 5) & 7) | (((o >> 6) & 3) << 3));
  else return o;
}

// ------------------------------------------------------------------ plans
// L: transform length; E: elements per thread; TF = L / E threads per
// transform; R[]: radices in pass order.  The first and last pass give every
// thread E / R butterflies; a middle pass whose butterfly count L / R is not
// a multiple of TF leaves the threads past it idle (1280: four points per
// thread, 320 threads, the radix-5 pass on 256 of them).
// Plan A = 0 is the default of each length: four points per thread from 128
// to 1280 (more waves per transform, one pass more), eight at 2048.  Plan
// A = 1, where a length has one, is the other choice the tile autotuner may
// take: eight points per thread from 128 to 1024.  A length without an
// alternative has FftPlan<L, 1> equal to FftPlan<L, 0> (alt = false), and no
// kernels are built for it.  (Four points per thread at 2048, radices
// 4,4,8,4,4, was slower and rounded its transforms less closely: five
// passes against four.)
template <int L, int A = 0> struct FftPlan : FftPlan<L, 0> {
  static constexpr bool alt = false;
};
#define SGP_FFT_PLAN(L_, A_, E_, NP_, R0, R1, R2, R3, R4)                    \
  template <> struct FftPlan<L_, A_> {                                      \
    static constexpr int len = L_, E = E_, TF = L_ / E_, NP = NP_;          \
    static constexpr int r0 = R0, r1 = R1, r2 = R2, r3 = R3, r4 = R4;       \
    static constexpr bool alt = A_ == 1;                                    \
  };
SGP_FFT_PLAN(16, 0, 4, 2, 4, 4, 1, 1, 1)
SGP_FFT_PLAN(32, 0, 8, 2, 8, 4, 1, 1, 1)
SGP_FFT_PLAN(64, 0, 8, 2, 8, 8, 1, 1, 1)
SGP_FFT_PLAN(128, 0, 4, 4, 4, 2, 4, 4, 1)
SGP_FFT_PLAN(128, 1, 8, 3, 8, 4, 4, 1, 1)
SGP_FFT_PLAN(256, 0, 4, 4, 4, 4, 4, 4, 1)
SGP_FFT_PLAN(256, 1, 8, 3, 8, 8, 4, 1, 1)
SGP_FFT_PLAN(512, 0, 4, 4, 4, 4, 8, 4, 1)
SGP_FFT_PLAN(512, 1, 8, 3, 8, 8, 8, 1, 1)
SGP_FFT_PLAN(1024, 0, 4, 5, 4, 4, 4, 4, 4)
SGP_FFT_PLAN(1024, 1, 8, 4, 8, 8, 4, 4, 1)
SGP_FFT_PLAN(2048, 0, 8, 4, 8, 8, 8, 4, 1)
SGP_FFT_PLAN(4096, 0, 16, 4, 8, 8, 8, 8, 1)
SGP_FFT_PLAN(80, 0, 20, 3, 5, 4, 4, 1, 1)
SGP_FFT_PLAN(160, 0, 20, 4, 5, 4, 4, 2, 1)
SGP_FFT_PLAN(320, 0, 20, 4, 5, 4, 4, 4, 1)
SGP_FFT_PLAN(640, 0, 20, 5, 5, 4, 4, 4, 2)
SGP_FFT_PLAN(1280, 0, 4, 5, 4, 4, 5, 4, 4)
SGP_FFT_PLAN(2560, 0, 40, 4, 5, 8, 8, 8, 1)
#undef SGP_FFT_PLAN

// ------------------------------------------------------------- butterflies
// Forward DFT of R points held in registers, X_k = sum_n x_n exp(-2 pi i n k / R).
template <int R> __device__ __forceinline__ void dft(float2* v);

template <> __device__ __forceinline__ void dft<2>(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <> __device__ __forceinline__ void dft<4>(float2* v) {
  float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <> __device__ __forceinline__ void dft<8>(float2* v) {
  // two 4-point DFTs on even / odd samples, combined with W8^k
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft<4>(e);
  dft<4>(o);
  const float h = 0.70710678118654752440f;
  float2 w1 = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));   // o1 * e^{-i pi/4}
  float2 w2 = mul_mi(o[2]);                                                // o2 * e^{-i pi/2}
  float2 w3 = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));  // o3 * e^{-3 i pi/4}
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], w1);
  v[5] = csub(e[1], w1);
  v[2] = cadd(e[2], w2);
  v[6] = csub(e[2], w2);
  v[3] = cadd(e[3], w3);
  v[7] = csub(e[3], w3);
}

template <> __device__ __forceinline__ void dft<5>(float2* v) {
  const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
  const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
  const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
  const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
  float2 a1 = cadd(v[1], v[4]), a2 = cadd(v[2], v[3]);
  float2 b1 = csub(v[1], v[4]), b2 = csub(v[2], v[3]);
  float2 x0 = v[0];
  float2 t1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
  float2 t2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
  float2 u1 = make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
  float2 u2 = make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
  v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
  v[1] = cadd(t1, mul_mi(u1));
  v[4] = cadd(t1, mul_pi(u1));
  v[2] = cadd(t2, mul_mi(u2));
  v[3] = cadd(t2, mul_pi(u2));
}

// ---------------------------------------------------------------- twiddles
// Pass order layout of the twiddles.  The pass of stride NS > 1 and radix R
// needs W_{NS R}^{i k} for i = 1 .. R-1 and k = j mod NS; it keeps them at
// NS - r0 + (i - 1) NS + k.  The lanes of a wave hold consecutive k, so each
// of their twiddle reads covers consecutive entries and spreads over the LDS
// banks (a gather from the length-L table at stride i k L / (NS R) puts up
// to 32 lanes on one bank).  The offsets telescope: all passes together hold
// L - r0 entries.  The table is built once per length in this order
// (twiddle_pass_kernel), so a workgroup stages it with a contiguous copy.

// Exponent m of W_L^m at entry t of the pass-ordered table (-1 past its end).
template <class P>
__host__ __device__ constexpr int tw_pass_index(int t) {
  constexpr int L = P::len;
  const int rs[5] = {P::r0, P::r1, P::r2, P::r3, P::r4};
  int ns = P::r0;
  for (int p = 1; p < P::NP; ++p) {
    const int R = rs[p];
    const int lo = ns - P::r0, n = (R - 1) * ns;
    if (t >= lo && t < lo + n) {
      const int u = t - lo, i = u / ns + 1, k = u % ns;
      return i * k * (L / (ns * R));
    }
    ns *= R;
  }
  return -1;
}

// The pass-ordered table of length L: exp(-2 pi i m / L) from double
// precision, rounded to float (the value the natural-order table holds at m).
template <class P>
__global__ void twiddle_pass_kernel(float2* tw) {
  constexpr int L = P::len;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < L) {
    const int m = tw_pass_index<P>(t);
    float2 v = make_float2(0.f, 0.f);
    if (m >= 0) {
      double s, c;
      sincospi(2.0 * (double)m / (double)L, &s, &c);
      v = make_float2((float)c, (float)(-s));
    }
    tw[t] = v;
  }
}

// Copy of the pass-ordered table into LDS by NT threads, split so that a
// kernel issues the global loads early (load(), with its own data loads)
// and writes LDS later (store(), before the barrier that precedes the first
// pass reading twiddles).
template <class P, int NT>
struct TwStage {
  static constexpr int N = P::len - P::r0;
  static constexpr int PER = N > 0 ? (N + NT - 1) / NT : 1;
  float2 v[PER];
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int tid) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = tid + e * NT;
      v[e] = i < N ? tw[i] : make_float2(0.f, 0.f);
    }
  }
  __device__ __forceinline__ void store(float2* twl, int tid) const {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int i = tid + e * NT;
      if (i < N) twl[i] = v[e];
    }
  }
};

// ------------------------------------------------------------------ passes
template <class P, int R, int NS>
__device__ __forceinline__ void stockham_pass(float2* buf, int lane, const float2* __restrict__ tw) {
  constexpr int L = P::len, TF = P::TF;
  constexpr int NB = L / R;
  constexpr int PER = (NB + TF - 1) / TF;
  constexpr bool ALL = PER * TF == NB;  // else butterflies j >= NB are idle
  float2 v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = lane + q * TF;
    if (ALL || j < NB) {
#pragma unroll
      for (int i = 0; i < R; ++i) v[q][i] = buf[lds_idx<L>(j + i * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = lane + q * TF;
    if (!ALL && j >= NB) continue;
    const int k = j % NS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int i = 1; i < R; ++i) v[q][i] = cmul(v[q][i], tw[NS - P::r0 + (i - 1) * NS + k]);
    }
    dft<R>(v[q]);
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int i = 0; i < R; ++i) buf[lds_idx<L>(base + i * NS)] = v[q][i];
  }
  __syncthreads();
}

// A pass whose inputs come from registers (the first pass, NS = 1) or whose
// outputs stay in registers (the last pass, NS R = L).  In both, butterfly
// q of the thread touches elements lane + TF (q + PER i), so register e holds
// element lane + TF e: x[e] on entry to the first pass, and on exit from the
// last.  A register-fed first pass writes buf without a barrier before it:
// the caller makes sure no thread still reads buf.
template <class P, int R, int NS, bool FROM_REGS, bool TO_REGS>
__device__ __forceinline__ void stockham_pass_x(float2* buf, int lane, const float2* __restrict__ tw, float2* x) {
  constexpr int L = P::len, TF = P::TF;
  constexpr int NB = L / R;
  constexpr int PER = (NB + TF - 1) / TF;
  constexpr bool ALL = PER * TF == NB;  // else butterflies j >= NB are idle
  static_assert(ALL || (!FROM_REGS && !TO_REGS), "a register-fed pass gives every thread whole butterflies");
  static_assert(!FROM_REGS || NS == 1, "only the first pass reads registers");
  static_assert(!TO_REGS || NS * R == L, "only the last pass writes registers");
  float2 v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = lane + q * TF;
    if (ALL || j < NB) {
#pragma unroll
      for (int i = 0; i < R; ++i) v[q][i] = FROM_REGS ? x[q + PER * i] : buf[lds_idx<L>(j + i * NB)];
    }
  }
  if constexpr (!FROM_REGS) __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = lane + q * TF;
    if (!ALL && j >= NB) continue;
    const int k = j % NS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int i = 1; i < R; ++i) v[q][i] = cmul(v[q][i], tw[NS - P::r0 + (i - 1) * NS + k]);
    }
    dft<R>(v[q]);
    if constexpr (TO_REGS) {
#pragma unroll
      for (int i = 0; i < R; ++i) x[q + PER * i] = v[q][i];
    } else {
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int i = 0; i < R; ++i) buf[lds_idx<L>(base + i * NS)] = v[q][i];
    }
  }
  if constexpr (!TO_REGS) __syncthreads();
}

// Forward FFT with the input (IN) and / or the output (OUT) held in
// registers, x[e] = element lane + TF e of the transform; the other side is
// buf as in fft_lds.  Saves the LDS round trip of staging the data.  With
// IN, every thread must have finished reading buf before the call; with OUT,
// buf is free for writes after the call.
template <class P, bool IN, bool OUT>
__device__ __forceinline__ void fft_lds_x(float2* buf, int lane, const float2* __restrict__ tw,
                                          float2 (&x)[P::E]) {
  constexpr int N0 = 1, N1 = P::r0, N2 = N1 * P::r1, N3 = N2 * P::r2, N4 = N3 * P::r3;
  stockham_pass_x<P, P::r0, N0, IN, OUT && P::NP == 1>(buf, lane, tw, x);
  stockham_pass_x<P, P::r1, N1, false, OUT && P::NP == 2>(buf, lane, tw, x);
  if constexpr (P::NP > 2) stockham_pass_x<P, P::r2, N2, false, OUT && P::NP == 3>(buf, lane, tw, x);
  if constexpr (P::NP > 3) stockham_pass_x<P, P::r3, N3, false, OUT && P::NP == 4>(buf, lane, tw, x);
  if constexpr (P::NP > 4) stockham_pass_x<P, P::r4, N4, false, OUT && P::NP == 5>(buf, lane, tw, x);
}

// Forward FFT of buf (logical index i stored at lds_idx<L>(i)) in place,
// natural order in and out, by plan P, with the twiddles staged by
// TwStage<P, NT>.  Every thread of the workgroup must call this (it contains
// barriers).
template <class P>
__device__ __forceinline__ void fft_lds(float2* buf, int lane, const float2* __restrict__ tw) {
  stockham_pass<P, P::r0, 1>(buf, lane, tw);
  stockham_pass<P, P::r1, P::r0>(buf, lane, tw);
  if constexpr (P::NP > 2) stockham_pass<P, P::r2, P::r0 * P::r1>(buf, lane, tw);
  if constexpr (P::NP > 3) stockham_pass<P, P::r3, P::r0 * P::r1 * P::r2>(buf, lane, tw);
  if constexpr (P::NP > 4) stockham_pass<P, P::r4, P::r0 * P::r1 * P::r2 * P::r3>(buf, lane, tw);
}

}  // namespace sgp
