// Warm-start network: a 4-layer 5x5 convolutional net (1 -> 16 -> 16 -> 16 ->
// 1 channels, ReLU, softplus output) that maps an observed image to an SGP
// start image, with its forward, backward and Adam kernels.
//
//   s = max(mean(g - b), 1e-3), x = (g - b) / s
//   a_l = relu(conv(a_{l-1}; W_l, b_l)) (l = 1..3), o = conv(a_3; W_4, b_4)
//   f0 = s softplus(o)
//   conv: 5x5 cross-correlation with periodic padding,
//         out[co](y,x) = b[co] + sum W[co][ci][ky][kx] in[ci](y+ky-2, x+kx-2)
//   loss = mean over pixels of (sqrt(y + 1e-3) - sqrt(f_target / s + 1e-3))^2
//
// Convolution weights are used rounded to bfloat16 (round to nearest even),
// biases in FP32, with FP32 accumulation; Adam keeps FP32 master weights.  Convolutions work on 16x16
// output tiles staged in LDS with a 2-pixel halo; the weights are uniform
// across a workgroup and stream through the scalar cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sgpcnn.h"
#include "../../include/sgpdeconv.h"

namespace sgp {
void record_error(const std::string& msg);  // sgp_last_error() text
}

namespace sgpcnn {

constexpr int K = 5;
constexpr int T = 16;          // output tile edge
constexpr int TH = T + 4;      // tile with halo
constexpr int NT = 256;        // threads per workgroup
constexpr int C = 16;          // hidden channels
constexpr float EPS_LOSS = 1e-3f;
constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {1, C, C, C};
constexpr int kCout[kLayers] = {C, C, C, 1};

__host__ __device__ constexpr int layer_w(int l) { return kCout[l] * kCin[l] * K * K; }
__host__ __device__ constexpr int layer_off(int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += layer_w(i) + kCout[i];
  return o;
}
constexpr int kParams = layer_off(kLayers);

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ------------------------------------------------------------------ kernels
// Per-image scale and input, in two launches: partial sums of g - b over
// kPrepSlices slices of each image (FP64), then s = max(mean(g - b), 1e-3)
// (every workgroup sums the partials of its image in the same order) and
// x = (g - b) / s, t = f_target / s.
constexpr int kPrepSlices = 64;

__global__ __launch_bounds__(NT) void prep_sum_kernel(const float* const* g, const float* bgd, int H, int W,
                                                      double* part) {
  const int img = blockIdx.y;
  const float* gi = g[img];
  const double b = (double)bgd[img];
  const long long N = (long long)H * W;
  __shared__ double red[NT];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < N; i += (long long)kPrepSlices * NT)
    acc += (double)gi[i] - b;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[img * kPrepSlices + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void prep_scale_kernel(const float* const* g, const float* bgd,
                                                        const float* const* ft, const double* part, int H, int W,
                                                        float* x, float* t, float* s_out) {
  const int img = blockIdx.y;
  const long long N = (long long)H * W;
  __shared__ float s_sh;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int k = 0; k < kPrepSlices; ++k) m += part[img * kPrepSlices + k];
    m /= (double)N;
    s_sh = (float)(m > 1e-3 ? m : 1e-3);
    if (blockIdx.x == 0) s_out[img] = s_sh;
  }
  __syncthreads();
  const float s = s_sh;
  const float b = bgd[img];
  const long long i = (long long)blockIdx.x * NT + threadIdx.x;
  if (i < N) {
    x[img * N + i] = (g[img][i] - b) / s;
    if (t) t[img * N + i] = ft[img][i] / s;
  }
}

// out = act(conv(in)); RELU: ReLU output, else linear.  grid (W/T, H/T, images)
template <int CIN, int COUT, bool RELU>
__global__ __launch_bounds__(NT) void conv_fwd_kernel(const float* __restrict__ in, const float* __restrict__ w,
                                                      const float* __restrict__ bias, float* __restrict__ out,
                                                      int H, int W) {
  __shared__ float tile[CIN][TH][TH];
  const int img = blockIdx.z;
  const int x0 = blockIdx.x * T, y0 = blockIdx.y * T;
  const long long N = (long long)H * W;
  const float* inb = in + (long long)img * CIN * N;
  for (int i = threadIdx.x; i < CIN * TH * TH; i += NT) {
    const int c = i / (TH * TH), r = (i / TH) % TH, q = i % TH;
    tile[c][r][q] = inb[c * N + (long long)wrap(y0 + r - 2, H) * W + wrap(x0 + q - 2, W)];
  }
  __syncthreads();
  const int ty = threadIdx.x / T, tx = threadIdx.x % T;
  float acc[COUT];
#pragma unroll
  for (int co = 0; co < COUT; ++co) acc[co] = bias[co];
  for (int ci = 0; ci < CIN; ++ci) {
#pragma unroll
    for (int ky = 0; ky < K; ++ky) {
#pragma unroll
      for (int kx = 0; kx < K; ++kx) {
        const float v = tile[ci][ty + ky][tx + kx];
#pragma unroll
        for (int co = 0; co < COUT; ++co) acc[co] = fmaf(w[((co * CIN + ci) * K + ky) * K + kx], v, acc[co]);
      }
    }
  }
  float* ob = out + (long long)img * COUT * N + (long long)(y0 + ty) * W + (x0 + tx);
#pragma unroll
  for (int co = 0; co < COUT; ++co) ob[co * N] = RELU ? fmaxf(acc[co], 0.f) : acc[co];
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// relu(conv 16 -> 16 (in)) on the matrix cores: a workgroup of four waves
// computes one 16x16 output tile as an implicit GEMM, output pixels x output
// channels x K, K = 16 input channels x 25 taps, in FP32 MFMA steps of
// 16 pixels x 16 channels x 4 (v_mfma_f32_16x16x4_f32: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 (l / 16) + r][l % 16]
// in register r).  Wave w owns tile rows 4w .. 4w + 3, one 16-pixel row per
// accumulator.  grid (W/T, H/T, images)
__global__ __launch_bounds__(NT) void conv16_mfma_kernel(const float* __restrict__ in, const float* __restrict__ w,
                                                         const float* __restrict__ bias, float* __restrict__ out,
                                                         int H, int W) {
  constexpr int KK = C * K * K;  // 400
  __shared__ float tile[C][TH][TH];
  __shared__ float wk[KK][C];    // weights as [ci * 25 + ky * 5 + kx][co]
  const int img = blockIdx.z;
  const int x0 = blockIdx.x * T, y0 = blockIdx.y * T;
  const long long N = (long long)H * W;
  const float* inb = in + (long long)img * C * N;
  for (int i = threadIdx.x; i < C * TH * TH; i += NT) {
    const int c = i / (TH * TH), r = (i / TH) % TH, q = i % TH;
    tile[c][r][q] = inb[c * N + (long long)wrap(y0 + r - 2, H) * W + wrap(x0 + q - 2, W)];
  }
  for (int i = threadIdx.x; i < KK * C; i += NT) wk[i % KK][i / KK] = w[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  floatx4 acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int s = 0; s < KK / 4; ++s) {
    const int k = 4 * s + lk;
    const int ci = k / (K * K), t = k % (K * K), ky = t / K, kx = t % K;
    const float b = wk[k][li];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float a = tile[ci][4 * wave + r + ky][li + kx];
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[r], 0, 0, 0);
    }
  }
  // acc[r][q]: channel li at pixel (4 wave + r, 4 lk + q) of the tile
  const float bc = bias[li];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float4 v = make_float4(fmaxf(acc[r][0] + bc, 0.f), fmaxf(acc[r][1] + bc, 0.f), fmaxf(acc[r][2] + bc, 0.f),
                           fmaxf(acc[r][3] + bc, 0.f));
    float* o = out + ((long long)img * C + li) * N + (long long)(y0 + 4 * wave + r) * W + x0 + 4 * lk;
    *reinterpret_cast<float4*>(o) = v;
  }
}

// ---------------------------------------------------- inference, bfloat16
// Inference keeps the hidden activations as bfloat16 in pixel-major order,
// a[img][y][x][16] (32 bytes per pixel), so that the two 16 -> 16 layers run
// on the bf16 matrix cores: v_mfma_f32_16x16x32_bf16 with lane l supplying
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] (j < 8) and
// receiving D[4 (l / 16) + r][l % 16] in register r (checked on the GPU with
// an in-bounds probe before use).  A = weights (16 output channels x K),
// B = input patches (K x 16 pixels of one tile row), K = 25 taps x 16 input
// channels with the channel fastest, padded to 13 steps of 32 (a 26th tap
// of zero weight).  Sums are FP32 in the matrix core's order.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kKSteps = 13;                  // ceil(25 * 16 / 32)
constexpr int kPackedW = kKSteps * 64 * 8;   // bf16 words of one packed 16 -> 16 layer

__device__ __forceinline__ unsigned short bf16_bits(float v) {  // nearest bfloat16, ties to even
  const unsigned u = __float_as_uint(v);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Packed A operands of a layer with 16 input channels and cout <= 16 output
// channels from its bf16-rounded weights w [co][ci][5][5]: wp[step][lane][j]
// = W[co = lane % 16][ci = 8 ((lane / 16) % 2) + j][tap = 2 step + (lane / 16) / 2],
// 0 for tap 25 and for co >= cout.
__global__ void pack16_kernel(const float* __restrict__ w, int cout, unsigned short* __restrict__ wp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPackedW) return;
  const int j = i % 8, lane = (i / 8) % 64, step = i / (8 * 64);
  const int co = lane % 16, g = lane / 16;
  const int ci = 8 * (g % 2) + j, tap = 2 * step + g / 2;
  wp[i] = tap < K * K && co < cout ? bf16_bits(w[(co * C + ci) * K * K + tap]) : (unsigned short)0;
}

// a1 = bf16(relu(conv 1 -> 16 (x))) in pixel-major order.  grid (W/T, H/T, images)
__global__ __launch_bounds__(NT) void conv1_bf16_kernel(const float* __restrict__ in, const float* __restrict__ w,
                                                         const float* __restrict__ bias,
                                                         unsigned short* __restrict__ out, int H, int W) {
  __shared__ float tile[TH][TH];
  const int img = blockIdx.z;
  const int x0 = blockIdx.x * T, y0 = blockIdx.y * T;
  const long long N = (long long)H * W;
  const float* inb = in + (long long)img * N;
  for (int i = threadIdx.x; i < TH * TH; i += NT) {
    const int r = i / TH, q = i % TH;
    tile[r][q] = inb[(long long)wrap(y0 + r - 2, H) * W + wrap(x0 + q - 2, W)];
  }
  __syncthreads();
  const int ty = threadIdx.x / T, tx = threadIdx.x % T;
  float acc[C];
#pragma unroll
  for (int co = 0; co < C; ++co) acc[co] = bias[co];
#pragma unroll
  for (int ky = 0; ky < K; ++ky) {
#pragma unroll
    for (int kx = 0; kx < K; ++kx) {
      const float v = tile[ty + ky][tx + kx];
#pragma unroll
      for (int co = 0; co < C; ++co) acc[co] = fmaf(w[co * K * K + ky * K + kx], v, acc[co]);
    }
  }
  unsigned pk[C / 2];
#pragma unroll
  for (int c2 = 0; c2 < C / 2; ++c2)
    pk[c2] = (unsigned)bf16_bits(fmaxf(acc[2 * c2], 0.f)) | ((unsigned)bf16_bits(fmaxf(acc[2 * c2 + 1], 0.f)) << 16);
  uint4* o = reinterpret_cast<uint4*>(out + (((long long)img * H + y0 + ty) * W + x0 + tx) * C);
  o[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
  o[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
}

// bf16(relu(conv 16 -> 16 (in))), pixel-major bf16 in and out: a workgroup of
// four waves computes one 16x16 output tile; wave w takes tile rows
// 4w .. 4w + 3, each row one chain of 13 matrix-core steps.  The packed
// weights stay in registers; the input tile with its 2-pixel halo is staged
// in LDS as [row][column][channel].  FINAL: the output layer, conv 16 -> 1
// (weights of channels 1..15 packed as zero), written unrounded as float32
// planes to outf.  grid (W/T, H/T, images)
template <bool FINAL>
__global__ __launch_bounds__(NT) void conv16_bf16_kernel(const unsigned short* __restrict__ in,
                                                          const unsigned short* __restrict__ wp,
                                                          const float* __restrict__ bias,
                                                          unsigned short* __restrict__ out, float* __restrict__ outf,
                                                          int H, int W) {
  __shared__ uint4 tile[TH * TH * 2];  // [r][q][two halves of 8 channels]
  const int img = blockIdx.z;
  const int x0 = blockIdx.x * T, y0 = blockIdx.y * T;
  const unsigned short* inb = in + (long long)img * H * W * C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bf16x8 a[kKSteps];
  const uint4* wp4 = reinterpret_cast<const uint4*>(wp);
#pragma unroll
  for (int st = 0; st < kKSteps; ++st) {
    const uint4 u = wp4[st * 64 + lane];
    a[st] = __builtin_bit_cast(bf16x8, u);
  }
  for (int i = threadIdx.x; i < TH * TH * 2; i += NT) {
    const int p = i >> 1, h = i & 1, r = p / TH, q = p % TH;
    const long long off = ((long long)wrap(y0 + r - 2, H) * W + wrap(x0 + q - 2, W)) * C + 8 * h;
    tile[i] = *reinterpret_cast<const uint4*>(inb + off);
  }
  __syncthreads();
  const int n = lane & 15, g = lane >> 4;
  float bc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bc[r] = FINAL ? bias[0] : bias[4 * g + r];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int row = 4 * wave + rr;
    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < kKSteps; ++st) {
      const int tap = 2 * st + g / 2;
      const int t = tap < K * K ? tap : K * K - 1;  // the padding tap has zero weight
      const int ky = t / K, kx = t % K;
      const uint4 u = tile[((row + ky) * TH + n + kx) * 2 + (g & 1)];
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[st], __builtin_bit_cast(bf16x8, u), acc, 0, 0, 0);
    }
    // acc[r]: channel 4g + r at pixel (row, n) of the tile
    if constexpr (FINAL) {
      if (g == 0) outf[((long long)img * H + y0 + row) * W + x0 + n] = acc[0] + bc[0];
      continue;
    }
    const unsigned lo = (unsigned)bf16_bits(fmaxf(acc[0] + bc[0], 0.f)) |
                        ((unsigned)bf16_bits(fmaxf(acc[1] + bc[1], 0.f)) << 16);
    const unsigned hi = (unsigned)bf16_bits(fmaxf(acc[2] + bc[2], 0.f)) |
                        ((unsigned)bf16_bits(fmaxf(acc[3] + bc[3], 0.f)) << 16);
    *reinterpret_cast<uint2*>(out + (((long long)img * H + y0 + row) * W + x0 + n) * C + 4 * g) = make_uint2(lo, hi);
  }
}

// din[ci](q) = sum_co sum_k W[co][ci][k] dout[co](q - k + 2), times the ReLU
// mask (act > 0) of the layer input.  grid (W/T, H/T, images)
template <int CIN, int COUT>
__global__ __launch_bounds__(NT) void conv_bwd_data_kernel(const float* __restrict__ dout, const float* __restrict__ w,
                                                           const float* __restrict__ act, float* __restrict__ din,
                                                           int H, int W) {
  __shared__ float tile[COUT][TH][TH];
  const int img = blockIdx.z;
  const int x0 = blockIdx.x * T, y0 = blockIdx.y * T;
  const long long N = (long long)H * W;
  const float* db = dout + (long long)img * COUT * N;
  for (int i = threadIdx.x; i < COUT * TH * TH; i += NT) {
    const int c = i / (TH * TH), r = (i / TH) % TH, q = i % TH;
    tile[c][r][q] = db[c * N + (long long)wrap(y0 + r - 2, H) * W + wrap(x0 + q - 2, W)];
  }
  __syncthreads();
  const int ty = threadIdx.x / T, tx = threadIdx.x % T;
  float acc[CIN];
#pragma unroll
  for (int ci = 0; ci < CIN; ++ci) acc[ci] = 0.f;
  for (int co = 0; co < COUT; ++co) {
#pragma unroll
    for (int ky = 0; ky < K; ++ky) {
#pragma unroll
      for (int kx = 0; kx < K; ++kx) {
        const float v = tile[co][ty - ky + 4][tx - kx + 4];
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci) acc[ci] = fmaf(w[((co * CIN + ci) * K + ky) * K + kx], v, acc[ci]);
      }
    }
  }
  const long long pix = (long long)(y0 + ty) * W + (x0 + tx);
  const float* ab = act + (long long)img * CIN * N + pix;
  float* ob = din + (long long)img * CIN * N + pix;
#pragma unroll
  for (int ci = 0; ci < CIN; ++ci) ob[ci * N] = ab[ci * N] > 0.f ? acc[ci] : 0.f;
}

// Partial weight / bias gradients of one workgroup over a strided set of
// tiles: part[wg][pair][26] with pair = co * CIN + ci, entries 0..24 the
// 5x5 weights, 25 the bias (read back for ci = 0 only).  Thread (pair, grp)
// walks tile rows grp, grp + G, ...; along a row the 5x5 input window slides
// in registers, so each pixel costs five LDS reads for 26 FMAs.
template <int CIN, int COUT>
__global__ __launch_bounds__(NT) void conv_bwd_w_kernel(const float* __restrict__ in, const float* __restrict__ dout,
                                                        float* __restrict__ part, int H, int W, int nimg) {
  constexpr int NPAIR = CIN * COUT;
  constexpr int G = NT / NPAIR;            // pixel-row groups sharing a pair
  static_assert(G * NPAIR == NT && T % G == 0, "pairs must divide the workgroup");
  constexpr int IS = TH * TH + 1;          // odd channel strides spread the
  constexpr int DS = T * T + 1;            // channels of one wave over the banks
  constexpr int NA = K * K + 1;
  __shared__ float itile[CIN * IS];
  __shared__ float dtile[COUT * DS];
  __shared__ float red[G > 1 ? NT * NA : 1];
  const int pair = threadIdx.x % NPAIR, grp = threadIdx.x / NPAIR;
  const int co = pair / CIN, ci = pair % CIN;
  const long long N = (long long)H * W;
  const int tx_n = W / T, ty_n = H / T;
  const long long per_img = (long long)tx_n * ty_n;
  const long long ntiles = per_img * nimg;
  float acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k] = 0.f;
  for (long long tI = blockIdx.x; tI < ntiles; tI += gridDim.x) {
    const int img = (int)(tI / per_img);
    const int rem = (int)(tI % per_img);
    const int y0 = (rem / tx_n) * T, x0 = (rem % tx_n) * T;
    const float* ib = in + (long long)img * CIN * N;
    const float* db = dout + (long long)img * COUT * N;
    __syncthreads();
    for (int i = threadIdx.x; i < CIN * TH * TH; i += NT) {
      const int c = i / (TH * TH), r = (i / TH) % TH, q = i % TH;
      itile[c * IS + r * TH + q] = ib[c * N + (long long)wrap(y0 + r - 2, H) * W + wrap(x0 + q - 2, W)];
    }
    for (int i = threadIdx.x; i < COUT * T * T; i += NT) {
      const int c = i / (T * T), r = (i / T) % T, q = i % T;
      dtile[c * DS + r * T + q] = db[c * N + (long long)(y0 + r) * W + (x0 + q)];
    }
    __syncthreads();
    const float* it = itile + ci * IS;
    const float* dt = dtile + co * DS;
    for (int py = grp; py < T; py += G) {
      float win[K][K];
#pragma unroll
      for (int ky = 0; ky < K; ++ky)
#pragma unroll
        for (int kx = 0; kx < K - 1; ++kx) win[ky][kx] = it[(py + ky) * TH + kx];
#pragma unroll
      for (int px = 0; px < T; ++px) {
#pragma unroll
        for (int ky = 0; ky < K; ++ky) win[ky][K - 1] = it[(py + ky) * TH + px + K - 1];
        const float d = dt[py * T + px];
#pragma unroll
        for (int ky = 0; ky < K; ++ky)
#pragma unroll
          for (int kx = 0; kx < K; ++kx) acc[ky * K + kx] = fmaf(d, win[ky][kx], acc[ky * K + kx]);
        acc[K * K] += d;
#pragma unroll
        for (int ky = 0; ky < K; ++ky)
#pragma unroll
          for (int kx = 0; kx < K - 1; ++kx) win[ky][kx] = win[ky][kx + 1];
      }
    }
  }
  float* o = part + ((long long)blockIdx.x * NPAIR + pair) * NA;
  if constexpr (G == 1) {
#pragma unroll
    for (int k = 0; k < NA; ++k) o[k] = acc[k];
  } else {
    // combine the G row groups of each pair in a fixed order
#pragma unroll
    for (int k = 0; k < NA; ++k) red[threadIdx.x * NA + k] = acc[k];
    __syncthreads();
    if (grp == 0) {
      for (int q = 1; q < G; ++q)
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k] += red[(q * NPAIR + pair) * NA + k];
#pragma unroll
      for (int k = 0; k < NA; ++k) o[k] = acc[k];
    }
  }
}

// grad of layer l from the partials of nwg workgroups (fixed-order FP64 sums).
__global__ void reduce_wgrad_kernel(const float* __restrict__ part, int nwg, int cin, int cout,
                                    float* __restrict__ grad_w, float* __restrict__ grad_b) {
  const int npair = cin * cout;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npair * (K * K + 1)) return;
  const int pair = i / (K * K + 1), k = i % (K * K + 1);
  double s = 0.0;
  for (int g = 0; g < nwg; ++g) s += part[((long long)g * npair + pair) * (K * K + 1) + k];
  const int co = pair / cin, ci = pair % cin;
  if (k < K * K) grad_w[(co * cin + ci) * K * K + k] = (float)s;
  else if (ci == 0) grad_b[co] = (float)s;
}

__device__ __forceinline__ float softplusf(float o) { return o > 20.f ? o : log1pf(expf(o)); }

// dL/do and per-workgroup loss partials (FP64) for a batch of n images.
__global__ __launch_bounds__(NT) void loss_grad_kernel(const float* __restrict__ o, const float* __restrict__ t,
                                                       long long total, float* __restrict__ d_o,
                                                       double* __restrict__ lpart) {
  __shared__ double red[NT];
  double acc = 0.0;
  const float inv = 1.0f / (float)total;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < total; i += (long long)gridDim.x * NT) {
    const float ov = o[i];
    const float y = softplusf(ov);
    const float sy = sqrtf(y + EPS_LOSS), st = sqrtf(t[i] + EPS_LOSS);
    const float r = sy - st;
    acc += (double)r * (double)r;
    d_o[i] = r / sy * inv / (1.f + expf(-ov));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// f0 = s softplus(o) for each image (pointer table of outputs)
__global__ void output_kernel(const float* __restrict__ o, const float* __restrict__ s, float* const* f0, int H,
                              int W) {
  const int img = blockIdx.y;
  const long long N = (long long)H * W;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) f0[img][i] = s[img] * softplusf(o[img * N + i]);
}

__device__ __forceinline__ float bf16_round(float v) {
  unsigned u = __float_as_uint(v);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// Adam on the FP32 master weights, then the bf16-rounded copy used by the
// kernels.  t: step count from 1.
__global__ void adam_kernel(float* theta, float* m, float* v, const float* grad, float* wr, int n, float lr,
                            float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = 0.9f * m[i] + 0.1f * g;
  const float vi = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mi;
  v[i] = vi;
  const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  theta[i] = th;
  wr[i] = bf16_round(th);
}

__global__ void round_kernel(const float* theta, float* wr, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wr[i] = bf16_round(theta[i]);
}

// ------------------------------------------------------------------ host
#define CNN_HIP(x)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      sgp::record_error(std::string(#x) + ": " + hipGetErrorString(e_));                \
      return SGP_E_HIP;                                                                 \
    }                                                                                   \
  } while (0)

struct Net {
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *wr = nullptr;
  unsigned short* wp = nullptr;  // packed bf16 A operands of layers 2-4 (inference)
  int step = 0;
  // work buffers, sized for cap_px pixels over at most cap_n images; the
  // training buffers exist only once a training call has been made
  size_t cap_px = 0;
  int cap_n = 0;
  bool cap_train = false;
  float *x = nullptr, *t = nullptr, *s = nullptr, *a[3] = {nullptr, nullptr, nullptr}, *o = nullptr;
  float *da = nullptr, *db = nullptr, *d_o = nullptr, *part = nullptr;
  double* lpart = nullptr;
  double* host_lpart = nullptr;
  double* ppart = nullptr;  // [cap_n][kPrepSlices] partial sums of the input scale
  const float** gtab = nullptr;
  const float** fttab = nullptr;
  float** f0tab = nullptr;
  float* btab = nullptr;
  ~Net() { release(); free_params(); }
  void release() {
    void* p[] = {x, t, s, a[0], a[1], a[2], o, da, db, d_o, part, lpart, ppart, (void*)gtab, (void*)fttab, (void*)f0tab, btab};
    for (void* q : p)
      if (q) (void)hipFree(q);
    if (host_lpart) (void)hipHostFree(host_lpart);
    x = t = s = o = da = db = d_o = part = btab = nullptr;
    a[0] = a[1] = a[2] = nullptr;
    lpart = nullptr;
    ppart = nullptr;
    host_lpart = nullptr;
    gtab = fttab = nullptr;
    f0tab = nullptr;
    cap_px = 0;
    cap_n = 0;
    cap_train = false;
  }
  void free_params() {
    void* p[] = {theta, m, v, grad, wr, wp};
    for (void* q : p)
      if (q) (void)hipFree(q);
    theta = m = v = grad = wr = nullptr;
    wp = nullptr;
  }
};

constexpr int kWgPart = 1024;   // workgroups of the weight-gradient kernels
constexpr int kLossWg = 256;

template <class T>
static int dal(T** p, size_t n) {
  hipError_t e = hipMalloc((void**)p, sizeof(T) * (n ? n : 1));
  if (e != hipSuccess) {
    sgp::record_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return SGP_E_HIP;
  }
  return 0;
}

static int ensure(Net* net, int n, int H, int W, bool train) {
  const size_t N = (size_t)H * W * n;
  if (net->cap_px >= N && net->cap_n >= n && (!train || net->cap_train)) return 0;
  const size_t px = std::max(N, net->cap_px);
  const int nn = std::max(n, net->cap_n);
  const bool tr = train || net->cap_train;
  net->release();
  int rc;
  if ((rc = dal(&net->x, px)) || (rc = dal(&net->s, nn)) || (rc = dal(&net->o, px)) ||
      (rc = dal(&net->a[0], px * C)) || (rc = dal(&net->a[1], px * C)) || (rc = dal(&net->gtab, nn)) ||
      (rc = dal(&net->fttab, nn)) || (rc = dal(&net->f0tab, nn)) || (rc = dal(&net->btab, nn)) ||
      (rc = dal(&net->ppart, (size_t)nn * kPrepSlices)))
    return rc;
  if (tr) {
    if ((rc = dal(&net->a[2], px * C)) || (rc = dal(&net->t, px)) || (rc = dal(&net->da, px * C)) ||
        (rc = dal(&net->db, px * C)) || (rc = dal(&net->d_o, px)) ||
        (rc = dal(&net->part, (size_t)kWgPart * C * C * (K * K + 1))) || (rc = dal(&net->lpart, kLossWg)))
      return rc;
    CNN_HIP(hipHostMalloc((void**)&net->host_lpart, sizeof(double) * kLossWg, hipHostMallocDefault));
  }
  net->cap_px = px;
  net->cap_n = nn;
  net->cap_train = tr;
  return 0;
}

static const float* wl(const Net* net, int l) { return net->wr + layer_off(l); }
// biases stay FP32: they are read from the master copy
static const float* bl(const Net* net, int l) { return net->theta + layer_off(l) + layer_w(l); }

// forward of n images into o; training keeps all three hidden activations,
// inference overwrites the first with the third
static int forward(Net* net, int n, int H, int W, bool train, hipStream_t s) {
  const dim3 grid(W / T, H / T, n);
  float* a3 = train ? net->a[2] : net->a[0];
  hipLaunchKernelGGL((conv_fwd_kernel<1, C, true>), grid, dim3(NT), 0, s, net->x, wl(net, 0), bl(net, 0), net->a[0], H, W);
  hipLaunchKernelGGL(conv16_mfma_kernel, grid, dim3(NT), 0, s, net->a[0], wl(net, 1), bl(net, 1), net->a[1], H, W);
  hipLaunchKernelGGL(conv16_mfma_kernel, grid, dim3(NT), 0, s, net->a[1], wl(net, 2), bl(net, 2), a3, H, W);
  hipLaunchKernelGGL((conv_fwd_kernel<C, 1, false>), grid, dim3(NT), 0, s, a3, wl(net, 3), bl(net, 3), net->o, H, W);
  CNN_HIP(hipGetLastError());
  return 0;
}

// inference forward of n images into o: hidden activations as bfloat16 in
// pixel-major order (a[0], a[1] hold them at half their float32 capacity),
// the 16 -> 16 layers on the bf16 matrix cores
static int forward_infer(Net* net, int n, int H, int W, hipStream_t s) {
  const dim3 grid(W / T, H / T, n);
  unsigned short* a0 = reinterpret_cast<unsigned short*>(net->a[0]);
  unsigned short* a1 = reinterpret_cast<unsigned short*>(net->a[1]);
  for (int l = 1; l <= 3; ++l)
    hipLaunchKernelGGL(pack16_kernel, dim3((kPackedW + 255) / 256), dim3(256), 0, s, wl(net, l), kCout[l],
                       net->wp + (l - 1) * kPackedW);
  hipLaunchKernelGGL(conv1_bf16_kernel, grid, dim3(NT), 0, s, net->x, wl(net, 0), bl(net, 0), a0, H, W);
  hipLaunchKernelGGL(conv16_bf16_kernel<false>, grid, dim3(NT), 0, s, a0, net->wp, bl(net, 1), a1, nullptr, H, W);
  hipLaunchKernelGGL(conv16_bf16_kernel<false>, grid, dim3(NT), 0, s, a1, net->wp + kPackedW, bl(net, 2), a0,
                     nullptr, H, W);
  hipLaunchKernelGGL(conv16_bf16_kernel<true>, grid, dim3(NT), 0, s, a0, net->wp + 2 * kPackedW, bl(net, 3),
                     nullptr, net->o, H, W);
  CNN_HIP(hipGetLastError());
  return 0;
}

// network input (and training target) of n images into x (t)
static int prep(Net* net, int n, int H, int W, bool train, hipStream_t s) {
  const long long N = (long long)H * W;
  hipLaunchKernelGGL(prep_sum_kernel, dim3(kPrepSlices, n), dim3(NT), 0, s, (const float* const*)net->gtab,
                     (const float*)net->btab, H, W, net->ppart);
  hipLaunchKernelGGL(prep_scale_kernel, dim3((unsigned)((N + NT - 1) / NT), n), dim3(NT), 0, s,
                     (const float* const*)net->gtab, (const float*)net->btab,
                     train ? (const float* const*)net->fttab : (const float* const*)nullptr, (const double*)net->ppart,
                     H, W, net->x, train ? net->t : (float*)nullptr, net->s);
  CNN_HIP(hipGetLastError());
  return 0;
}

static int check_shape(int n, int H, int W) {
  if (n < 1 || H < T || W < T || H % T || W % T) {
    sgp::record_error("warm-start network needs n >= 1 and image sides that are multiples of 16");
    return SGP_E_INVALID_ARG;
  }
  return 0;
}

static int set_tables(Net* net, int n, const float* const* g, const float* b, const float* const* ft,
                      float* const* f0, hipStream_t s) {
  CNN_HIP(hipMemcpy(net->gtab, g, sizeof(float*) * n, hipMemcpyHostToDevice));
  CNN_HIP(hipMemcpy(net->btab, b, sizeof(float) * n, hipMemcpyHostToDevice));
  if (ft) CNN_HIP(hipMemcpy(net->fttab, ft, sizeof(float*) * n, hipMemcpyHostToDevice));
  if (f0) CNN_HIP(hipMemcpy(net->f0tab, f0, sizeof(float*) * n, hipMemcpyHostToDevice));
  (void)s;
  return 0;
}

}  // namespace sgpcnn

using namespace sgpcnn;

struct sgp_cnn : sgpcnn::Net {};

extern "C" {

int sgp_cnn_create(const float* host_params, size_t nparams, sgp_cnn** out) {
  if (!out) return SGP_E_INVALID_ARG;
  *out = nullptr;
  if (!host_params || nparams != (size_t)kParams) {
    sgp::record_error("warm-start network expects " + std::to_string(kParams) + " parameters");
    return SGP_E_INVALID_ARG;
  }
  int dev_n = 0;
  if (hipGetDeviceCount(&dev_n) != hipSuccess || dev_n <= 0) return SGP_E_NO_DEVICE;
  sgp_cnn* net = new sgp_cnn();
  int rc;
  if ((rc = dal(&net->theta, kParams)) || (rc = dal(&net->m, kParams)) || (rc = dal(&net->v, kParams)) ||
      (rc = dal(&net->grad, kParams)) || (rc = dal(&net->wr, kParams)) || (rc = dal(&net->wp, 3 * kPackedW))) {
    delete net;
    return rc;
  }
  hipError_t e = hipMemcpy(net->theta, host_params, sizeof(float) * kParams, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(net->m, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMemset(net->v, 0, sizeof(float) * kParams);
  if (e != hipSuccess) {
    sgp::record_error(hipGetErrorString(e));
    delete net;
    return SGP_E_HIP;
  }
  hipLaunchKernelGGL(round_kernel, dim3((kParams + 255) / 256), dim3(256), 0, nullptr, net->theta, net->wr, kParams);
  if (hipDeviceSynchronize() != hipSuccess) {
    delete net;
    return SGP_E_HIP;
  }
  *out = net;
  return SGP_OK;
}

int sgp_cnn_num_params(void) { return kParams; }

int sgp_cnn_get_params(sgp_cnn* h, float* host_out, size_t nparams) {
  Net* net = h;
  if (!net || !host_out || nparams != (size_t)kParams) return SGP_E_INVALID_ARG;
  CNN_HIP(hipMemcpy(host_out, net->theta, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  return SGP_OK;
}

int sgp_cnn_infer(sgp_cnn* h, int n, const float* const* g, const float* b, int ny, int nx, float* const* f0,
                  void* stream) {
  Net* net = h;
  if (!net || !g || !b || !f0) return SGP_E_INVALID_ARG;
  int rc;
  if ((rc = check_shape(n, ny, nx))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = ensure(net, n, ny, nx, false))) return rc;
  if ((rc = set_tables(net, n, g, b, nullptr, f0, s))) return rc;
  if ((rc = prep(net, n, ny, nx, false, s))) return rc;
  if ((rc = forward_infer(net, n, ny, nx, s))) return rc;
  const long long N = (long long)ny * nx;
  hipLaunchKernelGGL(output_kernel, dim3((unsigned)((N + 255) / 256), n), dim3(256), 0, s, net->o, net->s,
                     net->f0tab, ny, nx);
  CNN_HIP(hipGetLastError());
  CNN_HIP(hipStreamSynchronize(s));
  return SGP_OK;
}

int sgp_cnn_loss_grad(sgp_cnn* h, int n, const float* const* g, const float* b, const float* const* f_target, int ny,
                      int nx, double* loss, float* host_grad, void* stream) {
  Net* net = h;
  if (!net || !g || !b || !f_target) return SGP_E_INVALID_ARG;
  int rc;
  if ((rc = check_shape(n, ny, nx))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = ensure(net, n, ny, nx, true))) return rc;
  if ((rc = set_tables(net, n, g, b, f_target, nullptr, s))) return rc;
  if ((rc = prep(net, n, ny, nx, true, s))) return rc;
  if ((rc = forward(net, n, ny, nx, true, s))) return rc;
  const long long total = (long long)n * ny * nx;
  hipLaunchKernelGGL(loss_grad_kernel, dim3(kLossWg), dim3(NT), 0, s, net->o, net->t, total, net->d_o, net->lpart);
  const dim3 grid(nx / T, ny / T, n);
  const int nwg = (int)std::min<long long>(kWgPart, (long long)(nx / T) * (ny / T) * n);
  float* gw[kLayers];
  float* gb[kLayers];
  for (int l = 0; l < kLayers; ++l) {
    gw[l] = net->grad + layer_off(l);
    gb[l] = gw[l] + layer_w(l);
  }
  auto reduce = [&](int l) {
    const int cnt = kCin[l] * kCout[l] * (K * K + 1);
    hipLaunchKernelGGL(reduce_wgrad_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, net->part, nwg, kCin[l],
                       kCout[l], gw[l], gb[l]);
  };
  // layer 4
  hipLaunchKernelGGL((conv_bwd_w_kernel<C, 1>), dim3(nwg), dim3(NT), 0, s, net->a[2], net->d_o, net->part, ny, nx, n);
  reduce(3);
  hipLaunchKernelGGL((conv_bwd_data_kernel<C, 1>), grid, dim3(NT), 0, s, net->d_o, wl(net, 3), net->a[2], net->da, ny, nx);
  // layer 3
  hipLaunchKernelGGL((conv_bwd_w_kernel<C, C>), dim3(nwg), dim3(NT), 0, s, net->a[1], net->da, net->part, ny, nx, n);
  reduce(2);
  hipLaunchKernelGGL((conv_bwd_data_kernel<C, C>), grid, dim3(NT), 0, s, net->da, wl(net, 2), net->a[1], net->db, ny, nx);
  // layer 2
  hipLaunchKernelGGL((conv_bwd_w_kernel<C, C>), dim3(nwg), dim3(NT), 0, s, net->a[0], net->db, net->part, ny, nx, n);
  reduce(1);
  hipLaunchKernelGGL((conv_bwd_data_kernel<C, C>), grid, dim3(NT), 0, s, net->db, wl(net, 1), net->a[0], net->da, ny, nx);
  // layer 1
  hipLaunchKernelGGL((conv_bwd_w_kernel<1, C>), dim3(nwg), dim3(NT), 0, s, net->x, net->da, net->part, ny, nx, n);
  reduce(0);
  CNN_HIP(hipGetLastError());
  CNN_HIP(hipMemcpyAsync(net->host_lpart, net->lpart, sizeof(double) * kLossWg, hipMemcpyDeviceToHost, s));
  CNN_HIP(hipStreamSynchronize(s));
  if (loss) {
    double L = 0.0;
    for (int i = 0; i < kLossWg; ++i) L += net->host_lpart[i];
    *loss = L / (double)total;
  }
  if (host_grad) CNN_HIP(hipMemcpy(host_grad, net->grad, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  return SGP_OK;
}

int sgp_cnn_adam_step(sgp_cnn* h, float lr, void* stream) {
  Net* net = h;
  if (!net || !(lr > 0)) return SGP_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  net->step += 1;
  const float c1 = 1.0f - powf(0.9f, (float)net->step);
  const float c2 = 1.0f - powf(0.999f, (float)net->step);
  hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, net->theta, net->m, net->v,
                     net->grad, net->wr, kParams, lr, c1, c2);
  CNN_HIP(hipGetLastError());
  CNN_HIP(hipStreamSynchronize(s));
  return SGP_OK;
}

int sgp_cnn_train_step(sgp_cnn* h, int n, const float* const* g, const float* b, const float* const* f_target, int ny,
                       int nx, float lr, double* loss, void* stream) {
  int rc = sgp_cnn_loss_grad(h, n, g, b, f_target, ny, nx, loss, nullptr, stream);
  if (rc) return rc;
  return sgp_cnn_adam_step(h, lr, stream);
}

int sgp_cnn_destroy(sgp_cnn* h) {
  delete h;
  return SGP_OK;
}

}  // extern "C"
