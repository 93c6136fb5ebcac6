// Size dispatch and the size-independent pointwise kernels.
#include "launch.hpp"
#include "pix.hpp"

#define SGP_SIZES(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) \
                     X(80) X(160) X(320) X(640) X(1280)

namespace sgp {

#define SGP_DECL(L)                                                           \
  void launch_row_##L(int op, int v, dim3 grid, const Args& a, hipStream_t s); \
  void launch_col_##L(int mode, int conj, int v, dim3 grid, const Args& a, hipStream_t s); \
  int col_width_##L(int v);                                                   \
  int row_threads_##L(int v);                                                 \
  int row_pairs_##L(int v);                                                   \
  int col_threads_##L(int v);                                                 \
  int plan_of_##L(int v);                                                     \
  void launch_twiddle_##L(float2* tw, int a, hipStream_t s);
SGP_SIZES(SGP_DECL)
#undef SGP_DECL

bool size_supported(int L) {
  switch (L) {
#define SGP_CASE(L) case L: return true;
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: return false;
  }
}

int col_width(int L, int v) {
  switch (L) {
#define SGP_CASE(L) case L: return col_width_##L(v);
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: return 0;
  }
}

int row_pairs(int L, int v) {
  switch (L) {
#define SGP_CASE(L) case L: return row_pairs_##L(v);
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: return 0;
  }
}

int row_threads(int L, int v) {
  switch (L) {
#define SGP_CASE(L) case L: return row_threads_##L(v);
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: return 0;
  }
}

int plan_of(int L, int v) {
  switch (L) {
#define SGP_CASE(L) case L: return plan_of_##L(v);
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: return 0;
  }
}

int col_threads(int L, int v) {
  switch (L) {
#define SGP_CASE(L) case L: return col_threads_##L(v);
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: return 0;
  }
}

void launch_row(int L, int v, int op, dim3 grid, const Args& a, hipStream_t s) {
  switch (L) {
#define SGP_CASE(L) case L: launch_row_##L(op, v, grid, a, s); break;
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: break;
  }
}

void launch_col(int L, int v, int mode, int conj, dim3 grid, const Args& a, hipStream_t s) {
  switch (L) {
#define SGP_CASE(L) case L: launch_col_##L(mode, conj, v, grid, a, s); break;
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: break;
  }
}

void launch_pix(int op, dim3 grid, const Args& a, hipStream_t s) {
  const dim3 blk(kPixThreads);
  switch (op) {
#define SGP_PIX_CASE(OPV) case OPV: hipLaunchKernelGGL((pix_kernel<OPV>), grid, blk, 0, s, a); break;
    SGP_PIX_CASE(PIX_VALIDATE)
    SGP_PIX_CASE(PIX_PSFSUM)
    SGP_PIX_CASE(PIX_FLATSUM)
    SGP_PIX_CASE(PIX_INITF)
    SGP_PIX_CASE(PIX_INVW)
    SGP_PIX_CASE(PIX_ARMIJO)
    SGP_PIX_CASE(PIX_FLUX_INIT)
    SGP_PIX_CASE(PIX_FLUX_NEWTON)
    SGP_PIX_CASE(PIX_FSUM)
    SGP_PIX_CASE(PIX_FSCALE)
    SGP_PIX_CASE(PIX_CHOOSE)
    SGP_PIX_CASE(PIX_INVWJ)
    SGP_PIX_CASE(PIX_FCOPY)
    SGP_PIX_CASE(PIX_RMSE)
    SGP_PIX_CASE(PIX_RL2MAX)
    SGP_PIX_CASE(PIX_RL2ZERO)
#undef SGP_PIX_CASE
    default: break;
  }
}

bool row_fin_deferred(int op) { return row_deferred_fin(op); }

void launch_row_fin(int op, int nz, const Args& a, hipStream_t s) {
  const dim3 grid(1, 1, nz), blk(kFinThreads);
  switch (op) {
    case ROW_DIR: hipLaunchKernelGGL((row_fin_kernel<ROW_DIR>), grid, blk, 0, s, a); break;
    case ROW_AD: hipLaunchKernelGGL((row_fin_kernel<ROW_AD>), grid, blk, 0, s, a); break;
    case ROW_UPD: hipLaunchKernelGGL((row_fin_kernel<ROW_UPD>), grid, blk, 0, s, a); break;
    case ROW_GRAD: hipLaunchKernelGGL((row_fin_kernel<ROW_GRAD>), grid, blk, 0, s, a); break;
    default: break;
  }
}

void launch_resume(DevState* st, int n, int nitems, hipStream_t s) {
  hipLaunchKernelGGL(resume_kernel, dim3((nitems + 63) / 64), dim3(64), 0, s, st, n, nitems);
}

void launch_zero(unsigned* c, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, c, n);
}

void launch_twiddle(float2* tw, int L, int a, hipStream_t s) {
  switch (L) {
#define SGP_CASE(L) case L: launch_twiddle_##L(tw, a, s); break;
    SGP_SIZES(SGP_CASE)
#undef SGP_CASE
    default: break;
  }
}

}  // namespace sgp
