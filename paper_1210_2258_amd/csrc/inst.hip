// Kernels specialised for one FFT length, SGP_L (set by the build for each
// supported length): row kernels for rows of length SGP_L and column kernels
// for columns of length SGP_L.
#include "kernels.hpp"
#include "launch.hpp"

#ifndef SGP_L
#error "SGP_L must be defined"
#endif
#define SGP_CAT2(a, b) a##b
#define SGP_CAT(a, b) SGP_CAT2(a, b)

namespace sgp {

template <int V>
static void launch_row_v(int op, dim3 grid, const Args& a, hipStream_t s) {
  constexpr int L = SGP_L;
  const dim3 blk(RowCfg<L, V>::NT);
  switch (op) {
#define SGP_ROW_CASE(OPV) case OPV: hipLaunchKernelGGL((row_kernel<L, OPV, V>), grid, blk, 0, s, a); break;
    SGP_ROW_CASE(ROW_PSF)
    SGP_ROW_CASE(ROW_MASKS)
    SGP_ROW_CASE(ROW_STORE)
    SGP_ROW_CASE(ROW_FIELD)
    SGP_ROW_CASE(ROW_RATIO)
    SGP_ROW_CASE(ROW_RLUPD)
    SGP_ROW_CASE(ROW_SETUPGRAD)
    SGP_ROW_CASE(ROW_DIR)
    SGP_ROW_CASE(ROW_AD)
    SGP_ROW_CASE(ROW_UPD)
    SGP_ROW_CASE(ROW_GRAD)
#undef SGP_ROW_CASE
    default: break;
  }
}

// Tile variants v = 0..3 (bit 0 the workgroup shape, bit 1 the transform
// plan).  A variant equal to a lower one (the length has no alternative
// plan, or the shape cannot change) is not instantiated: canon_* maps every
// v to the variant that runs it.
constexpr bool kAlt = FftPlan<SGP_L, 1>::alt;
constexpr bool row_shape_differs(int a) {
  return a == 0 ? RowCfg<SGP_L, 1>::RP != RowCfg<SGP_L, 0>::RP : RowCfg<SGP_L, 3>::RP != RowCfg<SGP_L, 2>::RP;
}
constexpr bool col_shape_differs(int a) {
  return a == 0 ? ColCfg<SGP_L, 1>::C != ColCfg<SGP_L, 0>::C : ColCfg<SGP_L, 3>::C != ColCfg<SGP_L, 2>::C;
}
constexpr int canon_row(int v) {
  const int a = kAlt ? (v >> 1) & 1 : 0;
  return 2 * a + (((v & 1) && row_shape_differs(a)) ? 1 : 0);
}
constexpr int canon_col(int v) {
  const int a = kAlt ? (v >> 1) & 1 : 0;
  return 2 * a + (((v & 1) && col_shape_differs(a)) ? 1 : 0);
}

void SGP_CAT(launch_row_, SGP_L)(int op, int v, dim3 grid, const Args& a, hipStream_t s) {
  switch (canon_row(v)) {
    case 1: if constexpr (row_shape_differs(0)) launch_row_v<1>(op, grid, a, s); break;
    case 2: if constexpr (kAlt) launch_row_v<2>(op, grid, a, s); break;
    case 3: if constexpr (kAlt && row_shape_differs(1)) launch_row_v<3>(op, grid, a, s); break;
    default: launch_row_v<0>(op, grid, a, s); break;
  }
}

template <int V>
static void launch_col_v(int mode, int conj, dim3 grid, const Args& a, hipStream_t s) {
  constexpr int L = SGP_L;
  const dim3 blk(ColCfg<L, V>::NT);
  if (mode == COL_FWD) hipLaunchKernelGGL((col_kernel<L, COL_FWD, 0, V>), grid, blk, 0, s, a);
  else if (mode == COL_CONV && (a.jn ? a.jn : a.p) == 1) {
    if (conj) hipLaunchKernelGGL((col_kernel<L, COL_CONV1, 1, V>), grid, blk, 0, s, a);
    else hipLaunchKernelGGL((col_kernel<L, COL_CONV1, 0, V>), grid, blk, 0, s, a);
  }
  else if (mode == COL_CONV && !conj) hipLaunchKernelGGL((col_kernel<L, COL_CONV, 0, V>), grid, blk, 0, s, a);
  else if (mode == COL_CONV) hipLaunchKernelGGL((col_kernel<L, COL_CONV, 1, V>), grid, blk, 0, s, a);
  else if (a.p == 1) hipLaunchKernelGGL((col_kernel<L, COL_CORR1, 1, V>), grid, blk, 0, s, a);
  else hipLaunchKernelGGL((col_kernel<L, COL_CORRSUM, 1, V>), grid, blk, 0, s, a);
}

void SGP_CAT(launch_col_, SGP_L)(int mode, int conj, int v, dim3 grid, const Args& a, hipStream_t s) {
  switch (canon_col(v)) {
    case 1: if constexpr (col_shape_differs(0)) launch_col_v<1>(mode, conj, grid, a, s); break;
    case 2: if constexpr (kAlt) launch_col_v<2>(mode, conj, grid, a, s); break;
    case 3: if constexpr (kAlt && col_shape_differs(1)) launch_col_v<3>(mode, conj, grid, a, s); break;
    default: launch_col_v<0>(mode, conj, grid, a, s); break;
  }
}

int SGP_CAT(col_width_, SGP_L)(int v) {
  const int c = canon_col(v);
  return c == 0 ? ColCfg<SGP_L, 0>::C : c == 1 ? ColCfg<SGP_L, 1>::C : c == 2 ? ColCfg<SGP_L, 2>::C : ColCfg<SGP_L, 3>::C;
}
int SGP_CAT(col_threads_, SGP_L)(int v) {
  const int c = canon_col(v);
  return c == 0 ? ColCfg<SGP_L, 0>::NT : c == 1 ? ColCfg<SGP_L, 1>::NT : c == 2 ? ColCfg<SGP_L, 2>::NT
                                                                               : ColCfg<SGP_L, 3>::NT;
}
int SGP_CAT(row_pairs_, SGP_L)(int v) {
  const int c = canon_row(v);
  return c == 0 ? RowCfg<SGP_L, 0>::RP : c == 1 ? RowCfg<SGP_L, 1>::RP : c == 2 ? RowCfg<SGP_L, 2>::RP
                                                                              : RowCfg<SGP_L, 3>::RP;
}
int SGP_CAT(row_threads_, SGP_L)(int v) {
  const int c = canon_row(v);
  return c == 0 ? RowCfg<SGP_L, 0>::NT : c == 1 ? RowCfg<SGP_L, 1>::NT : c == 2 ? RowCfg<SGP_L, 2>::NT
                                                                              : RowCfg<SGP_L, 3>::NT;
}
// the transform plan a variant runs (0 or 1)
int SGP_CAT(plan_of_, SGP_L)(int v) { return kAlt ? (v >> 1) & 1 : 0; }

// the twiddle table of length SGP_L in the pass order of plan a's transforms
void SGP_CAT(launch_twiddle_, SGP_L)(float2* tw, int a, hipStream_t s) {
  if (a && kAlt)
    hipLaunchKernelGGL((twiddle_pass_kernel<FftPlan<SGP_L, 1>>), dim3((SGP_L + 255) / 256), dim3(256), 0, s, tw);
  else
    hipLaunchKernelGGL((twiddle_pass_kernel<FftPlan<SGP_L, 0>>), dim3((SGP_L + 255) / 256), dim3(256), 0, s, tw);
}

}  // namespace sgp
