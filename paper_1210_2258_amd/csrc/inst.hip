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

// a tile variant equal to variant 0 is not instantiated
constexpr bool kRowV1 = RowCfg<SGP_L, 1>::RP != RowCfg<SGP_L, 0>::RP;
constexpr bool kColV1 = ColCfg<SGP_L, 1>::C != ColCfg<SGP_L, 0>::C;

void SGP_CAT(launch_row_, SGP_L)(int op, int v, dim3 grid, const Args& a, hipStream_t s) {
  if constexpr (kRowV1) {
    if (v == 1) return launch_row_v<1>(op, grid, a, s);
  }
  launch_row_v<0>(op, grid, a, s);
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
  if constexpr (kColV1) {
    if (v == 1) return launch_col_v<1>(mode, conj, grid, a, s);
  }
  launch_col_v<0>(mode, conj, grid, a, s);
}

int SGP_CAT(col_width_, SGP_L)(int v) { return v == 1 ? ColCfg<SGP_L, 1>::C : ColCfg<SGP_L, 0>::C; }
int SGP_CAT(row_threads_, SGP_L)(int v) { return v == 1 ? RowCfg<SGP_L, 1>::NT : RowCfg<SGP_L, 0>::NT; }
int SGP_CAT(row_pairs_, SGP_L)(int v) { return v == 1 ? RowCfg<SGP_L, 1>::RP : RowCfg<SGP_L, 0>::RP; }
int SGP_CAT(col_threads_, SGP_L)(int v) { return v == 1 ? ColCfg<SGP_L, 1>::NT : ColCfg<SGP_L, 0>::NT; }

// the twiddle table of length SGP_L in the pass order of its transforms
void SGP_CAT(launch_twiddle_, SGP_L)(float2* tw, hipStream_t s) {
  hipLaunchKernelGGL((twiddle_pass_kernel<SGP_L>), dim3((SGP_L + 255) / 256), dim3(256), 0, s, tw);
}

}  // namespace sgp
