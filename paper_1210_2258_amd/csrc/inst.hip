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

void SGP_CAT(launch_row_, SGP_L)(int op, dim3 grid, const Args& a, hipStream_t s) {
  constexpr int L = SGP_L;
  const dim3 blk(RowCfg<L>::NT);
  switch (op) {
#define SGP_ROW_CASE(OPV) case OPV: hipLaunchKernelGGL((row_kernel<L, OPV>), grid, blk, 0, s, a); break;
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

void SGP_CAT(launch_col_, SGP_L)(int mode, int conj, dim3 grid, const Args& a, hipStream_t s) {
  constexpr int L = SGP_L;
  const dim3 blk(ColCfg<L>::NT);
  if (mode == COL_FWD) hipLaunchKernelGGL((col_kernel<L, COL_FWD, 0>), grid, blk, 0, s, a);
  else if (mode == COL_CONV && (a.jn ? a.jn : a.p) == 1) {
    if (conj) hipLaunchKernelGGL((col_kernel<L, COL_CONV1, 1>), grid, blk, 0, s, a);
    else hipLaunchKernelGGL((col_kernel<L, COL_CONV1, 0>), grid, blk, 0, s, a);
  }
  else if (mode == COL_CONV && !conj) hipLaunchKernelGGL((col_kernel<L, COL_CONV, 0>), grid, blk, 0, s, a);
  else if (mode == COL_CONV) hipLaunchKernelGGL((col_kernel<L, COL_CONV, 1>), grid, blk, 0, s, a);
  else if (a.p == 1) hipLaunchKernelGGL((col_kernel<L, COL_CORR1, 1>), grid, blk, 0, s, a);
  else hipLaunchKernelGGL((col_kernel<L, COL_CORRSUM, 1>), grid, blk, 0, s, a);
}

int SGP_CAT(col_width_, SGP_L)() { return ColCfg<SGP_L>::C; }
int SGP_CAT(row_threads_, SGP_L)() { return RowCfg<SGP_L>::NT; }
int SGP_CAT(row_pairs_, SGP_L)() { return RowCfg<SGP_L>::RP; }
int SGP_CAT(col_threads_, SGP_L)() { return ColCfg<SGP_L>::NT; }

}  // namespace sgp
