// Host-side launchers of the size-specialised kernels.
#pragma once
#include "common.hpp"

namespace sgp {

bool size_supported(int L);
// columns handled by one column-kernel workgroup for FFT length L
int col_width(int L);
int row_threads(int L);
// row pairs handled by one row-kernel workgroup for row length L
int row_pairs(int L);
int col_threads(int L);
void launch_row(int L, int op, dim3 grid, const Args& a, hipStream_t s);
void launch_col(int L, int mode, int conj, dim3 grid, const Args& a, hipStream_t s);
void launch_pix(int op, dim3 grid, const Args& a, hipStream_t s);
// second reduction stage of the row iteration kernels (one workgroup per item)
void launch_row_fin(int op, int nz, const Args& a, hipStream_t s);
bool row_fin_deferred(int op);
void launch_twiddle(float2* tw, int L, hipStream_t s);
void launch_resume(DevState* st, int n, int nitems, hipStream_t s);

}  // namespace sgp
