// Host-side launchers of the size-specialised kernels.
#pragma once
#include "common.hpp"

namespace sgp {

bool size_supported(int L);
// Tile variant v (0..3) of the row / column kernels of FFT length L: bit 0
// the workgroup shape, bit 1 the transform plan (points per thread and
// radices), chosen per length by the autotuner (variant 0 by default).
// columns handled by one column-kernel workgroup
int col_width(int L, int v);
int row_threads(int L, int v);
// row pairs handled by one row-kernel workgroup
int row_pairs(int L, int v);
int col_threads(int L, int v);
// the transform plan (0 or 1) that variant v runs
int plan_of(int L, int v);
void launch_row(int L, int v, int op, dim3 grid, const Args& a, hipStream_t s);
void launch_col(int L, int v, int mode, int conj, dim3 grid, const Args& a, hipStream_t s);
void launch_pix(int op, dim3 grid, const Args& a, hipStream_t s);
// second reduction stage of the row iteration kernels (one workgroup per item)
void launch_row_fin(int op, int nz, const Args& a, hipStream_t s);
bool row_fin_deferred(int op);
// the twiddle table of length L in the pass order of plan a's transforms (L entries)
void launch_twiddle(float2* tw, int L, int a, hipStream_t s);
void launch_zero(unsigned* c, int n, hipStream_t s);
void launch_resume(DevState* st, int n, int nitems, hipStream_t s);

}  // namespace sgp
