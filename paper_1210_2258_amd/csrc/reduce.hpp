// Deterministic two-stage FP64 reductions.
//
// Every workgroup reduces its per-thread accumulators with wavefront shuffles
// and writes one partial per slot; the last workgroup to arrive (counted with
// a device-scope atomic) sums the partials in a fixed order, so the result is
// bitwise reproducible run to run, and hands the totals to a finaliser that
// updates the solver state.  No float atomics are used.
#pragma once
#include <hip/hip_runtime.h>

namespace sgp {

enum { RED_SUM = 0, RED_MIN = 1, RED_MAX = 2 };

__device__ __forceinline__ double red_combine(int kind, double a, double b) {
  return kind == RED_SUM ? a + b : (kind == RED_MIN ? fmin(a, b) : fmax(a, b));
}
__device__ __forceinline__ double red_identity(int kind) {
  return kind == RED_SUM ? 0.0 : (kind == RED_MIN ? __builtin_inf() : -__builtin_inf());
}

template <int NT>
__device__ __forceinline__ double wave_reduce(int kind, double v) {
  constexpr int W = NT < 64 ? NT : 64;
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v = red_combine(kind, v, __shfl_xor(v, off, W));
  return v;
}

// Reduces acc[0..NS) over the grid.  Returns true in exactly one thread
// (thread 0 of the last workgroup) with tot[] holding the grid totals.
// kinds(s) gives the reduction kind of slot s.  Must be called by every thread
// of every participating workgroup.
template <int NT, int NS, class Kinds>
__device__ bool grid_reduce(double (&acc)[NS], Kinds kinds, double* part, unsigned* counter,
                            int nblk, int bid, double (&tot)[NS]) {
  constexpr int NW = NT < 64 ? 1 : NT / 64;
  __shared__ double sh[NS][NW];
  __shared__ int is_last;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double v = wave_reduce<NT>(kinds(s), acc[s]);
    if (lane == 0) sh[s][wave] = v;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double v = sh[s][0];
      for (int w = 1; w < NW; ++w) v = red_combine(kinds(s), v, sh[s][w]);
      part[(size_t)s * nblk + bid] = v;
    }
    __threadfence();
    unsigned prev = atomicAdd(counter, 1u);
    is_last = (prev == (unsigned)(nblk - 1));
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
  double loc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) loc[s] = red_identity(kinds(s));
  for (int i = tid; i < nblk; i += NT) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double v = __hip_atomic_load(&part[(size_t)s * nblk + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      loc[s] = red_combine(kinds(s), loc[s], v);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double v = wave_reduce<NT>(kinds(s), loc[s]);
    if (lane == 0) sh[s][wave] = v;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double v = sh[s][0];
      for (int w = 1; w < NW; ++w) v = red_combine(kinds(s), v, sh[s][w]);
      tot[s] = v;
    }
    atomicExch(counter, 0u);
    return true;
  }
  return false;
}

// First stage only: thread 0 of each workgroup writes the workgroup's partial
// of every slot.  No cross-workgroup synchronisation: a later launch sums the
// partials (sum_partials), the kernel boundary making them visible.
template <int NT, int NS, class Kinds>
__device__ void block_partials(double (&acc)[NS], Kinds kinds, double* part, int nblk, int bid) {
  constexpr int NW = NT < 64 ? 1 : NT / 64;
  __shared__ double sh[NS][NW];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double v = wave_reduce<NT>(kinds(s), acc[s]);
    if (lane == 0) sh[s][wave] = v;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double v = sh[s][0];
      for (int w = 1; w < NW; ++w) v = red_combine(kinds(s), v, sh[s][w]);
      part[(size_t)s * nblk + bid] = v;
    }
  }
}

// Second stage in one workgroup of NT threads: the totals of nblk partials
// per slot, summed in a fixed order.  Must be called by every thread; tot is
// valid in thread 0.
template <int NT, int NS, class Kinds>
__device__ void sum_partials(Kinds kinds, const double* part, int nblk, double (&tot)[NS]) {
  constexpr int NW = NT < 64 ? 1 : NT / 64;
  __shared__ double sh[NS][NW];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  double loc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) loc[s] = red_identity(kinds(s));
  for (int i = tid; i < nblk; i += NT) {
#pragma unroll
    for (int s = 0; s < NS; ++s) loc[s] = red_combine(kinds(s), loc[s], part[(size_t)s * nblk + i]);
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double v = wave_reduce<NT>(kinds(s), loc[s]);
    if (lane == 0) sh[s][wave] = v;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double v = sh[s][0];
      for (int w = 1; w < NW; ++w) v = red_combine(kinds(s), v, sh[s][w]);
      tot[s] = v;
    }
  }
}

}  // namespace sgp
