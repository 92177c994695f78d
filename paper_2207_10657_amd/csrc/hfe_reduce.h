// Deterministic block reductions: every block writes one row of NV partial
// sums; a single-block kernel later adds the rows in a fixed order. The order
// of every addition is fixed by the launch shape, so repeated runs give the
// same bits.
#pragma once

#include <hip/hip_runtime.h>

#include "hfe_internal.h"

namespace hfe {

// Sum over the 64 lanes of a wavefront (butterfly with xor shuffles).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Reduce acc[NV] over the block (blockDim.x a multiple of 64, at most 1024)
// and store the block's row partials[blockIdx.x * NV + k].
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double* partials,
                                                   int row = -1) {
  __shared__ double red[16][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += red[w][threadIdx.x];
    partials[(size_t)(row < 0 ? (int)blockIdx.x : row) * NV + threadIdx.x] = s;
  }
}

// Fixed-order sum of nb rows of NV partials, done by the first 256 threads
// of the block so that the order of the additions does not depend on the
// block size (blockDim.x >= 256). The totals end in thread 0's tot. Every
// thread of the block must call it.
template <int NV>
__device__ __forceinline__ void block_sum_rows(const double* __restrict__ rows, int nb,
                                               double (&tot)[NV]) {
  __shared__ double ws[4][NV];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < 256) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int r = tid; r < nb; r += 256) s += rows[(size_t)r * NV + k];
      s = wave_sum(s);
      if (lane == 0) ws[wave][k] = s;
    }
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = ((ws[0][k] + ws[1][k]) + ws[2][k]) + ws[3][k];
  }
  __syncthreads();
}

}  // namespace hfe
