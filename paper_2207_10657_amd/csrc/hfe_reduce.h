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
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double* partials) {
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
    partials[(size_t)blockIdx.x * NV + threadIdx.x] = s;
  }
}

}  // namespace hfe

namespace hfe {

// Block reduction followed by the final reduction in the last block.
// Returns true in the last block; its thread 0 then holds the grid totals in
// `total` (other threads: unspecified). The counter is reset for the next
// kernel on the stream.
template <int NV>
__device__ __forceinline__ bool block_reduce_last(double (&acc)[NV], const Reducer& r,
                                                  double (&total)[NV]) {
  block_reduce_store<NV>(acc, r.partials);
  __shared__ int am_last;
  __shared__ double wsum[16][NV];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int t = atomicAdd(r.counter, 1u);
    am_last = (t == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!am_last) return false;
  __threadfence();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int row = threadIdx.x; row < (int)gridDim.x; row += blockDim.x)
      s += __builtin_nontemporal_load(&r.partials[(size_t)row * NV + k]);
    s = wave_sum(s);
    if (lane == 0) wsum[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nwaves; ++w) s += wsum[w][k];
      total[k] = s;
    }
    *r.counter = 0u;
  }
  return true;
}

}  // namespace hfe
