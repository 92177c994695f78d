// Deterministic reductions: every block (or, for the Hessian, every
// canonical tile) writes one row of NV partial sums; a single block later
// adds the rows in a fixed order. Where a kernel has launch shapes to choose
// from (the Hessian, the fused FFT passes), the order of every addition is
// independent of the shape, so every shape gives the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include "hfe_internal.h"

namespace hfe {


// The value of lane i ^ 32 and of lane i ^ 16 (gfx950 permlane swaps: with
// both operands v, the swap's second result holds the upper half-wave's
// values in the lower lanes and its first result the lower half's in the
// upper lanes; the 16-lane swap does the same between neighbouring rows).
__device__ __forceinline__ unsigned int lane_xor32(unsigned int v) {
  const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return (threadIdx.x & 32) ? r[0] : r[1];
}
__device__ __forceinline__ unsigned int lane_xor16(unsigned int v) {
  const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return (threadIdx.x & 16) ? r[0] : r[1];
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront: the butterfly that adds lane i ^ 32,
// then i ^ 16, 8, 4, 2, 1 (every lane ends with the same value). The
// exchanges run in registers (permlane swaps for 32 and 16; DPP row_ror:8,
// which is i ^ 8 within a row; row_ror:4, which gives the value of i ^ 4
// once values depend on i mod 8 only; quad perms for 2 and 1), with the
// bits of the shuffle form of the same butterfly. Every lane must take part.
__device__ __forceinline__ double wave_sum(double v) {
  {
    const long long b = __double_as_longlong(v);
    const unsigned int lo = lane_xor32((unsigned int)b), hi = lane_xor32((unsigned int)(b >> 32));
    v += __longlong_as_double(((long long)hi << 32) | lo);
  }
  {
    const long long b = __double_as_longlong(v);
    const unsigned int lo = lane_xor16((unsigned int)b), hi = lane_xor16((unsigned int)(b >> 32));
    v += __longlong_as_double(((long long)hi << 32) | lo);
  }
  v += dpp_mov<0x128>(v);   // row_ror:8
  v += dpp_mov<0x124>(v);   // row_ror:4
  v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  return v;
}

// Cross-lane sums by DPP (no LDS traffic). dpp_add<CTRL, ROWS> adds to v the
// value of the lane the DPP control selects; lanes of rows (16 lanes each)
// outside the row mask add 0. A double moves as its two 32-bit halves under
// the same control. Floating-point addition is commutative, so after each of
// the symmetric steps below every lane of the group holds the same value.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each row of 16 lanes, in every lane of the row: lane pairs (xor 1),
// quads (xor 2), half-rows (mirror within 8), the two half-rows (mirror
// within 16).
__device__ __forceinline__ double row16_sum(double v) {
  v = dpp_add<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v = dpp_add<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v = dpp_add<0x141>(v);   // row_half_mirror
  v = dpp_add<0x140>(v);   // row_mirror
  return v;
}

// Sum of a canonical tile's 32 column sums (hfe_internal.h), held by the
// lanes of a half-wave whose bits 0..4 are q = x + 8 y: each row of 16, then
// the second row adds the first (row_bcast:15). The tile's sum is in the
// half-wave's lanes q = 16..31; the halves do not mix. Every lane of the
// wave must take part.
__device__ __forceinline__ double tile_sum32(double v) {
  v = row16_sum(v);
  return dpp_add<0x142, 0xa>(v);
}

// Sum over the 64 lanes of a wave in lane 63 (the other lanes hold partial
// sums): each half-wave as in tile_sum32, then the upper half adds the lower
// half's sum (row_bcast:31).
__device__ __forceinline__ double wave_total63(double v) {
  v = tile_sum32(v);
  return dpp_add<0x143, 0xc>(v);
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

// Thread t's share of a fixed-order row sum: s[k] = the sum, in ascending r,
// of rows[r * NV + k] over r = t, t + stride, ... < nb. The rows are loaded
// in batches of 8 before they are added (in the same order), so a thread
// waits for one memory latency per batch instead of one per row.
template <int NV>
__device__ __forceinline__ void strided_row_sums(const double* __restrict__ rows, int nb, int t,
                                                 int stride, double (&s)[NV]) {
  constexpr int kB = 8;
#pragma unroll
  for (int k = 0; k < NV; ++k) s[k] = 0.0;
  for (int r0 = t; r0 < nb; r0 += kB * stride) {
    double v[kB][NV];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int r = r0 + u * stride;
#pragma unroll
      for (int k = 0; k < NV; ++k) v[u][k] = r < nb ? rows[(size_t)r * NV + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (r0 + u * stride < nb) {
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += v[u][k];
      }
  }
}

// The same for a row length nv known at run time, one column k.
__device__ __forceinline__ double strided_row_sum(const double* __restrict__ rows, int nb, int nv,
                                                  int k, int t, int stride) {
  constexpr int kB = 8;
  double s = 0.0;
  for (int r0 = t; r0 < nb; r0 += kB * stride) {
    double v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int r = r0 + u * stride;
      v[u] = r < nb ? rows[(size_t)r * nv + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (r0 + u * stride < nb) s += v[u];
  }
  return s;
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
    double s[NV];
    strided_row_sums<NV>(rows, nb, tid, 256, s);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double sk = wave_sum(s[k]);
      if (lane == 0) ws[wave][k] = sk;
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
