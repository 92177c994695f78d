// Vector kernels of the truncated CG (Algorithm 1) in displacement
// coordinates: updates of the iterate, residual and direction, each fused
// with the inner products the next decision needs, and the single-block
// finish kernels that add the per-block partial sums in a fixed order and
// take that decision on the device-resident CgState, so a CG iteration runs
// without a host round trip.
#include "hfe_cg.h"
#include "hfe_internal.h"
#include "hfe_reduce.h"

#include <type_traits>

namespace hfe {
namespace {

constexpr int kVecBlocksMax = 1024;   // grid-stride loops: at most this many blocks

inline int vec_blocks(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b > kVecBlocksMax) b = kVecBlocksMax;
  if (b < 1) b = 1;
  return (int)b;
}

__global__ void __launch_bounds__(kBlock) k_axpy(long long n, double alpha,
                                                 const double* __restrict__ y,
                                                 double* __restrict__ x) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] += alpha * y[i];
}

__global__ void __launch_bounds__(kBlock) k_axpy_to(long long n, const double* __restrict__ x,
                                                    double alpha, const double* __restrict__ y,
                                                    double* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = x[i] + alpha * y[i];
}

// out = alpha x + beta y, elementwise; out may alias x or y (no restrict)
__global__ void __launch_bounds__(kBlock) k_lincomb(long long n, double alpha, const double* x,
                                                    double beta, const double* y, double* out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = alpha * x[i] + beta * y[i];
}

__global__ void __launch_bounds__(kBlock) k_dot(long long n, const double* __restrict__ x,
                                                const double* __restrict__ y, Reducer r) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc[0] += x[i] * y[i];
  block_reduce_store<1>(acc, r.partials);
}

__global__ void __launch_bounds__(kBlock) k_cg_zg(long long n, const double* __restrict__ d,
                                                  const double* __restrict__ Kd,
                                                  double* __restrict__ z,
                                                  double* __restrict__ g,
                                                  const CgState* __restrict__ st) {
  if (st->done) {
    if (!st->apply_tau) return;
    const double tau = st->tau;   // exit on the trust-region sphere: p = z + tau d
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
      z[i] += tau * d[i];
    return;
  }
  const double alpha = st->alpha;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    z[i] += alpha * d[i];
    g[i] += alpha * Kd[i];
  }
}

__global__ void __launch_bounds__(kBlock) k_cg_y(long long n, const double* __restrict__ w,
                                                 double* __restrict__ y,
                                                 const double* __restrict__ g, Reducer r,
                                                 const CgState* st) {
  if (st->done) return;
  const double alpha = st->alpha;
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double yo = y[i];
    const double yn = yo + alpha * w[i];
    y[i] = yn;
    const double gi = g[i];
    acc[0] += yn * gi;   // <r_{j+1}, r_{j+1}>
    acc[1] += yo * gi;   // <r_{j+1}, r_j> (restart test)
  }
  block_reduce_store<2>(acc, r.partials);
}

// d = -y + beta d with the sums {g.d, z.g} (FP64 in either precision). With
// rows_res set, every block first takes the residual decision on its own copy
// of st from the rows of the inverse plane pass (block 0 stores it in st_out).
template <typename R>
__global__ void __launch_bounds__(kBlock) k_cg_d(long long n, const R* __restrict__ y,
                                                 R* __restrict__ d, const R* __restrict__ g,
                                                 const R* __restrict__ z, Reducer r,
                                                 const CgState* st, const double* rows_res,
                                                 int nb_res, CgState* st_out, double* trace) {
  __shared__ CgState sst;
  // the vectors do not depend on the decision: the first kPre elements of
  // this thread are loaded before the row sums, so the latencies overlap
  constexpr int kPre = 4;
  const long long first = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  R py[kPre], pd[kPre], pz[kPre];
  double pg[kPre];
  auto load_round = [&](long long base) {
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const long long i = base + u * stride;
      if (i < n) {
        py[u] = y[i];
        pd[u] = d[i];
        pg[u] = g[i];
        pz[u] = z[i];
      }
    }
  };
  if (!st->done) load_round(first);
  copy_state_block(&sst, st);
  __syncthreads();
  if (rows_res) {
    if (!sst.done) {
      double t[2];
      block_sum_rows<2>(rows_res, nb_res, t);
      if (threadIdx.x == 0) {
        cg_decide_residual(&sst, blockIdx.x == 0 ? trace : nullptr, t[0], t[1]);
        cg_tail_direction(&sst);
      }
    } else if (threadIdx.x == 0) {
      sst.apply_tau = 0;   // the exit step was formed by the forward plane pass
    }
    __syncthreads();
    if (blockIdx.x == 0) copy_state_block(st_out, &sst);
  }
  if (sst.done) return;
  const R beta = (R)sst.beta;
  double acc[2] = {0.0, 0.0};
  for (long long base = first; base < n; base += kPre * stride) {
    if (base != first) load_round(base);
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const long long i = base + u * stride;
      if (i < n) {
        // beta = 0 starts a new direction without using the old one
        const R dn = beta == R(0) ? -py[u] : -py[u] + beta * pd[u];
        d[i] = dn;
        const double gi = pg[u];
        acc[0] += gi * (double)dn;       // <r, d>
        acc[1] += (double)pz[u] * gi;    // z . g for <z, d>
      }
    }
  }
  block_reduce_store<2>(acc, r.partials);
}

__global__ void __launch_bounds__(kBlock) k_cg_start(long long n, const double* __restrict__ g0,
                                                     const double* __restrict__ y0,
                                                     double* __restrict__ z, double* __restrict__ g,
                                                     double* __restrict__ y, double* __restrict__ d,
                                                     Reducer r) {
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double gi = g0[i], yi = y0[i];
    const double dn = -yi;
    z[i] = 0.0;
    g[i] = gi;
    y[i] = yi;
    d[i] = dn;
    acc[0] += gi * dn;
    acc[1] += 0.0 * gi;   // z . g with z = 0, as in k_cg_d
  }
  block_reduce_store<2>(acc, r.partials);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_dot_t(long long n, const R* __restrict__ x,
                                                  const R* __restrict__ y, Reducer r) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc[0] += (double)x[i] * (double)y[i];
  block_reduce_store<1>(acc, r.partials);
}

template <typename S, typename D>
__global__ void __launch_bounds__(kBlock) k_convert(long long n, const S* __restrict__ x,
                                                    D* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = (D)x[i];
}

// out = x + y rounded to FP32, the sum taken in FP64
__global__ void __launch_bounds__(kBlock) k_add_f32(long long n, const float* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    float* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (float)((double)x[i] + y[i]);
}

// Fixed-order sum of nblocks rows of nv partials (one block), then the action.
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_finish(Reducer r, int nblocks, int nv,
                                                   double* __restrict__ out, CgState* st,
                                                   double* trace) {
  if (KIND != FIN_OUT && st->done) {
    // the exit step (if any) was formed by k_cg_zg earlier in this iteration
    if (KIND == FIN_RESIDUAL) st->apply_tau = 0;
    return;
  }
  __shared__ double wsum[kBlock / 64][kMaxPartials];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the row widths in use get all their columns loaded together
  auto cols = [&](auto nvc) {
    constexpr int NV = decltype(nvc)::value;
    double sk[NV];
    strided_row_sums<NV>(r.partials, nblocks, threadIdx.x, blockDim.x, sk);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double t = wave_sum(sk[k]);
      if (lane == 0) wsum[wave][k] = t;
    }
  };
  switch (nv) {
    case 1: cols(std::integral_constant<int, 1>()); break;
    case 2: cols(std::integral_constant<int, 2>()); break;
    case TRI_NV: cols(std::integral_constant<int, TRI_NV>()); break;
    case RES_NV: cols(std::integral_constant<int, RES_NV>()); break;
    default:
      for (int k = 0; k < nv; ++k) {
        double t = strided_row_sum(r.partials, nblocks, nv, k, threadIdx.x, blockDim.x);
        t = wave_sum(t);
        if (lane == 0) wsum[wave][k] = t;
      }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[kMaxPartials];
  for (int k = 0; k < nv; ++k) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += wsum[w][k];
    tot[k] = s;
  }
  if (KIND == FIN_OUT) {
    for (int k = 0; k < nv; ++k) out[k] = tot[k];
  } else if (KIND == FIN_CURVATURE) {
    cg_decide_curvature(st, trace, tot[0], tot[1]);
  } else if (KIND == FIN_RESIDUAL) {
    cg_decide_residual(st, trace, tot[0], tot[1]);
  } else {
    cg_decide_direction(st, tot[0], tot[1]);
  }
}

// Fixed-order sum of nb rows of 2 partials into thread 0's tot (one block).
__device__ __forceinline__ void sum_rows2(const double* __restrict__ rows, int nb, double (&tot)[2]) {
  __shared__ double wsum[kBlock / 64][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s[2];
  strided_row_sums<2>(rows, nb, threadIdx.x, blockDim.x, s);
  for (int k = 0; k < 2; ++k) {
    const double sk = wave_sum(s[k]);
    if (lane == 0) wsum[wave][k] = sk;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 2; ++k) {
      double s = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) s += wsum[w][k];
      tot[k] = s;
    }
  }
  __syncthreads();
}

// The direction update of the previous iteration, then the curvature decision
// of this one (both need the state in this order).
__global__ void __launch_bounds__(kBlock) k_finish_dc(Reducer rd, int nbd, Reducer rc, int nbc,
                                                      CgState* st, double* trace) {
  if (st->done) return;
  double td[2], tc[2];
  sum_rows2(rd.partials, nbd, td);
  sum_rows2(rc.partials, nbc, tc);
  if (threadIdx.x != 0) return;
  cg_decide_direction(st, td[0], td[1]);
  cg_decide_curvature(st, trace, tc[0], tc[1]);
}

__global__ void k_cg_resume(CgState* st) {
  st->beta = 0.0;
  st->restart = 0;
  st->done = 0;
  st->flag = CG_RUN;
}

}  // namespace

hipError_t vec_axpy(long long n, double alpha, const double* y, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, alpha, y, x);
  return hipGetLastError();
}

hipError_t vec_axpy_to(long long n, const double* x, double alpha, const double* y, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_to, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, x, alpha, y, out);
  return hipGetLastError();
}

hipError_t cg_start(long long n, const double* g0, const double* y0, double* z, double* g,
                    double* y, double* d, const Reducer& r, hipStream_t s, int* nblocks) {
  *nblocks = vec_blocks(n);
  hipLaunchKernelGGL(k_cg_start, dim3(*nblocks), dim3(kBlock), 0, s, n, g0, y0, z, g, y, d, r);
  return hipGetLastError();
}

hipError_t vec_lincomb(long long n, double alpha, const double* x, double beta, const double* y,
                       double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, alpha, x, beta, y, out);
  return hipGetLastError();
}

hipError_t vec_dot(long long n, const double* x, const double* y, const Reducer& r,
                   hipStream_t s, int* nblocks) {
  *nblocks = vec_blocks(n);
  hipLaunchKernelGGL(k_dot, dim3(*nblocks), dim3(kBlock), 0, s, n, x, y, r);
  return hipGetLastError();
}

hipError_t cg_step_zg(long long n, const double* d, const double* Kd, double* z, double* g,
                      CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_zg, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, d, Kd, z, g, st);
  return hipGetLastError();
}

hipError_t cg_step_y(long long n, const double* w, double* y, const double* g, const Reducer& r,
                     const CgState* st, hipStream_t s, int* nblocks) {
  *nblocks = vec_blocks(n);
  hipLaunchKernelGGL(k_cg_y, dim3(*nblocks), dim3(kBlock), 0, s, n, w, y, g, r, st);
  return hipGetLastError();
}

template <typename R>
hipError_t cg_step_d(long long n, const R* y, R* d, const R* g, const R* z, const Reducer& r,
                     const CgState* st, hipStream_t s, int* nblocks, const double* rows_res,
                     int nb_res, CgState* st_out, double* trace) {
  if (rows_res && (!st_out || nb_res < 1)) return hipErrorInvalidValue;
  *nblocks = vec_blocks(n);
  hipLaunchKernelGGL((k_cg_d<R>), dim3(*nblocks), dim3(kBlock), 0, s, n, y, d, g, z, r, st,
                     rows_res, nb_res, st_out, trace);
  return hipGetLastError();
}
template hipError_t cg_step_d<double>(long long, const double*, double*, const double*,
                                      const double*, const Reducer&, const CgState*, hipStream_t,
                                      int*, const double*, int, CgState*, double*);
template hipError_t cg_step_d<float>(long long, const float*, float*, const float*, const float*,
                                     const Reducer&, const CgState*, hipStream_t, int*,
                                     const double*, int, CgState*, double*);

hipError_t vec_dot_f32(long long n, const float* x, const float* y, const Reducer& r,
                       hipStream_t s, int* nblocks) {
  *nblocks = vec_blocks(n);
  hipLaunchKernelGGL((k_dot_t<float>), dim3(*nblocks), dim3(kBlock), 0, s, n, x, y, r);
  return hipGetLastError();
}

hipError_t vec_to_f32(long long n, const double* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, float>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, x, y);
  return hipGetLastError();
}

hipError_t vec_to_f64(long long n, const float* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<float, double>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, x, y);
  return hipGetLastError();
}

hipError_t vec_add_f32(long long n, const float* x, const double* y, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f32, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, x, y, out);
  return hipGetLastError();
}

hipError_t finish(int kind, const Reducer& r, int nblocks, int nv, double* out, CgState* st,
                  double* trace, hipStream_t s) {
  switch (kind) {
    case FIN_OUT:
      hipLaunchKernelGGL(k_finish<FIN_OUT>, dim3(1), dim3(kBlock), 0, s, r, nblocks, nv, out, st, trace);
      break;
    case FIN_CURVATURE:
      hipLaunchKernelGGL(k_finish<FIN_CURVATURE>, dim3(1), dim3(kBlock), 0, s, r, nblocks, nv, out, st, trace);
      break;
    case FIN_RESIDUAL:
      hipLaunchKernelGGL(k_finish<FIN_RESIDUAL>, dim3(1), dim3(kBlock), 0, s, r, nblocks, nv, out, st, trace);
      break;
    default:
      hipLaunchKernelGGL(k_finish<FIN_DIRECTION>, dim3(1), dim3(kBlock), 0, s, r, nblocks, nv, out, st, trace);
      break;
  }
  return hipGetLastError();
}

hipError_t finish_direction_curvature(const Reducer& rd, int nbd, const Reducer& rc, int nbc,
                                      CgState* st, double* trace, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_dc, dim3(1), dim3(kBlock), 0, s, rd, nbd, rc, nbc, st, trace);
  return hipGetLastError();
}

hipError_t cg_resume(CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_resume, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

}  // namespace hfe
