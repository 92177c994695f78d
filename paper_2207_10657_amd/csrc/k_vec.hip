// Vector kernels of the truncated CG (Algorithm 1): axpy updates of the
// iterate, residual and direction in displacement coordinates, each fused
// with the inner products the next scalar decision needs, and the final
// fixed-order reduction of per-block partial sums.
#include "hfe_internal.h"
#include "hfe_reduce.h"

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

__global__ void __launch_bounds__(kBlock) k_dot(long long n, const double* __restrict__ x,
                                                const double* __restrict__ y,
                                                double* __restrict__ partials) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc[0] += x[i] * y[i];
  block_reduce_store<1>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_cg_zg(long long n, double alpha,
                                                  const double* __restrict__ d,
                                                  const double* __restrict__ Kd,
                                                  double* __restrict__ z,
                                                  double* __restrict__ g) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    z[i] += alpha * d[i];
    g[i] += alpha * Kd[i];
  }
}

__global__ void __launch_bounds__(kBlock) k_cg_y(long long n, double alpha,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ y,
                                                 const double* __restrict__ g,
                                                 double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double yo = y[i];
    const double yn = yo + alpha * w[i];
    y[i] = yn;
    const double gi = g[i];
    acc[0] += yn * gi;
    acc[1] += yo * gi;
  }
  block_reduce_store<2>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_cg_d(long long n, double beta,
                                                 const double* __restrict__ y,
                                                 double* __restrict__ d,
                                                 const double* __restrict__ g,
                                                 const double* __restrict__ z,
                                                 double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    // beta = 0 starts a new direction without reading the old one
    const double dn = beta == 0.0 ? -y[i] : -y[i] + beta * d[i];
    d[i] = dn;
    const double gi = g[i];
    acc[0] += gi * dn;
    acc[1] += z[i] * gi;
  }
  block_reduce_store<2>(acc, partials);
}

// One block; thread t adds rows t, t + 256, ... in order, then a fixed tree.
__global__ void __launch_bounds__(kBlock) k_reduce(const double* __restrict__ partials,
                                                   int nblocks, int nv,
                                                   double* __restrict__ out) {
  __shared__ double sh[kBlock];
  for (int k = 0; k < nv; ++k) {
    double s = 0.0;
    for (int r = threadIdx.x; r < nblocks; r += blockDim.x) s += partials[(size_t)r * nv + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
    __syncthreads();
  }
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

hipError_t vec_dot(long long n, const double* x, const double* y, double* partials,
                   hipStream_t s, int* nblocks) {
  const int nb = vec_blocks(n);
  *nblocks = nb;
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBlock), 0, s, n, x, y, partials);
  return hipGetLastError();
}

hipError_t cg_step_zg(long long n, double alpha, const double* d, const double* Kd, double* z,
                      double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_zg, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, alpha, d, Kd, z, g);
  return hipGetLastError();
}

hipError_t cg_step_y(long long n, double alpha, const double* w, double* y, const double* g,
                     double* partials, hipStream_t s, int* nblocks) {
  const int nb = vec_blocks(n);
  *nblocks = nb;
  hipLaunchKernelGGL(k_cg_y, dim3(nb), dim3(kBlock), 0, s, n, alpha, w, y, g, partials);
  return hipGetLastError();
}

hipError_t cg_step_d(long long n, double beta, const double* y, double* d, const double* g,
                     const double* z, double* partials, hipStream_t s, int* nblocks) {
  const int nb = vec_blocks(n);
  *nblocks = nb;
  hipLaunchKernelGGL(k_cg_d, dim3(nb), dim3(kBlock), 0, s, n, beta, y, d, g, z, partials);
  return hipGetLastError();
}

hipError_t reduce_partials(const double* partials, int nblocks, int nv, double* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, partials, nblocks, nv, out);
  return hipGetLastError();
}

}  // namespace hfe
