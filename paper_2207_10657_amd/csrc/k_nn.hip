// Kernels of the learned warm start: a small 3D convolutional network on the
// periodic voxel grid that predicts the displacement increment of a load
// step from the cell's state, with its training. Activations and weights are
// stored in BF16; the convolutions accumulate their products in FP32, the
// weight-gradient sums over all voxels in FP64; gradients and the Adam
// moments are FP32 (master weights in FP32, a BF16 copy for the forward
// passes).
//
// Layout: fields are channels-major [C][nz][ny][nx], x fastest; a 3x3x3
// filter bank is [cout][cin][27] with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1);
// the grid is periodic (the cell is), so every tap wraps.
//
// All reductions (weight gradients, the loss) add per-block partial sums in
// a fixed order, so training runs give the same bits every time.
#include <hip/hip_runtime.h>
#include <cstdint>
#include <mutex>

#include "hfe_internal.h"
#include "hfe_reduce.h"

namespace hfe {
namespace {

// BF16 = the upper 16 bits of an IEEE binary32 value; conversion rounds to
// nearest, ties to even (NaN stays NaN).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int kNnBlock = 256;

__device__ __forceinline__ int wrapi(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// out[co][v] = b[co] + sum_{ci, t} w[co][ci][t] in[ci][v + off(t)]; optional
// ReLU; FP32 result (and a BF16 copy when out16 is set). Weights of the
// block in LDS as FP32.
template <int CIN, int COUT>
__global__ void __launch_bounds__(kNnBlock) k_conv_fwd(const uint16_t* __restrict__ in,
                                                      const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias,
                                                      int nx, int ny, int nz, int relu,
                                                      float* __restrict__ out,
                                                      uint16_t* __restrict__ out16) {
  constexpr int cin = CIN, cout = COUT;
  __shared__ float sw[COUT * CIN * 27];   // [cout][cin][27]
  constexpr int nw = cout * cin * 27;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) sw[i] = from_bf16(w[i]);
  __syncthreads();
  const long long N = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
  float acc[COUT];
#pragma unroll
  for (int co = 0; co < cout; ++co) acc[co] = bias ? bias[co] : 0.f;
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const long long u = (long long)wrapi(x + dx, nx) +
                        (long long)nx * (wrapi(y + dy, ny) + (long long)ny * wrapi(z + dz, nz));
#pragma unroll
    for (int ci = 0; ci < cin; ++ci) {
      const float a = from_bf16(in[(long long)ci * N + u]);
#pragma unroll
      for (int co = 0; co < cout; ++co) acc[co] += sw[(co * cin + ci) * 27 + t] * a;
    }
  }
#pragma unroll
  for (int co = 0; co < cout; ++co) {
    float r = acc[co];
    if (relu) r = fmaxf(r, 0.f);
    out[(long long)co * N + v] = r;
    if (out16) out16[(long long)co * N + v] = to_bf16(r);
  }
}

// gin[ci][v] = sum_{co, t} w[co][ci][t] g[co][v - off(t)] (the adjoint of the
// convolution), g masked by (act > 0) when act is set (ReLU backward).
template <int CIN, int COUT>
__global__ void __launch_bounds__(kNnBlock) k_conv_bwd_data(const float* __restrict__ g,
                                                           const float* __restrict__ act,
                                                           const uint16_t* __restrict__ w,
                                                           int nx, int ny, int nz,
                                                           float* __restrict__ gin) {
  constexpr int cin = CIN, cout = COUT;
  __shared__ float sw[COUT * CIN * 27];
  constexpr int nw = cout * cin * 27;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) sw[i] = from_bf16(w[i]);
  __syncthreads();
  const long long N = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
  float acc[CIN];
#pragma unroll
  for (int ci = 0; ci < cin; ++ci) acc[ci] = 0.f;
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const long long u = (long long)wrapi(x - dx, nx) +
                        (long long)nx * (wrapi(y - dy, ny) + (long long)ny * wrapi(z - dz, nz));
#pragma unroll
    for (int co = 0; co < cout; ++co) {
      float gg = g[(long long)co * N + u];
      if (act && !(act[(long long)co * N + u] > 0.f)) gg = 0.f;
#pragma unroll
      for (int ci = 0; ci < cin; ++ci) acc[ci] += sw[(co * cin + ci) * 27 + t] * gg;
    }
  }
#pragma unroll
  for (int ci = 0; ci < cin; ++ci) gin[(long long)ci * N + v] = acc[ci];
}

// Wide layers, whose filter bank does not fit the LDS of the kernels above
// (the 64-channel levels of the widening encoder-decoder): a block computes a
// tile of CT channels (outputs of the convolution, inputs of its adjoint) for
// its voxels, with cin and cout runtime values, and reads the weights from
// global memory at addresses uniform across the block (they stay in the
// caches). The additions run in the same order as in k_conv_fwd and
// k_conv_bwd_data: taps outer, then channels.
constexpr int kWideTile = 16;

__global__ void __launch_bounds__(kNnBlock) k_conv_fwd_wide(const uint16_t* __restrict__ in,
                                                           int cin,
                                                           const uint16_t* __restrict__ w,
                                                           const float* __restrict__ bias,
                                                           int cout, int nx, int ny, int nz,
                                                           int relu, float* __restrict__ out,
                                                           uint16_t* __restrict__ out16) {
  constexpr int CT = kWideTile;
  const int co0 = blockIdx.y * CT;
  const long long N = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
  float acc[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) acc[c] = (bias && co0 + c < cout) ? bias[co0 + c] : 0.f;
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const long long u = (long long)wrapi(x + dx, nx) +
                        (long long)nx * (wrapi(y + dy, ny) + (long long)ny * wrapi(z + dz, nz));
    for (int ci = 0; ci < cin; ++ci) {
      const float a = from_bf16(in[(long long)ci * N + u]);
#pragma unroll
      for (int c = 0; c < CT; ++c)
        if (co0 + c < cout) acc[c] += from_bf16(w[((co0 + c) * cin + ci) * 27 + t]) * a;
    }
  }
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (co0 + c >= cout) break;
    float r = acc[c];
    if (relu) r = fmaxf(r, 0.f);
    out[(long long)(co0 + c) * N + v] = r;
    if (out16) out16[(long long)(co0 + c) * N + v] = to_bf16(r);
  }
}

__global__ void __launch_bounds__(kNnBlock) k_conv_bwd_data_wide(const float* __restrict__ g,
                                                                int cout,
                                                                const float* __restrict__ act,
                                                                const uint16_t* __restrict__ w,
                                                                int cin, int nx, int ny, int nz,
                                                                float* __restrict__ gin) {
  constexpr int CT = kWideTile;
  const int ci0 = blockIdx.y * CT;
  const long long N = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
  float acc[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) acc[c] = 0.f;
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const long long u = (long long)wrapi(x - dx, nx) +
                        (long long)nx * (wrapi(y - dy, ny) + (long long)ny * wrapi(z - dz, nz));
    for (int co = 0; co < cout; ++co) {
      float gg = g[(long long)co * N + u];
      if (act && !(act[(long long)co * N + u] > 0.f)) gg = 0.f;
#pragma unroll
      for (int c = 0; c < CT; ++c)
        if (ci0 + c < cin) acc[c] += from_bf16(w[(co * cin + ci0 + c) * 27 + t]) * gg;
    }
  }
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (ci0 + c >= cin) break;
    gin[(long long)(ci0 + c) * N + v] = acc[c];
  }
}

// One block per (co, ci): rows of partial sums over voxels for the 27 taps,
// gw[co][ci][t] = sum_v gm[co][v] in[ci][v + off(t)], and (ci == 0) the bias
// gradient sum_v gm[co][v]; gm = g masked by (act > 0) when act is set.
__global__ void __launch_bounds__(kNnBlock) k_conv_bwd_w(const float* __restrict__ g, int cout,
                                                        const float* __restrict__ act,
                                                        const uint16_t* __restrict__ in, int cin,
                                                        int nx, int ny, int nz,
                                                        float* __restrict__ gw,
                                                        float* __restrict__ gb) {
  const int co = blockIdx.x / cin, ci = blockIdx.x % cin;
  const long long N = (long long)nx * ny * nz;
  double acc[28];
#pragma unroll
  for (int t = 0; t < 28; ++t) acc[t] = 0.0;
  for (long long v = threadIdx.x; v < N; v += blockDim.x) {
    float gg = g[(long long)co * N + v];
    if (act && !(act[(long long)co * N + v] > 0.f)) gg = 0.f;
    if (gg == 0.f) continue;
    const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      const long long u = (long long)wrapi(x + dx, nx) +
                          (long long)nx * (wrapi(y + dy, ny) + (long long)ny * wrapi(z + dz, nz));
      acc[t] += (double)(gg * from_bf16(in[(long long)ci * N + u]));
    }
    acc[27] += (double)gg;
  }
  // fixed-order block reduction of the 28 sums
  __shared__ double red[kNnBlock / 64][28];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < 28; ++t) {
    const double s = wave_sum(acc[t]);
    if (lane == 0) red[wave][t] = s;
  }
  __syncthreads();
  if (threadIdx.x < 28) {
    double s = 0.0;
    for (int wv = 0; wv < kNnBlock / 64; ++wv) s += red[wv][threadIdx.x];
    if (threadIdx.x < 27) gw[(co * cin + ci) * 27 + threadIdx.x] = (float)s;
    else if (ci == 0 && gb) gb[co] = (float)s;
  }
}

// grad = 2 (pred - target) / n, rows of partial sums of (pred - target)^2
__global__ void __launch_bounds__(kNnBlock) k_mse(const float* __restrict__ pred,
                                                 const float* __restrict__ target, long long n,
                                                 float* __restrict__ grad, double* partials) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float d = pred[i] - target[i];
    grad[i] = 2.f * d / (float)n;
    acc[0] += (double)d * (double)d;
  }
  block_reduce_store<1>(acc, partials);
}

__global__ void __launch_bounds__(kNnBlock) k_sum_rows(const double* __restrict__ partials, int nb,
                                                      long long n, double* out) {
  double t[1];
  block_sum_rows<1>(partials, nb, t);
  if (threadIdx.x == 0) *out = t[0] / (double)n;
}

// Adam on FP32 master weights; the BF16 copy for the forward passes.
__global__ void __launch_bounds__(kNnBlock) k_adam(float* __restrict__ w, float* __restrict__ m,
                                                  float* __restrict__ v,
                                                  const float* __restrict__ g, long long n,
                                                  float lr, float b1, float b2, float eps,
                                                  float c1, float c2, uint16_t* __restrict__ w16) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (w16) w16[i] = to_bf16(wi);
  }
}

// 2x2x2 mean pooling of c channels on a fine grid (nx, ny, nz even): one
// thread per coarse voxel and channel; the 8 children are added in a fixed
// order in FP32 and divided by 8 (exact).
__global__ void __launch_bounds__(kNnBlock) k_pool2(const float* __restrict__ in, int c, int nx,
                                                   int ny, int nz, float* __restrict__ out,
                                                   uint16_t* __restrict__ out16) {
  const int mx = nx / 2, my = ny / 2, mz = nz / 2;
  const long long M = (long long)mx * my * mz, N = (long long)nx * ny * nz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M * c;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i / M);
    const long long r = i - (long long)ch * M;
    const int x = (int)(r % mx), y = (int)((r / mx) % my), z = (int)(r / ((long long)mx * my));
    const float* src = in + (long long)ch * N;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int fx = 2 * x + (k & 1), fy = 2 * y + ((k >> 1) & 1), fz = 2 * z + ((k >> 2) & 1);
      s += src[fx + (long long)nx * (fy + (long long)ny * fz)];
    }
    s *= 0.125f;
    if (out) out[i] = s;
    if (out16) out16[i] = to_bf16(s);
  }
}

// gin (fine) += the adjoint of k_pool2 applied to g (coarse): g / 8 to each
// of the 8 children.
__global__ void __launch_bounds__(kNnBlock) k_pool2_bwd(const float* __restrict__ g, int c, int nx,
                                                       int ny, int nz, float* __restrict__ gin) {
  const long long N = (long long)nx * ny * nz;
  const int mx = nx / 2, my = ny / 2;
  const long long M = (long long)mx * my * (nz / 2);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N * c;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i / N);
    const long long r = i - (long long)ch * N;
    const int x = (int)(r % nx), y = (int)((r / nx) % ny), z = (int)(r / ((long long)nx * ny));
    gin[i] += 0.125f * g[(long long)ch * M + x / 2 + (long long)mx * (y / 2 + (long long)my * (z / 2))];
  }
}

// Nearest doubling of every axis: coarse (mx, my, mz) -> fine, c channels.
__global__ void __launch_bounds__(kNnBlock) k_upsample2(const float* __restrict__ in, int c, int mx,
                                                       int my, int mz, float* __restrict__ out,
                                                       uint16_t* __restrict__ out16) {
  const int nx = 2 * mx, ny = 2 * my;
  const long long N = (long long)nx * ny * (2 * mz), M = (long long)mx * my * mz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N * c;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i / N);
    const long long r = i - (long long)ch * N;
    const int x = (int)(r % nx), y = (int)((r / nx) % ny), z = (int)(r / ((long long)nx * ny));
    const float v = in[(long long)ch * M + x / 2 + (long long)mx * (y / 2 + (long long)my * (z / 2))];
    if (out) out[i] = v;
    if (out16) out16[i] = to_bf16(v);
  }
}

// The adjoint of k_upsample2: gin (coarse) = sum over the 8 children of g.
__global__ void __launch_bounds__(kNnBlock) k_upsample2_bwd(const float* __restrict__ g, int c,
                                                           int mx, int my, int mz,
                                                           float* __restrict__ gin) {
  const int nx = 2 * mx, ny = 2 * my;
  const long long N = (long long)nx * ny * (2 * mz), M = (long long)mx * my * mz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M * c;
       i += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(i / M);
    const long long r = i - (long long)ch * M;
    const int x = (int)(r % mx), y = (int)((r / mx) % my), z = (int)(r / ((long long)mx * my));
    const float* src = g + (long long)ch * N;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int fx = 2 * x + (k & 1), fy = 2 * y + ((k >> 1) & 1), fz = 2 * z + ((k >> 2) & 1);
      s += src[fx + (long long)nx * (fy + (long long)ny * fz)];
    }
    gin[i] = s;
  }
}

__global__ void __launch_bounds__(kNnBlock) k_to_bf16(const float* __restrict__ x, long long n,
                                                     uint16_t* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = to_bf16(x[i]);
}

// The channel counts the kernels are built for (32: the decoder's input, the
// skip connection and the upsampled coarse level side by side).
#define HFE_NN_CHANNELS(X) X(1) X(2) X(3) X(4) X(6) X(8) X(16) X(32)

template <int CIN>
hipError_t conv_fwd_cin(int cout, const uint16_t* in, const uint16_t* w, const float* bias,
                        const int n[3], int relu, float* out, uint16_t* out16, hipStream_t s) {
  const long long N = (long long)n[0] * n[1] * n[2];
  const dim3 grid((unsigned)((N + kNnBlock - 1) / kNnBlock));
  switch (cout) {
#define HFE_NN_FWD(C)                                                                          \
    case C:                                                                                    \
      hipLaunchKernelGGL((k_conv_fwd<CIN, C>), grid, dim3(kNnBlock), 0, s, in, w, bias, n[0], \
                         n[1], n[2], relu, out, out16);                                        \
      return hipGetLastError();
    HFE_NN_CHANNELS(HFE_NN_FWD)
#undef HFE_NN_FWD
    default: return hipErrorInvalidValue;
  }
}

template <int CIN>
hipError_t conv_bwd_data_cin(int cout, const float* g, const float* act, const uint16_t* w,
                             const int n[3], float* gin, hipStream_t s) {
  const long long N = (long long)n[0] * n[1] * n[2];
  const dim3 grid((unsigned)((N + kNnBlock - 1) / kNnBlock));
  switch (cout) {
#define HFE_NN_BWD(C)                                                                          \
    case C:                                                                                    \
      hipLaunchKernelGGL((k_conv_bwd_data<CIN, C>), grid, dim3(kNnBlock), 0, s, g, act, w,    \
                         n[0], n[1], n[2], gin);                                               \
      return hipGetLastError();
    HFE_NN_CHANNELS(HFE_NN_BWD)
#undef HFE_NN_BWD
    default: return hipErrorInvalidValue;
  }
}

constexpr int kGridMax = 4096;      // blocks of a grid-stride 1D launch

int grid_1d(long long n) {
  long long b = (n + kNnBlock - 1) / kNnBlock;
  return (int)(b < 1 ? 1 : (b > kGridMax ? kGridMax : b));
}

bool dims_ok(const int n[3]) { return n && n[0] >= 1 && n[1] >= 1 && n[2] >= 1; }

}  // namespace
}  // namespace hfe

using namespace hfe;

// Library-owned scratch of hfe_nn_mse_noalloc: one row of partial sums per
// block of the loss kernel, whose grid never exceeds kGridMax blocks, so the
// array fits every n (32 KiB per device, held until the process ends). Host
// code uses the per-device address from hipGetSymbolAddress, never the
// array's name.
static __device__ __align__(256) double scratch[kGridMax];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device, resolved once per device.
hipError_t scratch_rows(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

static bool channels_ok(int c) {
  return c == 1 || c == 2 || c == 3 || c == 4 || c == 6 || c == 8 || c == 16 || c == 32;
}
constexpr int kMaxChannels = 512;
static bool wide_ok(int c) { return c >= 1 && c <= kMaxChannels; }
// the LDS kernels take the listed channel counts; any other pair of counts
// (up to kMaxChannels) runs in the wide kernels
static bool lds_pair(int cin, int cout) { return channels_ok(cin) && channels_ok(cout); }

static dim3 wide_grid(const int n[3], int channels) {
  const long long N = (long long)n[0] * n[1] * n[2];
  return dim3((unsigned)((N + kNnBlock - 1) / kNnBlock),
              (unsigned)((channels + kWideTile - 1) / kWideTile));
}

hfe_status hfe_nn_conv3d(const uint16_t* in, int cin, const uint16_t* w, const float* bias, int cout,
                         const int n[3], int relu, float* out, uint16_t* out_bf16, void* stream) {
  if (!in || !w || !out || !dims_ok(n) || !wide_ok(cin) || !wide_ok(cout)) return HFE_EINVAL;
  if (!lds_pair(cin, cout)) {
    hipLaunchKernelGGL(k_conv_fwd_wide, wide_grid(n, cout), dim3(kNnBlock), 0,
                       (hipStream_t)stream, in, cin, w, bias, cout, n[0], n[1], n[2], relu, out,
                       out_bf16);
    return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
  }
  hipError_t e = hipErrorInvalidValue;
  switch (cin) {
#define HFE_NN_CIN(C)                                                                          \
    case C:                                                                                    \
      e = conv_fwd_cin<C>(cout, in, w, bias, n, relu, out, out_bf16, (hipStream_t)stream);    \
      break;
    HFE_NN_CHANNELS(HFE_NN_CIN)
#undef HFE_NN_CIN
  }
  return e == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

hfe_status hfe_nn_conv3d_backward_data(const float* gout, int cout, const float* act,
                                       const uint16_t* w, int cin, const int n[3], float* gin,
                                       void* stream) {
  if (!gout || !w || !gin || !dims_ok(n) || !wide_ok(cin) || !wide_ok(cout)) return HFE_EINVAL;
  if (!lds_pair(cin, cout)) {
    hipLaunchKernelGGL(k_conv_bwd_data_wide, wide_grid(n, cin), dim3(kNnBlock), 0,
                       (hipStream_t)stream, gout, cout, act, w, cin, n[0], n[1], n[2], gin);
    return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
  }
  hipError_t e = hipErrorInvalidValue;
  switch (cin) {
#define HFE_NN_CIN(C)                                                                          \
    case C:                                                                                    \
      e = conv_bwd_data_cin<C>(cout, gout, act, w, n, gin, (hipStream_t)stream);              \
      break;
    HFE_NN_CHANNELS(HFE_NN_CIN)
#undef HFE_NN_CIN
  }
  return e == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

hfe_status hfe_nn_conv3d_backward_weights(const float* gout, int cout, const float* act,
                                          const uint16_t* in, int cin, const int n[3], float* gw,
                                          float* gb, void* stream) {
  if (!gout || !in || !gw || !dims_ok(n) || !wide_ok(cin) || !wide_ok(cout)) return HFE_EINVAL;
  hipLaunchKernelGGL(k_conv_bwd_w, dim3(cout * cin), dim3(kNnBlock), 0, (hipStream_t)stream, gout,
                     cout, act, in, cin, n[0], n[1], n[2], gw, gb);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

size_t hfe_nn_mse_partials(long long n) { return (size_t)grid_1d(n); }

hfe_status hfe_nn_mse_noalloc(const float* pred, const float* target, long long n, float* grad,
                              double* loss, void* stream) {
  if (!pred || !target || !grad || !loss || n < 1) return HFE_EINVAL;
  const int nb = grid_1d(n);
  static_assert(sizeof(scratch) / sizeof(double) >= (size_t)kGridMax, "scratch holds every row");
  if (nb > kGridMax) return HFE_EINVAL;
  double* rows = nullptr;
  if (scratch_rows(&rows) != hipSuccess) return HFE_EDEVICE;
  // every row the sum reads is written by this call's first kernel: nothing
  // to clear between calls
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kNnBlock), 0, (hipStream_t)stream, pred, target, n, grad,
                     rows);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kNnBlock), 0, (hipStream_t)stream, rows, nb, n, loss);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

hfe_status hfe_nn_mse(const float* pred, const float* target, long long n, float* grad,
                      double* partials, double* loss, void* stream) {
  if (!pred || !target || !grad || !partials || !loss || n < 1) return HFE_EINVAL;
  const int nb = grid_1d(n);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kNnBlock), 0, (hipStream_t)stream, pred, target, n, grad,
                     partials);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kNnBlock), 0, (hipStream_t)stream, partials, nb, n,
                     loss);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

hfe_status hfe_nn_adam(float* w, float* m, float* v, const float* g, long long n, float lr,
                       float beta1, float beta2, float eps, int step, uint16_t* w_bf16,
                       void* stream) {
  if (!w || !m || !v || !g || n < 1 || step < 1) return HFE_EINVAL;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_1d(n)), dim3(kNnBlock), 0, (hipStream_t)stream, w, m, v, g,
                     n, lr, beta1, beta2, eps, c1, c2, w_bf16);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

static bool even_dims(const int n[3]) {
  return dims_ok(n) && n[0] % 2 == 0 && n[1] % 2 == 0 && n[2] % 2 == 0;
}

hfe_status hfe_nn_pool2(const float* in, int c, const int n[3], float* out, uint16_t* out_bf16,
                        void* stream) {
  if (!in || c < 1 || !even_dims(n) || (!out && !out_bf16)) return HFE_EINVAL;
  const long long M = (long long)c * (n[0] / 2) * (n[1] / 2) * (n[2] / 2);
  hipLaunchKernelGGL(k_pool2, dim3(grid_1d(M)), dim3(kNnBlock), 0, (hipStream_t)stream, in, c,
                     n[0], n[1], n[2], out, out_bf16);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

hfe_status hfe_nn_pool2_backward(const float* gout, int c, const int n[3], float* gin,
                                 void* stream) {
  if (!gout || !gin || c < 1 || !even_dims(n)) return HFE_EINVAL;
  const long long N = (long long)c * n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_pool2_bwd, dim3(grid_1d(N)), dim3(kNnBlock), 0, (hipStream_t)stream, gout,
                     c, n[0], n[1], n[2], gin);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

hfe_status hfe_nn_upsample2(const float* in, int c, const int m[3], float* out,
                            uint16_t* out_bf16, void* stream) {
  if (!in || c < 1 || !dims_ok(m) || (!out && !out_bf16)) return HFE_EINVAL;
  const long long N = 8LL * c * m[0] * m[1] * m[2];
  hipLaunchKernelGGL(k_upsample2, dim3(grid_1d(N)), dim3(kNnBlock), 0, (hipStream_t)stream, in, c,
                     m[0], m[1], m[2], out, out_bf16);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

hfe_status hfe_nn_upsample2_backward(const float* gout, int c, const int m[3], float* gin,
                                     void* stream) {
  if (!gout || !gin || c < 1 || !dims_ok(m)) return HFE_EINVAL;
  const long long M = (long long)c * m[0] * m[1] * m[2];
  hipLaunchKernelGGL(k_upsample2_bwd, dim3(grid_1d(M)), dim3(kNnBlock), 0, (hipStream_t)stream,
                     gout, c, m[0], m[1], m[2], gin);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

hfe_status hfe_nn_to_bf16(const float* x, long long n, uint16_t* y, void* stream) {
  if (!x || !y || n < 1) return HFE_EINVAL;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_1d(n)), dim3(kNnBlock), 0, (hipStream_t)stream, x, n, y);
  return hipGetLastError() == hipSuccess ? HFE_OK : HFE_EDEVICE;
}

}  // extern "C"
