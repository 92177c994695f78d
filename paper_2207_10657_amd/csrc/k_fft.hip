// Hand-written FFT and FE Green's operator for gfx950, in FP64 and (for the
// mixed-precision CG) FP32.
//
// The projector of Sec. 2.1 is block diagonal in the wave vector (eq.
// conv_to_fourier). In displacement coordinates its only non-trivial part is
// the inverse of the FE Laplacian L = D^T D, whose Fourier symbol is
// S(k) = sum_{q,j} |Dhat_qj(k)|^2 (the denominator of eq. proj_operator), with
// the k = 0 mode set to zero (ghat(0) = 0). The 3D transform runs in three
// passes over HBM:
//   k_plane<FWD>   per z-plane and component: real-to-complex along x (two
//                  real samples packed per complex value, a half-length
//                  complex FFT and a split step), then a complex FFT along y,
//                  all in LDS;
//   k_pencil       per chunk of consecutive (ky, kx) columns and component:
//                  FFT along z, multiply by 1/(S(k) N), inverse FFT along z,
//                  all in LDS;
//   k_plane<INV>   the inverse of the first pass.
// In 2D a single k_plane<GREEN2D> does forward, multiply and inverse.
//
// The 1D transforms are Stockham autosort passes (radix 8, 4, 3, then 2)
// on lines held in LDS, with every thread staging its butterflies in
// registers between two barriers so that one LDS buffer suffices.
#include "hfe_internal.h"
#include "hfe_reduce.h"

#include <mutex>

namespace hfe {
namespace {

// Complex values of either precision: V is double2 or float2, ScalarOf<V> its
// component type.
template <typename V> struct ScalarOf;
template <> struct ScalarOf<double2> { using T = double; };
template <> struct ScalarOf<float2> { using T = float; };

template <typename V>
__device__ __forceinline__ V mk(typename ScalarOf<V>::T a, typename ScalarOf<V>::T b) {
  V v;
  v.x = a;
  v.y = b;
  return v;
}
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cconj(V a) { return mk<V>(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V>
__device__ __forceinline__ V mul_mi(V a) {
  return INV ? mk<V>(-a.y, a.x) : mk<V>(a.y, -a.x);
}

// Copy `total` elements with up to kStage independent loads in flight per
// thread (all loads of a round are issued before any store).
constexpr int kStage = 8;
template <typename V, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int total, Load load, Store store) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int base = 0; base < total; base += kStage * nt) {
    V r[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int i = base + u * nt + tid;
      if (i < total) r[u] = load(i);
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int i = base + u * nt + tid;
      if (i < total) store(i, r[u]);
    }
  }
}

constexpr int radix_of(int rem) {
  return rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : (rem % 3 == 0 ? 3 : 2));
}

template <int R, bool INV> struct Bfly;
template <bool INV> struct Bfly<2, INV> {
  template <typename V> __device__ static void run(V (&v)[2]) {
    const V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <bool INV> struct Bfly<3, INV> {
  template <typename V> __device__ static void run(V (&v)[3]) {
    using S = typename ScalarOf<V>::T;
    const S kS = S(0.86602540378443864676);  // sin(2 pi / 3)
    const V a = v[0], b = v[1], c = v[2];
    const V t1 = cadd(b, c);
    const V t2 = mk<V>(a.x - S(0.5) * t1.x, a.y - S(0.5) * t1.y);
    const V d = csub(b, c);
    const V t3 = mk<V>(kS * d.x, kS * d.y);
    v[0] = cadd(a, t1);
    v[1] = cadd(t2, mul_mi<INV>(t3));
    v[2] = csub(t2, mul_mi<INV>(t3));
  }
};
template <bool INV> struct Bfly<4, INV> {
  template <typename V> __device__ static void run(V (&v)[4]) {
    const V t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const V t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, mul_mi<INV>(t3));
    v[3] = csub(t1, mul_mi<INV>(t3));
  }
};

template <bool INV> struct Bfly<8, INV> {
  // 8-point DFT = two 4-point DFTs (even, odd samples) and one radix-2 stage
  // with the twiddles e^{-+ 2 pi i k / 8}
  template <typename V> __device__ static void run(V (&v)[8]) {
    using S = typename ScalarOf<V>::T;
    const S kR = S(0.70710678118654752440);   // 1/sqrt(2)
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<4, INV>::run(e);
    Bfly<4, INV>::run(o);
    // w^1 o[1], w^2 o[2], w^3 o[3] with w = e^{-2 pi i/8} (conjugate for INV)
    const V o1 = INV ? mk<V>(kR * (o[1].x - o[1].y), kR * (o[1].x + o[1].y))
                     : mk<V>(kR * (o[1].x + o[1].y), kR * (o[1].y - o[1].x));
    const V o2 = mul_mi<INV>(o[2]);
    const V o3 = INV ? mk<V>(-kR * (o[3].x + o[3].y), kR * (o[3].x - o[3].y))
                     : mk<V>(kR * (o[3].y - o[3].x), -kR * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// One Stockham pass of radix R on `nlines` lines of length L; element k of
// line l is buf[l*ls + k*es]. `tw` holds e^{-2 pi i k / L}, k < L.
template <int L, int R, int NS, bool INV, typename V>
__device__ __forceinline__ void fft_pass(V* buf, int nlines, int ls, int es,
                                         const V* __restrict__ tw) {
  constexpr int NB = L / R;       // butterflies per line
  constexpr int MAXB = 16 / R;    // butterflies staged per thread (caller guarantees enough threads)
  V v[MAXB][R];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int total = nlines * NB;
#pragma unroll
  for (int it = 0; it < MAXB; ++it) {
    const int b = tid + it * nt;
    if (b < total) {
      const int line = b / NB, j = b - line * NB;
      const int k = j % NS;
      const V* base = buf + line * ls;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        V x = base[(j + r * NB) * es];
        if (NS > 1 && r > 0) {
          V w = tw[k * r * (L / (NS * R))];
          if (INV) w.y = -w.y;
          x = cmul(x, w);
        }
        v[it][r] = x;
      }
      Bfly<R, INV>::run(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXB; ++it) {
    const int b = tid + it * nt;
    if (b < total) {
      const int line = b / NB, j = b - line * NB;
      const int k = j % NS;
      const int idx = (j / NS) * NS * R + k;
      V* base = buf + line * ls;
#pragma unroll
      for (int r = 0; r < R; ++r) base[(idx + r * NS) * es] = v[it][r];
    }
  }
  __syncthreads();
}

template <int L, int REM, int NS, bool INV>
struct Passes {
  template <typename V>
  __device__ static void run(V* buf, int nl, int ls, int es, const V* tw) {
    constexpr int R = radix_of(REM);
    fft_pass<L, R, NS, INV>(buf, nl, ls, es, tw);
    Passes<L, REM / R, NS * R, INV>::run(buf, nl, ls, es, tw);
  }
};
template <int L, int NS, bool INV>
struct Passes<L, 1, NS, INV> {
  template <typename V>
  __device__ static void run(V*, int, int, int, const V*) {}
};

// In-place transform of nl lines of runtime length L (uniform over the block).
template <bool INV, typename V>
__device__ __forceinline__ void lds_fft(int L, V* buf, int nl, int ls, int es, const V* tw) {
  switch (L) {
    case 2: Passes<2, 2, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 3: Passes<3, 3, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 4: Passes<4, 4, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 6: Passes<6, 6, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 8: Passes<8, 8, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 12: Passes<12, 12, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 16: Passes<16, 16, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 24: Passes<24, 24, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 32: Passes<32, 32, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 48: Passes<48, 48, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 64: Passes<64, 64, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 96: Passes<96, 96, 1, INV>::run(buf, nl, ls, es, tw); break;
    case 128: Passes<128, 128, 1, INV>::run(buf, nl, ls, es, tw); break;
    default: break;  // L = 1: identity
  }
}

// Split step of the packed real transform along x: row y holds
// Z[m] = FFT_M(x[2m] + i x[2m+1]) in columns 0..M-1; afterwards columns
// 0..M hold X[k] = sum_n x[n] e^{-2 pi i k n / nx}. W[k] = e^{-2 pi i k / nx}.
template <typename V>
__device__ void split_r2c(V* buf, int M, int ny, int P, const V* __restrict__ W) {
  using S = typename ScalarOf<V>::T;
  const int npair = M / 2 + 1;
  for (int i = threadIdx.x; i < ny * npair; i += blockDim.x) {
    const int y = i / npair, k = i - y * npair;
    V* row = buf + y * P;
    if (k == 0) {
      const V z0 = row[0];
      row[0] = mk<V>(z0.x + z0.y, S(0));
      row[M] = mk<V>(z0.x - z0.y, S(0));
    } else {
      const int k2 = M - k;
      const V A = row[k], B = row[k2];
      // X[k] = (A + B*)/2 - i W^k (A - B*)/2
      {
        const V Bc = cconj(B);
        const V s = cadd(A, Bc), d = csub(A, Bc);
        const V wd = cmul(W[k], d);
        row[k] = mk<V>(S(0.5) * (s.x + wd.y), S(0.5) * (s.y - wd.x));
      }
      if (k2 != k) {
        const V Ac = cconj(A);
        const V s = cadd(B, Ac), d = csub(B, Ac);
        const V wd = cmul(W[k2], d);
        row[k2] = mk<V>(S(0.5) * (s.x + wd.y), S(0.5) * (s.y - wd.x));
      }
    }
  }
  __syncthreads();
}

// Inverse of split_r2c, scaled so that the unscaled inverse FFT of length M
// that follows returns nx times the real samples (packed in pairs).
template <typename V>
__device__ void merge_c2r(V* buf, int M, int ny, int P, const V* __restrict__ W) {
  const int npair = M / 2 + 1;
  for (int i = threadIdx.x; i < ny * npair; i += blockDim.x) {
    const int y = i / npair, k = i - y * npair;
    V* row = buf + y * P;
    if (k == 0) {
      const V X0 = row[0], XM = cconj(row[M]);
      const V s = cadd(X0, XM), d = csub(X0, XM);
      row[0] = mk<V>(s.x - d.y, s.y + d.x);
    } else {
      const int k2 = M - k;
      const V A = row[k], B = row[k2];
      // Z[k] = (A + B*) + i W^{-k} (A - B*)
      {
        const V Bc = cconj(B);
        const V s = cadd(A, Bc), d = csub(A, Bc);
        const V wd = cmul(cconj(W[k]), d);
        row[k] = mk<V>(s.x - wd.y, s.y + wd.x);
      }
      if (k2 != k) {
        const V Ac = cconj(A);
        const V s = cadd(B, Ac), d = csub(B, Ac);
        const V wd = cmul(cconj(W[k2]), d);
        row[k2] = mk<V>(s.x - wd.y, s.y + wd.x);
      }
    }
  }
  __syncthreads();
}

// S(k) from the per-axis 1D symbols s_m = 2 - 2 cos(theta_m).
template <typename R>
__device__ __forceinline__ R green_q1(R sx, R sy, R sz) {
  const R px = R(3) - R(0.5) * sx, py = R(3) - R(0.5) * sy, pz = R(3) - R(0.5) * sz;
  return R(8.0 / 9.0) * (sx * py * pz + sy * px * pz + sz * px * py);
}
template <typename R>
__device__ __forceinline__ R green_p1(R sx, R sy) { return R(2) * (sx + sy); }

enum { PLANE_FWD = 0, PLANE_INV = 1, PLANE_GREEN2D = 2, PLANE_FWD_CG = 3, PLANE_INV_CG = 4 };

template <int MODE, typename R>
__global__ void __launch_bounds__(1024) k_plane(Grid g, FftTablesT<R> t, const R* __restrict__ in,
                                                R* __restrict__ out, C2<R>* __restrict__ spec,
                                                R scale, const CgState* skip, CgFuse<R> cf) {
  using V = C2<R>;
  const int nx = g.nx, ny = g.ny, M = nx / 2, P = M + 1;
  const int z = blockIdx.x, c = blockIdx.y;
  const long long plane = (long long)c * g.N + (long long)z * nx * ny;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int npairs = M * ny;   // the plane's reals in pairs (x even, x odd)
  // The fused CG passes read vectors of the plane that do not depend on the
  // decisions or on the transform: their first kPre pairs per thread are
  // loaded before the decisions (forward) or the spectrum (inverse), so that
  // these memory latencies overlap.
  constexpr int kPre = 4;
  constexpr bool kFused = MODE == PLANE_FWD_CG || MODE == PLANE_INV_CG;
  V pa[kFused ? kPre : 1], pb[kFused ? kPre : 1], pc[MODE == PLANE_FWD_CG ? kPre : 1],
      pd[MODE == PLANE_FWD_CG ? kPre : 1];
  // forward: pa = Kd, pb = z, pc = d, pd = g; inverse: pa = y, pb = g
  auto load_round = [&](int base) {
    if constexpr (MODE == PLANE_FWD_CG) {
      const V* kd2 = reinterpret_cast<const V*>(in + plane);
      const V* z2 = reinterpret_cast<const V*>(cf.z + plane);
      const V* d2 = reinterpret_cast<const V*>(cf.d + plane);
      const V* g2 = reinterpret_cast<const V*>(cf.g + plane);
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int i = base + u * nt + tid;
        if (i < npairs) {
          pa[u] = kd2[i];
          pb[u] = z2[i];
          pc[u] = d2[i];
          pd[u] = g2[i];
        }
      }
    } else if constexpr (MODE == PLANE_INV_CG) {
      const V* y2 = reinterpret_cast<const V*>(cf.y + plane);
      const V* g2 = reinterpret_cast<const V*>(cf.g + plane);
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int i = base + u * nt + tid;
        if (i < npairs) {
          pa[u] = y2[i];
          pb[u] = g2[i];
        }
      }
    }
  };
  // CG state of this pass: the forward pass takes the direction and
  // curvature decisions itself (every block on its own copy, from the same
  // rows in the same order, so all copies agree); the inverse pass reads it
  __shared__ CgState sst;
  if constexpr (MODE == PLANE_FWD_CG) {
    const bool run = !cf.st_in->done;
    copy_state_block(&sst, cf.st_in);
    if (run) {
      // (the barriers of the row sums complete the copy)
      double td[2], tc[2], tt[6];
      block_sum_rows<2>(cf.rows_dir, cf.nb_dir, td);
      block_sum_rows<2>(cf.rows_hes, cf.nb_hes, tc);
      if (cf.rows_tail) block_sum_rows<6>(cf.rows_tail, cf.nb_hes, tt);
      // the plane's vectors are in flight while one lane takes the decisions
      // (issued after the row sums, whose unrolled loads need the registers)
      load_round(0);
      if (tid == 0) {
        const bool first = blockIdx.x == 0 && blockIdx.y == 0;
        cg_decide_direction(&sst, td[0], td[1]);
        cg_decide_curvature(&sst, first ? cf.trace : nullptr, tc[0], tc[1],
                            cf.rows_tail ? tt : nullptr);
      }
    }
    __syncthreads();
    if (blockIdx.x == 0 && blockIdx.y == 0) copy_state_block(cf.st_out, &sst);
    if (sst.done) {
      // the CG stopped on the trust-region sphere in this iteration: p = z + tau d
      if (sst.apply_tau && !cf.st_in->done) {
        const R tau = (R)sst.tau;
        V* z2 = reinterpret_cast<V*>(cf.z + plane);
        for (int base = 0; base < npairs; base += kPre * nt) {
          if (base > 0) load_round(base);
#pragma unroll
          for (int u = 0; u < kPre; ++u) {
            const int i = base + u * nt + tid;
            if (i < npairs) z2[i] = mk<V>(pb[u].x + tau * pc[u].x, pb[u].y + tau * pc[u].y);
          }
        }
      }
      return;
    }
  }
  if constexpr (MODE == PLANE_INV_CG) {
    if (cf.st_in->done) return;
    load_round(0);
  }
  if (skip && skip->done) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  V* lds = reinterpret_cast<V*>(lds_raw);
  V* sp = spec + ((long long)c * g.nz + z) * (long long)ny * P;
  // twiddles of the x (length M) and y (length ny) transforms and of the
  // split step, staged once into LDS behind the plane
  V* twx = lds + P * ny;
  V* twy = twx + M;
  V* twp = twy + ny;
  for (int i = tid; i < 2 * M + 1 + ny; i += nt) {
    V v;
    if (i < M) v = t.tw[t.off_x + i];
    else if (i < M + ny) v = t.tw[t.off_y + i - M];
    else v = t.tw[t.off_post + i - M - ny];
    twx[i] = v;
  }
  // modes whose input is a real field (forward transform first); the others
  // start from the half spectrum
  constexpr bool kRealInput = MODE == PLANE_FWD || MODE == PLANE_FWD_CG || MODE == PLANE_GREEN2D;
  if (kRealInput) {
    if constexpr (MODE == PLANE_FWD_CG) {
      // z += alpha d, g += alpha Kd on this plane (Kd is the transform input)
      const R alpha = (R)sst.alpha;
      V* z2 = reinterpret_cast<V*>(cf.z + plane);
      V* g2 = reinterpret_cast<V*>(cf.g + plane);
      for (int base = 0; base < npairs; base += kPre * nt) {
        if (base > 0) load_round(base);
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
          const int i = base + u * nt + tid;
          if (i < npairs) {
            z2[i] = mk<V>(pb[u].x + alpha * pc[u].x, pb[u].y + alpha * pc[u].y);
            g2[i] = mk<V>(pd[u].x + alpha * pa[u].x, pd[u].y + alpha * pa[u].y);
            const int y = i / M, m = i - y * M;
            lds[y * P + m] = pa[u];
          }
        }
      }
    } else {
      const V* src = reinterpret_cast<const V*>(in + plane);
      staged_copy<V>(M * ny, [&](int i) { return src[i]; },
                     [&](int i, V v) {
                       const int y = i / M, m = i - y * M;
                       lds[y * P + m] = v;
                     });
    }
    __syncthreads();
    lds_fft<false>(M, lds, ny, P, 1, twx);
    split_r2c(lds, M, ny, P, twp);
    lds_fft<false>(ny, lds, P, 1, P, twy);
    if (MODE == PLANE_FWD || MODE == PLANE_FWD_CG) {
      for (int i = tid; i < P * ny; i += nt) sp[i] = lds[i];
      return;
    }
    // 2D: multiply by the FE Green's function
    for (int i = tid; i < P * ny; i += nt) {
      const int ky = i / P, kx = i - ky * P;
      const R S = green_p1(t.sx[kx], t.sy[ky]);
      const R m = (kx == 0 && ky == 0) ? R(0) : scale / S;
      lds[i] = mk<V>(lds[i].x * m, lds[i].y * m);
    }
    __syncthreads();
  } else {
    staged_copy<V>(P * ny, [&](int i) { return sp[i]; }, [&](int i, V v) { lds[i] = v; });
    __syncthreads();
  }
  lds_fft<true>(ny, lds, P, 1, P, twy);
  merge_c2r(lds, M, ny, P, twp);
  lds_fft<true>(M, lds, ny, P, 1, twx);
  if constexpr (MODE == PLANE_INV_CG) {
    // y += alpha w and the residual inner products (in FP64), w never leaves
    // LDS. The products are added in an order that does not depend on the
    // block size: pair i is lane i % 64 of the wave that handles the run of
    // 64 pairs holding it (block sizes are multiples of 64), each run is
    // summed across its lanes (wave_total63), and the runs in ascending order.
    constexpr int kMaxRuns = 15 * 1024 / 64;   // npairs < 15 * 1024 (fft_plane_fits)
    __shared__ double runs[2][kMaxRuns];
    const R alpha = (R)cf.st_in->alpha;
    V* y2 = reinterpret_cast<V*>(cf.y + plane);
    const int lane = tid & 63;
    for (int base = 0; base < npairs; base += kPre * nt) {
      if (base > 0) load_round(base);
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int i = base + u * nt + tid;
        const int run0 = i - lane;             // the same for the whole wave
        if (run0 < npairs) {
          double p0 = 0.0, p1 = 0.0;
          if (i < npairs) {
            const int yy = i / M, m = i - yy * M;
            const V w = lds[yy * P + m];
            const V yo = pa[u];
            const V gi = pb[u];
            const V yn = mk<V>(yo.x + alpha * w.x, yo.y + alpha * w.y);
            y2[i] = yn;
            p0 = (double)yn.x * (double)gi.x + (double)yn.y * (double)gi.y;
            p1 = (double)yo.x * (double)gi.x + (double)yo.y * (double)gi.y;
          }
          p0 = wave_total63(p0);
          p1 = wave_total63(p1);
          if (lane == 63) {
            runs[0][run0 / 64] = p0;
            runs[1][run0 / 64] = p1;
          }
        }
      }
    }
    __syncthreads();
    if (tid < 64) {
      const int nruns = (npairs + 63) / 64;
      double s0 = 0.0, s1 = 0.0;
      for (int r = tid; r < nruns; r += 64) {
        s0 += runs[0][r];
        s1 += runs[1][r];
      }
      s0 = wave_total63(s0);
      s1 = wave_total63(s1);
      if (tid == 63) {
        const size_t row = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        cf.partials[row * 2] = s0;
        cf.partials[row * 2 + 1] = s1;
      }
    }
    return;
  }
  V* dst = reinterpret_cast<V*>(out + plane);
  for (int i = tid; i < M * ny; i += nt) {
    const int y = i / M, m = i - y * M;
    dst[i] = lds[y * P + m];
  }
}

enum { PENCIL_GREEN = 0, PENCIL_FWD = 1, PENCIL_INV = 2 };

// Launch shape of the pencil pass: C columns per block (t.pencil_cols),
// t.pencil_threads threads; at most 256 threads.

// One block per run of C consecutive columns p = ky (nx/2+1) + kx of one
// component (the last run may be shorter); the column data of a z row are
// contiguous in the half spectrum.
template <int MODE, typename R>
__global__ void __launch_bounds__(256) k_pencil(Grid g, FftTablesT<R> t, C2<R>* __restrict__ spec,
                                               R scale, const CgState* skip) {
  using V = C2<R>;
  const int C = t.pencil_cols;
  if (skip && skip->done) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  V* lds = reinterpret_cast<V*>(lds_raw);
  const int P = g.nx / 2 + 1, ny = g.ny, nz = g.nz;
  const int ncol = P * ny;
  const int p0 = blockIdx.x * C;
  const int cv = min(C, ncol - p0);
  const int c = blockIdx.y;
  V* base = spec + (long long)c * nz * ncol + p0;
  const long long zs = ncol;
  const int tid = threadIdx.x, nt = blockDim.x;
  // LDS row pitch C + 1: consecutive z of one column fall in different banks
  const int CP = C + 1;
  V* twz = lds + CP * nz;    // z twiddles staged behind the pencils
  for (int i = tid; i < nz; i += nt) twz[i] = t.tw[t.off_z + i];
  staged_copy<V>(nz * cv, [&](int i) {
                   const int zz = i / cv, j = i - zz * cv;
                   return base[zz * zs + j];
                 },
                 [&](int i, V v) {
                   const int zz = i / cv, j = i - zz * cv;
                   lds[zz * CP + j] = v;
                 });
  __syncthreads();
  if (MODE != PENCIL_INV) lds_fft<false>(nz, lds, cv, 1, CP, twz);
  if (MODE == PENCIL_GREEN) {
    for (int i = tid; i < nz * cv; i += nt) {
      const int kz = i / cv, j = i - kz * cv;
      const int p = p0 + j;
      const int ky = p / P, kx = p - ky * P;
      const R S = green_q1(t.sx[kx], t.sy[ky], t.sz[kz]);
      const R m = (kx == 0 && ky == 0 && kz == 0) ? R(0) : scale / S;
      const V v = lds[kz * CP + j];
      lds[kz * CP + j] = mk<V>(v.x * m, v.y * m);
    }
    __syncthreads();
  }
  if (MODE != PENCIL_FWD) lds_fft<true>(nz, lds, cv, 1, CP, twz);
  for (int i = tid; i < nz * cv; i += nt) {
    const int zz = i / cv, j = i - zz * cv;
    base[zz * zs + j] = lds[zz * CP + j];
  }
}

}  // namespace

// A thread stages at most 15 complex values per Stockham pass (radix 3: 5
// butterflies), so a plane block of T threads covers 15 T cells and a pencil
// block of T threads 15 T column values.
bool fft_launch_valid(const Grid& g, int plane_threads, int pencil_cols, int pencil_threads,
                      size_t real_bytes) {
  const int cells = (g.nx / 2 + 1) * g.ny;
  if (plane_threads < 64 || plane_threads > 1024 || plane_threads % 64) return false;
  if (pencil_threads < 64 || pencil_threads > 256 || pencil_threads % 64) return false;
  if (pencil_cols < 1 || pencil_cols > 64) return false;
  if (cells > 15 * plane_threads) return false;
  if ((long long)pencil_cols * g.nz > 15LL * pencil_threads) return false;
  return ((size_t)(pencil_cols + 1) * g.nz + g.nz) * 2 * real_bytes <= 65536;
}

void fft_default_launch(const Grid& g, int* plane_threads, int* pencil_cols, int* pencil_threads) {
  // more threads than the minimum hide latency on the small planes, and short
  // runs of columns give the pencil pass enough blocks (measured on 64^3 and
  // 128^3 cells)
  const int cells = (g.nx / 2 + 1) * g.ny;
  *plane_threads = cells <= 15 * 128 ? 256 : (cells <= 15 * 512 ? 512 : 1024);
  *pencil_cols = 8;
  *pencil_threads = 128;
  while ((long long)*pencil_cols * g.nz > 15LL * *pencil_threads && *pencil_cols > 1) *pencil_cols /= 2;
}

namespace {

constexpr int kLdsPerCu = 160 * 1024;   // gfx950: LDS of one workgroup at most
constexpr int kMaxDevices = 64;

// Raise the dynamic-LDS limit of a plane kernel to what the 160 KiB of a
// workgroup leave beside its static LDS, once per device (the attribute is
// per function and device), not on every launch: launches happen from
// several host threads at once (batches of contexts) and inside graph
// captures.
template <int MODE, typename R>
hipError_t plane_lds_limit() {
  static std::mutex mu;
  static bool set[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (set[dev]) return hipSuccess;
  hipFuncAttributes fa;
  e = hipFuncGetAttributes(&fa, (const void*)k_plane<MODE, R>);
  if (e == hipSuccess && fa.sharedSizeBytes >= (size_t)kLdsPerCu) e = hipErrorInvalidValue;
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_plane<MODE, R>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            kLdsPerCu - (int)fa.sharedSizeBytes);
  if (e == hipSuccess) set[dev] = true;
  else (void)hipGetLastError();   // the failure is returned, not left for later calls
  return e;
}

template <int MODE, typename R>
hipError_t launch_plane(const Grid& g, const FftTablesT<R>& t, const R* in, R* out, C2<R>* spec,
                        R scale, hipStream_t s, const CgState* skip = nullptr,
                        CgFuse<R> cf = CgFuse<R>{}) {
  // every pointer the mode dereferences must be present (a missing one is an
  // error here, not a fault on the device)
  constexpr bool real_in = MODE == PLANE_FWD || MODE == PLANE_FWD_CG || MODE == PLANE_GREEN2D;
  constexpr bool real_out = MODE == PLANE_INV || MODE == PLANE_GREEN2D;
  constexpr bool cg = MODE == PLANE_FWD_CG || MODE == PLANE_INV_CG;
  if ((real_in && !in) || (real_out && !out) || !spec || !t.tw) return hipErrorInvalidValue;
  if (cg && (!cf.st_in || !cf.d || !cf.z || !cf.g || !cf.y || !cf.partials)) return hipErrorInvalidValue;
  if (MODE == PLANE_FWD_CG && (!cf.st_out || !cf.rows_dir || !cf.rows_hes || cf.nb_dir < 1 ||
                               cf.nb_hes < 1 || t.plane_threads < 256))
    return hipErrorInvalidValue;
  if (!fft_plane_fits<R>(g)) return hipErrorInvalidValue;
  if (!fft_launch_valid(g, t.plane_threads, t.pencil_cols, t.pencil_threads, sizeof(R)))
    return hipErrorInvalidValue;
  const size_t lds = fft_plane_lds_bytes<R>(g);
  if (lds > 65536) {
    const hipError_t e = plane_lds_limit<MODE, R>();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_plane<MODE, R>), dim3(g.nz, g.dim), dim3(t.plane_threads), lds, s, g, t,
                     in, out, spec, scale, skip, cf);
  return hipGetLastError();
}

template <int MODE, typename R>
hipError_t launch_pencil(const Grid& g, const FftTablesT<R>& t, C2<R>* spec, R scale,
                         hipStream_t s, const CgState* skip = nullptr) {
  if (!spec || !t.tw) return hipErrorInvalidValue;
  if (!fft_launch_valid(g, t.plane_threads, t.pencil_cols, t.pencil_threads, sizeof(R)))
    return hipErrorInvalidValue;
  const int C = t.pencil_cols;
  const int ncol = (g.nx / 2 + 1) * g.ny;
  const int nchunk = (ncol + C - 1) / C;
  const size_t lds = ((size_t)(C + 1) * g.nz + g.nz) * sizeof(C2<R>);
  hipLaunchKernelGGL((k_pencil<MODE, R>), dim3(nchunk, g.dim), dim3(t.pencil_threads), lds, s, g,
                     t, spec, scale, skip);
  return hipGetLastError();
}

}  // namespace

bool fft_length_supported(int L) {
  switch (L) {
    case 1: case 2: case 3: case 4: case 6: case 8: case 12: case 16: case 24: case 32:
    case 48: case 64: case 96: case 128:
      return true;
    default:
      return false;
  }
}

template <typename R>
size_t fft_plane_lds_bytes(const Grid& g) {
  const int M = g.nx / 2;
  return ((size_t)(M + 1) * g.ny + 2 * M + 1 + g.ny) * sizeof(C2<R>);
}

template <typename R>
bool fft_plane_fits(const Grid& g) {
  // LDS of one CU less 4 KiB for the passes' static LDS (the run sums of the
  // fused inverse pass), and at most 15 staged values per thread of a
  // 1024-thread block
  return fft_plane_lds_bytes<R>(g) <= 156 * 1024 && (long long)(g.nx / 2 + 1) * g.ny <= 15 * 1024;
}

namespace {
template <typename R>
hipError_t plane_limits_all(const Grid& g) {
  if (fft_plane_lds_bytes<R>(g) <= 65536) return hipSuccess;
  hipError_t e = plane_lds_limit<PLANE_FWD, R>();
  if (e == hipSuccess) e = plane_lds_limit<PLANE_INV, R>();
  if (e == hipSuccess) e = plane_lds_limit<PLANE_GREEN2D, R>();
  if (e == hipSuccess) e = plane_lds_limit<PLANE_FWD_CG, R>();
  if (e == hipSuccess) e = plane_lds_limit<PLANE_INV_CG, R>();
  return e;
}
}  // namespace

hipError_t fft_prepare(const Grid& g) {
  hipError_t e = plane_limits_all<double>(g);
  if (e == hipSuccess) e = plane_limits_all<float>(g);
  return e;
}

template <typename R>
hipError_t fft_plane_forward(const Grid& g, const FftTablesT<R>& t, const R* in, C2<R>* spec,
                             hipStream_t s, const CgState* skip) {
  return launch_plane<PLANE_FWD, R>(g, t, in, nullptr, spec, R(1), s, skip);
}

template <typename R>
hipError_t fft_plane_inverse(const Grid& g, const FftTablesT<R>& t, C2<R>* spec, R* out,
                             hipStream_t s, const CgState* skip) {
  return launch_plane<PLANE_INV, R>(g, t, nullptr, out, spec, R(1), s, skip);
}

template <typename R>
hipError_t fft_pencil_green(const Grid& g, const FftTablesT<R>& t, C2<R>* spec, hipStream_t s,
                            const CgState* skip) {
  return launch_pencil<PENCIL_GREEN, R>(g, t, spec, R(1.0 / (double)g.N), s, skip);
}

template <typename R>
hipError_t fft_plane_green2d(const Grid& g, const FftTablesT<R>& t, const R* in, R* out,
                             C2<R>* spec, hipStream_t s, const CgState* skip) {
  return launch_plane<PLANE_GREEN2D, R>(g, t, in, out, spec, R(1.0 / (double)g.N), s, skip);
}

template <typename R>
hipError_t fft_plane_forward_cg(const Grid& g, const FftTablesT<R>& t, const R* Kd, C2<R>* spec,
                                const CgFuse<R>& f, hipStream_t s) {
  return launch_plane<PLANE_FWD_CG, R>(g, t, Kd, nullptr, spec, R(1), s, nullptr, f);
}

template <typename R>
hipError_t fft_plane_inverse_cg(const Grid& g, const FftTablesT<R>& t, C2<R>* spec,
                                const CgFuse<R>& f, hipStream_t s, int* nblocks) {
  *nblocks = g.nz * g.dim;
  return launch_plane<PLANE_INV_CG, R>(g, t, nullptr, nullptr, spec, R(1), s, nullptr, f);
}

template <typename R>
hipError_t green_apply(const Grid& g, const FftTablesT<R>& t, const R* in, R* out, C2<R>* spec,
                       hipStream_t s, const CgState* skip) {
  if (g.dim == 2) return fft_plane_green2d(g, t, in, out, spec, s, skip);
  hipError_t e = fft_plane_forward(g, t, in, spec, s, skip);
  if (e != hipSuccess) return e;
  e = fft_pencil_green(g, t, spec, s, skip);
  if (e != hipSuccess) return e;
  return fft_plane_inverse(g, t, spec, out, s, skip);
}

hipError_t fft_forward(const Grid& g, const FftTables& t, const double* in, double2* spec,
                       hipStream_t s) {
  hipError_t e = launch_plane<PLANE_FWD, double>(g, t, in, nullptr, spec, 1.0, s);
  if (e != hipSuccess || g.nz == 1) return e;
  return launch_pencil<PENCIL_FWD, double>(g, t, spec, 1.0, s);
}

hipError_t fft_inverse(const Grid& g, const FftTables& t, double2* spec, double* out,
                       hipStream_t s) {
  if (g.nz > 1) {
    hipError_t e = launch_pencil<PENCIL_INV, double>(g, t, spec, 1.0, s);
    if (e != hipSuccess) return e;
  }
  return launch_plane<PLANE_INV, double>(g, t, nullptr, out, spec, 1.0, s);
}

#define HFE_FFT_INSTANTIATE(R)                                                                  \
  template size_t fft_plane_lds_bytes<R>(const Grid&);                                          \
  template bool fft_plane_fits<R>(const Grid&);                                                 \
  template hipError_t fft_plane_forward<R>(const Grid&, const FftTablesT<R>&, const R*, C2<R>*, \
                                           hipStream_t, const CgState*);                        \
  template hipError_t fft_plane_inverse<R>(const Grid&, const FftTablesT<R>&, C2<R>*, R*,       \
                                           hipStream_t, const CgState*);                        \
  template hipError_t fft_pencil_green<R>(const Grid&, const FftTablesT<R>&, C2<R>*,            \
                                          hipStream_t, const CgState*);                         \
  template hipError_t fft_plane_green2d<R>(const Grid&, const FftTablesT<R>&, const R*, R*,     \
                                           C2<R>*, hipStream_t, const CgState*);                \
  template hipError_t fft_plane_forward_cg<R>(const Grid&, const FftTablesT<R>&, const R*,      \
                                              C2<R>*, const CgFuse<R>&, hipStream_t);           \
  template hipError_t fft_plane_inverse_cg<R>(const Grid&, const FftTablesT<R>&, C2<R>*,        \
                                              const CgFuse<R>&, hipStream_t, int*);             \
  template hipError_t green_apply<R>(const Grid&, const FftTablesT<R>&, const R*, R*, C2<R>*,   \
                                     hipStream_t, const CgState*);

HFE_FFT_INSTANTIATE(double)
HFE_FFT_INSTANTIATE(float)
#undef HFE_FFT_INSTANTIATE

}  // namespace hfe
