// Element-level kernels of the FE-projection scheme: discrete gradient at
// the quadrature points (Sec. 2.1, the FE derivative operator evaluated at
// quadrature points), the damage law and its consistent tangent at every
// point (the Hessian of eq. graient_and_hessian used in eq.
// project_stress_linear), and the FE divergence D^T that brings point
// stresses back to the nodes.
//
// One thread per node gathers the contributions of the elements around it;
// the element whose lowest corner is the node also writes the per-point
// state and adds the per-point terms of the reductions, so every point is
// counted once.
#include "hfe_internal.h"
#include "hfe_reduce.h"

#include <hip/hip_ext.h>
#include <type_traits>

namespace hfe {
namespace {

// Gauss abscissae of the 2-point rule on [0,1]: 1/2 -+ 1/(2 sqrt 3).
constexpr double kG0 = 0.21132486540518711775;
constexpr double kG1 = 0.78867513459481288225;

template <int EL> struct ET;
template <> struct ET<HFE_Q1> { static constexpr int D = 3, NQ = 8, NA = 8; };
template <> struct ET<HFE_P1_PAIR> { static constexpr int D = 2, NQ = 2, NA = 4; };

// dN_a/dx_j at the Gauss points of the Q1 element, as a table in constant
// memory for loops over points that are not unrolled (the index is uniform
// over the wavefront, so the values come through scalar loads).
template <typename R>
struct Q1Table {
  R v[8][8][3];
  constexpr Q1Table() : v{} {
    for (int q = 0; q < 8; ++q)
      for (int a = 0; a < 8; ++a) {
        const int o0 = a & 1, o1 = (a >> 1) & 1, o2 = (a >> 2) & 1;
        const double x0 = (q & 1) ? kG1 : kG0, x1 = (q & 2) ? kG1 : kG0, x2 = (q & 4) ? kG1 : kG0;
        const double l0 = o0 ? x0 : 1.0 - x0, l1 = o1 ? x1 : 1.0 - x1, l2 = o2 ? x2 : 1.0 - x2;
        v[q][a][0] = R((o0 ? 1.0 : -1.0) * l1 * l2);
        v[q][a][1] = R((o1 ? 1.0 : -1.0) * l0 * l2);
        v[q][a][2] = R((o2 ? 1.0 : -1.0) * l0 * l1);
      }
  }
};
__constant__ Q1Table<double> kQ1B = Q1Table<double>();
__constant__ Q1Table<float> kQ1Bf = Q1Table<float>();

template <typename R> __device__ __forceinline__ const Q1Table<R>& q1b();
template <> __device__ __forceinline__ const Q1Table<double>& q1b<double>() { return kQ1B; }
template <> __device__ __forceinline__ const Q1Table<float>& q1b<float>() { return kQ1Bf; }

// dN_a/dx_j at point q of a unit element. Local node a = ax + 2 ay (+ 4 az).
template <int EL>
__device__ __forceinline__ double shape_grad(int q, int a, int j);

template <>
__device__ __forceinline__ double shape_grad<HFE_Q1>(int q, int a, int j) {
  const int o0 = a & 1, o1 = (a >> 1) & 1, o2 = (a >> 2) & 1;
  const double x0 = (q & 1) ? kG1 : kG0, x1 = (q & 2) ? kG1 : kG0, x2 = (q & 4) ? kG1 : kG0;
  const double l0 = o0 ? x0 : 1.0 - x0, l1 = o1 ? x1 : 1.0 - x1, l2 = o2 ? x2 : 1.0 - x2;
  if (j == 0) return (o0 ? 1.0 : -1.0) * l1 * l2;
  if (j == 1) return (o1 ? 1.0 : -1.0) * l0 * l2;
  return (o2 ? 1.0 : -1.0) * l0 * l1;
}

// Two linear triangles per pixel: T1 = (0,0),(1,0),(0,1); T2 = (1,1),(0,1),(1,0).
template <>
__device__ __forceinline__ double shape_grad<HFE_P1_PAIR>(int q, int a, int j) {
  if (q == 0) {
    if (a == 0) return -1.0;
    if (a == 1) return j == 0 ? 1.0 : 0.0;
    if (a == 2) return j == 1 ? 1.0 : 0.0;
    return 0.0;
  }
  if (a == 3) return 1.0;
  if (a == 2) return j == 0 ? -1.0 : 0.0;
  if (a == 1) return j == 1 ? -1.0 : 0.0;
  return 0.0;
}

// Symmetric tensors are held as (xx, yy, zz, xy, xz, yz); in 2D zz, xz, yz of
// a strain are zero (plane strain). R = double, or float in the FP32 Hessian.
template <typename R> struct SymT { R v[6]; };
using Sym = SymT<double>;

template <typename R>
__device__ __forceinline__ R sym_dot(const SymT<R>& a, const SymT<R>& b) {
  return a.v[0] * b.v[0] + a.v[1] * b.v[1] + a.v[2] * b.v[2] +
         R(2) * (a.v[3] * b.v[3] + a.v[4] * b.v[4] + a.v[5] * b.v[5]);
}

// sym part of a full gradient H[i][j] (d x d, row i = displacement component)
template <int D, typename R>
__device__ __forceinline__ SymT<R> sym_of(const R (&H)[3][3]) {
  SymT<R> e;
  e.v[0] = H[0][0];
  e.v[1] = H[1][1];
  e.v[2] = D == 3 ? H[2][2] : R(0);
  e.v[3] = R(0.5) * (H[0][1] + H[1][0]);
  e.v[4] = D == 3 ? R(0.5) * (H[0][2] + H[2][0]) : R(0);
  e.v[5] = D == 3 ? R(0.5) * (H[1][2] + H[2][1]) : R(0);
  return e;
}

template <typename R>
__device__ __forceinline__ SymT<R> c_contract(const SymT<R>& e, R lam, R mu) {
  const R tr = e.v[0] + e.v[1] + e.v[2];
  SymT<R> s;
  s.v[0] = lam * tr + R(2) * mu * e.v[0];
  s.v[1] = lam * tr + R(2) * mu * e.v[1];
  s.v[2] = lam * tr + R(2) * mu * e.v[2];
  s.v[3] = R(2) * mu * e.v[3];
  s.v[4] = R(2) * mu * e.v[4];
  s.v[5] = R(2) * mu * e.v[5];
  return s;
}

// One Jacobi rotation in the (p, q) plane that zeroes A[p][q] of the symmetric
// 3x3 A, accumulated into the eigenvector columns of V (Rutishauser's form:
// t = tan of the angle, the smaller root, tau = s / (1 + c)).
template <int P, int Q>
__host__ __device__ __forceinline__ void jacobi_rotate(double (&A)[3][3], double (&V)[3][3]) {
  constexpr int Rr = 3 - P - Q;
  const double apq = A[P][Q];
  if (apq == 0.0) return;
  const double theta = (A[Q][Q] - A[P][P]) / (2.0 * apq);
  const double at = fabs(theta);
  double t = at > 1e150 ? 0.5 / at : 1.0 / (at + sqrt(at * at + 1.0));
  if (theta < 0.0) t = -t;
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c, tau = s / (1.0 + c);
  A[P][P] -= t * apq;
  A[Q][Q] += t * apq;
  A[P][Q] = A[Q][P] = 0.0;
  const double g = A[Rr][P], h = A[Rr][Q];
  A[Rr][P] = A[P][Rr] = g - s * (h + g * tau);
  A[Rr][Q] = A[Q][Rr] = h + s * (g - h * tau);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double vg = V[r][P], vh = V[r][Q];
    V[r][P] = vg - s * (vh + vg * tau);
    V[r][Q] = vh + s * (vg - vh * tau);
  }
}

// Tensile part eps_t = sum_i max(e_i, 0) q_i (x) q_i of a symmetric strain
// over its eigenpairs (e_i, q_i): the masked strain M eps M of Appendix A.
// Cyclic Jacobi sweeps until the off-diagonal part is below 1e-17 of the
// diagonal (quadratic convergence: a few sweeps); no division by an
// eigenvalue gap, so equal principal strains need no special case. In 2D
// the zz, xz and yz entries are zero and one rotation is exact.
__host__ __device__ inline Sym tensile_part(const Sym& e) {
  double A[3][3] = {{e.v[0], e.v[3], e.v[4]}, {e.v[3], e.v[1], e.v[5]}, {e.v[4], e.v[5], e.v[2]}};
  double V[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (!(off > 1e-34 * dia)) break;
    jacobi_rotate<0, 1>(A, V);
    jacobi_rotate<0, 2>(A, V);
    jacobi_rotate<1, 2>(A, V);
  }
  const double l0 = fmax(A[0][0], 0.0), l1 = fmax(A[1][1], 0.0), l2 = fmax(A[2][2], 0.0);
  auto ent = [&](int a, int b) {
    return l0 * V[a][0] * V[b][0] + l1 * V[a][1] * V[b][1] + l2 * V[a][2] * V[b][2];
  };
  Sym t;
  t.v[0] = ent(0, 0);
  t.v[1] = ent(1, 1);
  t.v[2] = ent(2, 2);
  t.v[3] = ent(0, 1);
  t.v[4] = ent(0, 2);
  t.v[5] = ent(1, 2);
  return t;
}

// The strain the law sees: sym(H) plus the phase's eigenstrain (Algorithm 2
// adds it before every evaluation; in 2D only its in-plane part is set).
template <int D, typename R>
__device__ __forceinline__ SymT<R> eval_strain(const R (&H)[3][3], const MatTable& m, int ph) {
  SymT<R> e = sym_of<D>(H);
#pragma unroll
  for (int k = 0; k < 6; ++k) e.v[k] += (R)m.eig[ph][k];
  return e;
}

// Norm^2 of the d x d block of a symmetric tensor (the plane-strain zz
// component is not part of the unknowns' inner product in 2D).
template <int D>
__device__ __forceinline__ double sym_norm2(const Sym& s) {
  if (D == 3) return sym_dot(s, s);
  return s.v[0] * s.v[0] + s.v[1] * s.v[1] + 2.0 * s.v[3] * s.v[3];
}

struct PointLaw {
  Sym s;        // C : eps
  Sym n;        // direction of the equivalent strain's derivative (TENS builds)
  double a;     // 1 - d
  double cp;    // c' of the rank-one softening term
  double kt;    // equivalent strain kappa_t
};

// Damage law at one point with the history kappa_hist frozen. law is the
// phase's kind: HFE_ELASTIC, HFE_DAMAGE_ENERGY_NORM (kappa_t the energy norm
// sqrt(eps:C:eps/E), d kappa_t/d eps = s/(E kappa_t)) or, in TENS builds,
// HFE_DAMAGE_TENSILE (Appendix A: kappa_t = |eps_t| of the tensile part,
// d kappa_t/d eps = eps_t/kappa_t). Both share the bilinear d(kappa); the
// tangent is a C - c' (n : deps) s with n = s or eps_t.
template <bool TENS = false>
__device__ __forceinline__ PointLaw eval_law(const Sym& eps, double lam, double mu, double E,
                                             int law, double k0, double kf, double kh) {
  PointLaw P;
  P.s = c_contract(eps, lam, mu);
  double scale = E;
  if (TENS && law == HFE_DAMAGE_TENSILE) {
    P.n = tensile_part(eps);
    P.kt = sqrt(sym_dot(P.n, P.n));
    scale = 1.0;
  } else {
    const double ecs = sym_dot(eps, P.s);
    P.kt = sqrt(fmax(ecs, 0.0) / E);
    if (TENS) P.n = P.s;
  }
  double d = 0.0, cp = 0.0;
  if (law) {
    const bool loading = P.kt > kh;
    const double ke = loading ? P.kt : kh;
    d = kf / ke * (ke - k0) / (kf - k0);
    d = fmin(fmax(d, 0.0), 1.0);
    if (loading && d > 0.0 && d < 1.0) {
      const double dprime = kf * k0 / ((kf - k0) * (P.kt * P.kt));
      cp = dprime / (scale * P.kt);
    }
  }
  P.a = 1.0 - d;
  P.cp = cp;
  return P;
}

// Equivalent strain kappa_t of either damage law (for the history commit).
__device__ inline double equiv_strain(const Sym& eps, double lam, double mu, double E, int law) {
  if (law == HFE_DAMAGE_TENSILE) {
    const Sym t = tensile_part(eps);
    return sqrt(sym_dot(t, t));
  }
  const Sym s = c_contract(eps, lam, mu);
  return sqrt(fmax(sym_dot(eps, s), 0.0) / E);
}

// Tangent applied to a perturbation: a C:deps - c' (n:deps) s (n = s for
// the energy-norm law).
template <typename R>
__device__ __forceinline__ SymT<R> apply_tangent(const SymT<R>& de, R a, R cp, const SymT<R>& s,
                                                 const SymT<R>& n, R lam, R mu) {
  SymT<R> t = c_contract(de, lam, mu);
#pragma unroll
  for (int k = 0; k < 6; ++k) t.v[k] *= a;
  if (cp != R(0)) {
    const R nde = sym_dot(n, de);
#pragma unroll
    for (int k = 0; k < 6; ++k) t.v[k] -= cp * nde * s.v[k];
  }
  return t;
}

template <typename R>
__device__ __forceinline__ R sym_at(const SymT<R>& s, int i, int j) {
  if (i == j) return s.v[i];
  const int k = (i + j == 1) ? 3 : ((i + j == 2) ? 4 : 5);
  return s.v[k];
}

struct Pos { int x, y, z; };

__device__ __forceinline__ long long lin(const Grid& g, int x, int y, int z) {
  return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

template <int EL>
__device__ __forceinline__ long long elem_node(const Grid& g, const Pos& e, int a) {
  int x = e.x + (a & 1), y = e.y + ((a >> 1) & 1), z = e.z + ((a >> 2) & 1);
  if (x >= g.nx) x -= g.nx;
  if (y >= g.ny) y -= g.ny;
  if (ET<EL>::D == 2) z = 0; else if (z >= g.nz) z -= g.nz;
  return lin(g, x, y, z);
}

template <int EL>
__device__ __forceinline__ void load_nodal(const Grid& g, const double* __restrict__ f,
                                           const Pos& e, double (&v)[3][ET<EL>::NA]) {
  constexpr int D = ET<EL>::D, NA = ET<EL>::NA;
#pragma unroll
  for (int b = 0; b < NA; ++b) {
    const long long n = elem_node<EL>(g, e, b);
#pragma unroll
    for (int i = 0; i < D; ++i) v[i][b] = f[i * g.N + n];
  }
}

// Full gradient at point q of a nodal field (element-local values).
template <int EL>
__device__ __forceinline__ void grad_at(int q, const double (&v)[3][ET<EL>::NA], double (&H)[3][3]) {
  constexpr int D = ET<EL>::D, NA = ET<EL>::NA;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) H[i][j] = 0.0;
#pragma unroll
  for (int b = 0; b < NA; ++b)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double w = shape_grad<EL>(q, b, j);
#pragma unroll
      for (int i = 0; i < D; ++i) H[i][j] += w * v[i][b];
    }
}

template <int EL>
__device__ __forceinline__ Pos elem_of(const Grid& g, int x, int y, int z, int al) {
  Pos e;
  e.x = x - (al & 1);
  e.y = y - ((al >> 1) & 1);
  e.z = (ET<EL>::D == 3) ? z - ((al >> 2) & 1) : 0;
  if (e.x < 0) e.x += g.nx;
  if (e.y < 0) e.y += g.ny;
  if (e.z < 0) e.z += g.nz;
  return e;
}

enum { MODE_RESIDUAL = 0, MODE_TRIAL = 1, MODE_HESSIAN = 2 };

template <int EL, int MODE, int NV>
__global__ void __launch_bounds__(kBlock) k_gather(ElemArgs A) {
  constexpr int D = ET<EL>::D, NQ = ET<EL>::NQ, NA = ET<EL>::NA;
  const Grid& g = A.g;
  if (MODE == MODE_HESSIAN && A.cg && A.cg->done) return;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (n < g.N) {
    const int x = (int)(n % g.nx);
    const int y = (int)((n / g.nx) % g.ny);
    const int z = (int)(n / ((long long)g.nx * g.ny));
    double fo[3] = {0.0, 0.0, 0.0};
    double Em[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Em[i][j] = (i < D && j < D) ? A.E[3 * i + j] : 0.0;
    // the trial pass only sums over points (no divergence): the element
    // this node owns is the only one it needs
    constexpr int kElems = MODE == MODE_TRIAL ? 1 : NA;
#pragma unroll 1
    for (int al = 0; al < kElems; ++al) {
      const Pos e = elem_of<EL>(g, x, y, z, al);
      const long long ei = lin(g, e.x, e.y, e.z);
      const int ph = A.phase[ei];
      const double lam = A.mat.lam[ph], mu = A.mat.mu[ph], Ey = A.mat.E[ph];
      const int dmg = A.mat.damage[ph];
      const double k0 = A.mat.k0[ph], kf = A.mat.kf[ph];
      const bool owner = (al == 0);
      double un[3][NA], vn[3][NA];
      if (MODE == MODE_HESSIAN) {
        bool need_s = false;
#pragma unroll
        for (int q = 0; q < NQ; ++q) need_s |= (A.cp[q * g.N + ei] != 0.0);
        load_nodal<EL>(g, A.v, e, vn);
        if (need_s) load_nodal<EL>(g, A.u, e, un);
        else {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int b = 0; b < NA; ++b) un[i][b] = 0.0;
        }
      } else {
        load_nodal<EL>(g, A.u, e, un);
        if (MODE == MODE_TRIAL) load_nodal<EL>(g, A.v, e, vn);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        Sym tau;
        if constexpr (MODE == MODE_HESSIAN) {
          double dH[3][3];
          grad_at<EL>(q, vn, dH);
          const double aq = A.a[q * g.N + ei], cq = A.cp[q * g.N + ei];
          Sym s, nv;
          if (cq != 0.0) {
            double H[3][3];
            grad_at<EL>(q, un, H);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j) H[i][j] += Em[i][j];
            const Sym eps = eval_strain<D>(H, A.mat, ph);
            s = c_contract(eps, lam, mu);
            nv = dmg == HFE_DAMAGE_TENSILE ? tensile_part(eps) : s;
          } else {
#pragma unroll
            for (int k = 0; k < 6; ++k) s.v[k] = nv.v[k] = 0.0;
          }
          tau = apply_tangent(sym_of<D>(dH), aq, cq, s, nv, lam, mu);
          if (owner) {
            double dd = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
              for (int j = 0; j < D; ++j) dd += dH[i][j] * dH[i][j];
            acc[HES_DD] += dd;
          }
        } else if constexpr (MODE == MODE_RESIDUAL) {
          double H[3][3];
          grad_at<EL>(q, un, H);
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) H[i][j] += Em[i][j];
          const Sym eps = eval_strain<D>(H, A.mat, ph);
          const double kh = A.khist[q * g.N + ei];
          const PointLaw P = eval_law<true>(eps, lam, mu, Ey, dmg, k0, kf, kh);
#pragma unroll
          for (int k = 0; k < 6; ++k) tau.v[k] = P.a * P.s.v[k];
          if (owner) {
            A.a_out[q * g.N + ei] = P.a;
            A.cp_out[q * g.N + ei] = P.cp;
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[RES_S0 + k] += tau.v[k];
            acc[RES_SS] += sym_norm2<D>(tau);
            double hh = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
              for (int j = 0; j < D; ++j) hh += H[i][j] * H[i][j];
            acc[RES_HH] += hh;
          }
        } else {  // MODE_TRIAL
          double H[3][3], p[3][3];
          grad_at<EL>(q, un, H);
          grad_at<EL>(q, vn, p);
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) H[i][j] += Em[i][j];
          double Ht[3][3];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Ht[i][j] = H[i][j] + p[i][j];
          const double kh = A.khist[q * g.N + ei];
          const PointLaw P = eval_law<true>(eval_strain<D>(Ht, A.mat, ph), lam, mu, Ey, dmg, k0, kf,
                                            kh);
#pragma unroll
          for (int k = 0; k < 6; ++k) tau.v[k] = P.a * P.s.v[k];
          if (owner) {
            const double ao = A.a[q * g.N + ei], co = A.cp[q * g.N + ei];
            const Sym eo = eval_strain<D>(H, A.mat, ph);
            const Sym so = c_contract(eo, lam, mu);
            const Sym no = (co != 0.0 && dmg == HFE_DAMAGE_TENSILE) ? tensile_part(eo) : so;
            const Sym ps = sym_of<D>(p);
            double sig_p = 0.0;  // sigma_old : p
            {
              Sym sig;
#pragma unroll
              for (int k = 0; k < 6; ++k) sig.v[k] = ao * so.v[k];
              sig_p = sym_dot(sig, ps);
            }
            const Sym Bp = apply_tangent(ps, ao, co, so, no, lam, mu);
            acc[TRI_SP] += sig_p;
            acc[TRI_PBP] += sym_dot(Bp, ps);
            acc[TRI_STP] += sym_dot(tau, ps);
            double pp = 0.0, hh = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
              for (int j = 0; j < D; ++j) {
                pp += p[i][j] * p[i][j];
                hh += Ht[i][j] * Ht[i][j];
              }
            acc[TRI_PP] += pp;
            acc[TRI_HH] += hh;
          }
        }
        // divergence: contribution of this point to the element's local node al
        if (MODE != MODE_TRIAL) {
#pragma unroll
          for (int j = 0; j < D; ++j) {
            const double w = shape_grad<EL>(q, al, j);
#pragma unroll
            for (int i = 0; i < D; ++i) fo[i] += w * sym_at(tau, i, j);
          }
        }
      }
    }
    if (MODE != MODE_TRIAL) {
#pragma unroll
      for (int i = 0; i < D; ++i) A.f[i * g.N + n] = fo[i];
    }
    if constexpr (MODE == MODE_HESSIAN) {
      double dk = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) dk += A.v[i * g.N + n] * fo[i];
      acc[HES_DKD] += dk;
    }
  }
  block_reduce_store<NV>(acc, A.red.partials);
}

template <int EL>
__global__ void __launch_bounds__(kBlock) k_commit(ElemArgs A) {
  constexpr int D = ET<EL>::D, NQ = ET<EL>::NQ, NA = ET<EL>::NA;
  const Grid& g = A.g;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int ph = A.phase[n];
  if (!A.mat.damage[ph]) return;
  Pos e;
  e.x = (int)(n % g.nx);
  e.y = (int)((n / g.nx) % g.ny);
  e.z = (int)(n / ((long long)g.nx * g.ny));
  double un[3][NA];
  load_nodal<EL>(g, A.u, e, un);
  double* kh = A.a_out;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double H[3][3];
    grad_at<EL>(q, un, H);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) H[i][j] += A.E[3 * i + j];
    const double kt = equiv_strain(eval_strain<D>(H, A.mat, ph), A.mat.lam[ph], A.mat.mu[ph],
                                   A.mat.E[ph], A.mat.damage[ph]);
    const long long idx = q * g.N + n;
    kh[idx] = fmax(kh[idx], kt);
  }
}

__global__ void __launch_bounds__(kBlock) k_init_history(ElemArgs A) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= A.g.N) return;
  const int ph = A.phase[n];
  const double v = A.mat.damage[ph] ? A.mat.k0[ph] : 0.0;
  for (int q = 0; q < A.g.nq; ++q) A.a_out[q * A.g.N + n] = v;
}

template <int EL>
__global__ void __launch_bounds__(kBlock) k_fields(ElemArgs A, double* out_h, double* out_s,
                                                  double* out_d, double* out_k) {
  constexpr int D = ET<EL>::D, NQ = ET<EL>::NQ, NA = ET<EL>::NA;
  const Grid& g = A.g;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.N) return;
  const int ph = A.phase[n];
  Pos e;
  e.x = (int)(n % g.nx);
  e.y = (int)((n / g.nx) % g.ny);
  e.z = (int)(n / ((long long)g.nx * g.ny));
  double un[3][NA];
  load_nodal<EL>(g, A.u, e, un);
  for (int q = 0; q < NQ; ++q) {
    double H[3][3];
    grad_at<EL>(q, un, H);
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) H[i][j] += A.E[3 * i + j];
    const long long base = (n * NQ + q) * D * D;
    if (out_h)
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) out_h[base + i * D + j] = H[i][j];
    if (out_s) {
      const Sym eps = eval_strain<D>(H, A.mat, ph);
      const double kh = A.khist[q * g.N + n];
      const PointLaw P = eval_law<true>(eps, A.mat.lam[ph], A.mat.mu[ph], A.mat.E[ph],
                                        A.mat.damage[ph], A.mat.k0[ph], A.mat.kf[ph], kh);
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) out_s[base + i * D + j] = P.a * sym_at(P.s, i, j);
    }
    const double kh = A.khist[q * g.N + n];
    if (out_k) out_k[n * NQ + q] = kh;
    if (out_d) {
      double d = 0.0;
      if (A.mat.damage[ph]) {
        const double k0 = A.mat.k0[ph], kf = A.mat.kf[ph];
        d = fmin(fmax(kf / kh * (kh - k0) / (kf - k0), 0.0), 1.0);
      }
      out_d[n * NQ + q] = d;
    }
  }
}

// ---- sum-factorised Q1 gradient and divergence --------------------------
//
// With the 2-point rule, dN_a/dx at a point is (+-1) times the 1D linear
// interpolation weights in y and z, so the x-derivative at the 8 points
// takes 4 differences along x and two interpolations (y, then z) and has
// only 4 distinct values (it does not depend on the x Gauss point); the same
// holds for y and z. G[c][j][m][n] is the derivative of component c along j
// at the two remaining Gauss coordinates (m, n) in increasing axis order:
// j = x: (gy, gz); j = y: (gx, gz); j = z: (gx, gy).
// The divergence is the transpose: point values summed over the Gauss
// coordinate along j, then the transposed interpolations, then +-1 onto the
// two node layers along j.

// 1D interpolation of (f0 at node 0, f1 at node 1) to Gauss point g.
template <typename R>
__device__ __forceinline__ R interp(R f0, R f1, int g) {
  const R w1 = g ? R(kG1) : R(kG0);       // weight of node 1 at point g
  return f0 + w1 * (f1 - f0);
}

// v[a], a = ax + 2 ay + 4 az  ->  G[j][m][n]
template <typename R>
__device__ __forceinline__ void q1_grad_sf(const R (&v)[8], R (&G)[3][2][2]) {
  // along x: differences over (ay, az), interpolate y then z
  {
    R t[2][2];
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
        t[gy][az] = interp(v[1 + 4 * az] - v[0 + 4 * az], v[3 + 4 * az] - v[2 + 4 * az], gy);
#pragma unroll
    for (int gy = 0; gy < 2; ++gy)
#pragma unroll
      for (int gz = 0; gz < 2; ++gz) G[0][gy][gz] = interp(t[gy][0], t[gy][1], gz);
  }
  // along y: differences over (ax, az), interpolate x then z
  {
    R t[2][2];
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
      for (int gx = 0; gx < 2; ++gx)
        t[gx][az] = interp(v[2 + 4 * az] - v[0 + 4 * az], v[3 + 4 * az] - v[1 + 4 * az], gx);
#pragma unroll
    for (int gx = 0; gx < 2; ++gx)
#pragma unroll
      for (int gz = 0; gz < 2; ++gz) G[1][gx][gz] = interp(t[gx][0], t[gx][1], gz);
  }
  // along z: differences over (ax, ay), interpolate x then y
  {
    R t[2][2];
#pragma unroll
    for (int ay = 0; ay < 2; ++ay)
#pragma unroll
      for (int gx = 0; gx < 2; ++gx)
        t[gx][ay] = interp(v[4 + 2 * ay] - v[0 + 2 * ay], v[5 + 2 * ay] - v[1 + 2 * ay], gx);
#pragma unroll
    for (int gx = 0; gx < 2; ++gx)
#pragma unroll
      for (int gy = 0; gy < 2; ++gy) G[2][gx][gy] = interp(t[gx][0], t[gx][1], gy);
  }
}

// Transpose of interp for both Gauss points: values r0, r1 at points 0, 1
// give the nodal sums n0 = kG1 r0 + kG0 r1 and n1 = kG0 r0 + kG1 r1 (the
// weight of node 1 at point g is kG0 for g = 0 and kG1 for g = 1).
template <typename R>
__device__ __forceinline__ void interp_t2(R r0, R r1, R& n0, R& n1) {
  n0 = R(kG1) * r0 + R(kG0) * r1;
  n1 = R(kG0) * r0 + R(kG1) * r1;
}

// T[j][m][n] (point values summed over the Gauss coordinate along j) -> f[a]
// (assigned: the x part writes every node once, y and z add to it)
template <typename R>
__device__ __forceinline__ void q1_div_sf(const R (&T)[3][2][2], R (&f)[8]) {
  // x: T[0][gy][gz] -> z transposed -> y transposed -> -1 / +1 on ax = 0 / 1
  {
    R u[2][2], w[2][2];                      // u[gy][az], w[ay][az]
#pragma unroll
    for (int gy = 0; gy < 2; ++gy) interp_t2(T[0][gy][0], T[0][gy][1], u[gy][0], u[gy][1]);
#pragma unroll
    for (int az = 0; az < 2; ++az) interp_t2(u[0][az], u[1][az], w[0][az], w[1][az]);
#pragma unroll
    for (int ay = 0; ay < 2; ++ay)
#pragma unroll
      for (int az = 0; az < 2; ++az) {
        f[1 + 2 * ay + 4 * az] = w[ay][az];
        f[0 + 2 * ay + 4 * az] = -w[ay][az];
      }
  }
  // y: T[1][gx][gz] -> z transposed -> x transposed -> -1 / +1 on ay = 0 / 1
  {
    R u[2][2], w[2][2];                      // u[gx][az], w[ax][az]
#pragma unroll
    for (int gx = 0; gx < 2; ++gx) interp_t2(T[1][gx][0], T[1][gx][1], u[gx][0], u[gx][1]);
#pragma unroll
    for (int az = 0; az < 2; ++az) interp_t2(u[0][az], u[1][az], w[0][az], w[1][az]);
#pragma unroll
    for (int ax = 0; ax < 2; ++ax)
#pragma unroll
      for (int az = 0; az < 2; ++az) {
        f[ax + 2 + 4 * az] += w[ax][az];
        f[ax + 0 + 4 * az] -= w[ax][az];
      }
  }
  // z: T[2][gx][gy] -> y transposed -> x transposed -> -1 / +1 on az = 0 / 1
  {
    R u[2][2], w[2][2];                      // u[gx][ay], w[ax][ay]
#pragma unroll
    for (int gx = 0; gx < 2; ++gx) interp_t2(T[2][gx][0], T[2][gx][1], u[gx][0], u[gx][1]);
#pragma unroll
    for (int ay = 0; ay < 2; ++ay) interp_t2(u[0][ay], u[1][ay], w[0][ay], w[1][ay]);
#pragma unroll
    for (int ax = 0; ax < 2; ++ax)
#pragma unroll
      for (int ay = 0; ay < 2; ++ay) {
        f[ax + 2 * ay + 4] += w[ax][ay];
        f[ax + 2 * ay + 0] -= w[ax][ay];
      }
  }
}

// Element mask word written by the residual pass for the Hessian: bits 0-7
// the softening points (as the soft mask), bits 8-10 the phase, bit 15 set
// when a = 1 at all 8 points (an intact element: its tangent is C and its
// a values are not read).
constexpr unsigned kIntact = 0x8000u;

// ---- brick kernels (Q1) ---------------------------------------------------
//
// One block per brick of BX x BY x BZ nodes. The block computes the
// (kB+1)^3 elements whose nodes include its own (one layer of halo elements
// on the low side of each axis, recomputed by the neighbouring block as
// well), one element per thread, with the nodal inputs staged in LDS. The
// element forces are added to the owned nodes in eight phases, one per local
// node a: within a phase the map element -> node e + o_a is one-to-one, so no
// two threads touch the same accumulator and the order of the additions is
// fixed. Per-element outputs and reduction terms come from the elements the
// brick owns (those whose lowest corner is one of its nodes).
//   k_hessian    : f = K v = D^T B D v;  rows {v.Kv, |D v|^2}
//   k_brick      : f = D^T sigma(E + D u), a/c' written;  rows RES_*
//   k_trial      : sums over the points only (no halo elements): rows TRI_*
// Brick shapes (nodes BX x BY x BZ; the block runs one thread per element of
// the (BX+1)(BY+1)(BZ+1) element brick, rounded up to whole wavefronts).
template <int BX, int BY, int BZ> struct BrickShape {
  static constexpr int tile = (BX + 2) * (BY + 2) * (BZ + 2);      // staged nodes
  static constexpr int own = BX * BY * BZ;                          // owned nodes
  static constexpr int elems = (BX + 1) * (BY + 1) * (BZ + 1);
  static constexpr int threads = (elems + 63) / 64 * 64;
};

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// Give every XCD a contiguous run of bricks so that the halos neighbouring
// bricks share are fetched once into that XCD's L2.
__device__ __forceinline__ int xcd_brick(int b, int nb) {
  const int q = nb / 8;
  if (b >= 8 * q) return b;
  return (b % 8) * q + b / 8;
}

__device__ __forceinline__ int wrap(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// Full gradient at point q of the element whose lowest tile node is t0, from
// a staged field (three components), plus an optional constant.
template <int TILE, typename R>
__device__ __forceinline__ void tile_grad(const R (*f)[TILE], int q, int t0, int sy, int sz,
                                          R (&H)[3][3]) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ti = t0 + (a & 1) + ((a >> 1) & 1) * sy + ((a >> 2) & 1) * sz;
    const R v0 = f[0][ti], v1 = f[1][ti], v2 = f[2][ti];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const R w = q1b<R>().v[q][a][j];
      H[0][j] += w * v0;
      H[1][j] += w * v1;
      H[2][j] += w * v2;
    }
  }
}

template <int MODE, int NV, int BX, int BY, int BZ, bool FULL, bool TENS>
__global__ void __launch_bounds__((BrickShape<BX, BY, BZ>::threads)) k_brick(ElemArgs A) {
  constexpr int kTile = BrickShape<BX, BY, BZ>::tile, kOwn = BrickShape<BX, BY, BZ>::own;
  const Grid& g = A.g;
  // one LDS area: the staged u tile su[3][kTile], then the element forces
  // F[8][3][kElems] (corner, component, element)
  constexpr int kElems = BrickShape<BX, BY, BZ>::elems;
  constexpr int kLds = 3 * kTile > 24 * kElems ? 3 * kTile : 24 * kElems;
  __shared__ double lds[kLds];
  double (*su)[kTile] = reinterpret_cast<double (*)[kTile]>(lds);
  const int nbx = (g.nx + BX - 1) / BX, nby = (g.ny + BY - 1) / BY;
  const int brick = xcd_brick(blockIdx.x, gridDim.x);
  const int bxi = brick % nbx, byi = (brick / nbx) % nby, bzi = brick / (nbx * nby);
  const int x0 = bxi * BX, y0 = byi * BY, z0 = bzi * BZ;
  const int bx = FULL ? BX : min(BX, g.nx - x0), by = FULL ? BY : min(BY, g.ny - y0),
            bz = FULL ? BZ : min(BZ, g.nz - z0);            // FULL: whole bricks only
  const int tx = bx + 2, ty = by + 2, tz = bz + 2;          // staged node tile
  const int ex_n = bx + 1, ey_n = by + 1, ez_n = bz + 1;    // element brick
  const int tid = threadIdx.x;
  constexpr int nt = BrickShape<BX, BY, BZ>::threads;
  const int ntile = tx * ty * tz;
  // local tile node l <-> global node (origin - 1 + l) mod n
  auto tile_node = [&](int i) {
    const int lx = i % tx, ly = (i / tx) % ty, lz = i / (tx * ty);
    return lin(g, wrap(x0 - 1 + lx, g.nx), wrap(y0 - 1 + ly, g.ny), wrap(z0 - 1 + lz, g.nz));
  };
  // stage a nodal field on the tile: every load of a thread is issued before
  // its LDS stores
  constexpr int kIt = (kTile + BrickShape<BX, BY, BZ>::threads - 1) / BrickShape<BX, BY, BZ>::threads;
  auto stage = [&](const double* __restrict__ src, double (*dst)[kTile]) {
    double r[kIt][3];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int i = tid + it * nt;
      if (i < ntile) {
        const long long n = tile_node(i);
#pragma unroll
        for (int c = 0; c < 3; ++c) r[it][c] = src[c * g.N + n];
      }
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int i = tid + it * nt;
      if (i < ntile) {
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[c][i] = r[it][c];
      }
    }
  };
  // this thread's element
  const int ne = ex_n * ey_n * ez_n;
  const bool active = tid < ne;
  const int ex = tid % ex_n, ey = (tid / ex_n) % ey_n, ez = tid / (ex_n * ey_n);
  long long eg = 0;
  int ph = 0;
  double kh[8];        // the history of the element's points, loaded with the tile
  if (active) {
    eg = lin(g, wrap(x0 - 1 + ex, g.nx), wrap(y0 - 1 + ey, g.ny), wrap(z0 - 1 + ez, g.nz));
    ph = A.phase[eg];
#pragma unroll
    for (int q = 0; q < 8; ++q) kh[q] = A.khist[q * g.N + eg];
  }
  stage(A.u, su);
  __syncthreads();
  double f[3][8];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 8; ++a) f[i][a] = 0.0;
  double red[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) red[k] = 0.0;
  if (active) {
    const double lam = A.mat.lam[ph], mu = A.mat.mu[ph];
    const int t0 = ex + tx * (ey + ty * ez);
    const int sy = tx, sz = tx * ty;
    const bool owned = ex >= 1 && ey >= 1 && ez >= 1;
    double Em[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Em[i][j] = A.E[3 * i + j];
    // sum-factorised gradient of u at the 8 points (as in the Hessian)
    double G[3][3][2][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double v[8];
#pragma unroll
      for (int a = 0; a < 8; ++a)
        v[a] = su[c][t0 + (a & 1) + ((a >> 1) & 1) * sy + ((a >> 2) & 1) * sz];
      q1_grad_sf(v, G[c]);
    }
    unsigned soft = 0;   // bit q: c' != 0 at point q
    bool intact = true;  // a = 1 at every point
    // T[c][j][m][n]: sigma_cj summed over the Gauss coordinate along j
    double T[3][3][2][2];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int gx = q & 1, gy = (q >> 1) & 1, gz = (q >> 2) & 1;
      double H[3][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        H[c][0] = Em[c][0] + G[c][0][gy][gz];
        H[c][1] = Em[c][1] + G[c][1][gx][gz];
        H[c][2] = Em[c][2] + G[c][2][gx][gy];
      }
      const PointLaw P = eval_law<TENS>(eval_strain<3>(H, A.mat, ph), lam, mu, A.mat.E[ph],
                                        A.mat.damage[ph], A.mat.k0[ph], A.mat.kf[ph], kh[q]);
      Sym tau;
#pragma unroll
      for (int k = 0; k < 6; ++k) tau.v[k] = P.a * P.s.v[k];
      if (owned) {
        A.a_out[q * g.N + eg] = P.a;
        intact = intact && P.a == 1.0;
        if (P.cp != 0.0) {
          // rank-one factor of the softening term (c' > 0 where loading)
          soft |= 1u << q;
          const double r = sqrt(P.cp);
#pragma unroll
          for (int k = 0; k < 6; ++k) A.sw_out[(q * 6 + k) * g.N + eg] = r * P.s.v[k];
          if (TENS) {
            // the second factor sqrt(c') n of a tangent that is not symmetric
#pragma unroll
            for (int k = 0; k < 6; ++k) A.sn_out[(q * 6 + k) * g.N + eg] = r * P.n.v[k];
          }
          red[RES_NSOFT] += 1.0;
        }
        double hh = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) hh += H[i][j] * H[i][j];
#pragma unroll
        for (int k = 0; k < 6; ++k) red[RES_S0 + k] += tau.v[k];
        red[RES_SS] += sym_dot(tau, tau);
        red[RES_HH] += hh;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double t0c = sym_at(tau, c, 0), t1c = sym_at(tau, c, 1), t2c = sym_at(tau, c, 2);
        if (gx == 0) T[c][0][gy][gz] = t0c; else T[c][0][gy][gz] += t0c;
        if (gy == 0) T[c][1][gx][gz] = t1c; else T[c][1][gx][gz] += t1c;
        if (gz == 0) T[c][2][gx][gy] = t2c; else T[c][2][gx][gy] += t2c;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) q1_div_sf(T[c], f[c]);
    if (owned) {
      A.soft_out[eg] = (uint8_t)soft;
      A.emask_out[eg] = (uint16_t)(soft | ((unsigned)ph << 8) | (intact ? kIntact : 0u));
    }
  }
  // Assembly: every owned node adds the forces of its 8 elements in the
  // fixed order of the corner a; the element forces go through the tile's
  // LDS once every element has read the tile.
  static_assert(kOwn <= nt, "one owned node per thread");
  __syncthreads();
  if (active) {
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) lds[(a * 3 + c) * kElems + tid] = f[c][a];
  }
  __syncthreads();
  if (tid < bx * by * bz) {
    const int lx = tid % bx, ly = (tid / bx) % by, lz = tid / (bx * by);
    const long long n = lin(g, x0 + lx, y0 + ly, z0 + lz);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int e = (lx + 1 - (a & 1)) + ex_n * ((ly + 1 - ((a >> 1) & 1)) +
                                                   ey_n * (lz + 1 - ((a >> 2) & 1)));
        v += lds[(a * 3 + c) * kElems + e];
      }
      A.f[c * g.N + n] = v;
    }
  }
  block_reduce_store<NV>(red, A.red.partials);
}

// Trial evaluation at u + v for the trust-region ratio (eq. rho_bar): per
// point of the elements the brick owns, with H = E + D u, p = D v and the
// history frozen,
//   TRI_SP  sigma(H) : p = a (s:p),      s = C : eps(H)
//   TRI_PBP p : B(H) : p = a (p:C:p) - c' (n:p)(s:p), n = s for the energy
//           norm (w:p)^2 with w = sqrt(c') s; TENS: (w:p)(w_n:p), w_n = sqrt(c') n
//   TRI_STP sigma(H + p) : p
//   TRI_PP  |p|^2,  TRI_HH |H + p|^2
// No nodal output, so no halo elements: one thread per owned element, the
// nodes of u and v staged on the (BX+1)(BY+1)(BZ+1) tile.
template <int BX, int BY, int BZ, bool FULL, bool TENS>
__global__ void __launch_bounds__(BX * BY * BZ) k_trial(ElemArgs A) {
  constexpr int kTile = (BX + 1) * (BY + 1) * (BZ + 1);
  const Grid& g = A.g;
  __shared__ double su[3][kTile];
  __shared__ double sv[3][kTile];
  const int nbx = (g.nx + BX - 1) / BX, nby = (g.ny + BY - 1) / BY;
  const int brick = xcd_brick(blockIdx.x, gridDim.x);
  const int bxi = brick % nbx, byi = (brick / nbx) % nby, bzi = brick / (nbx * nby);
  const int x0 = bxi * BX, y0 = byi * BY, z0 = bzi * BZ;
  const int bx = FULL ? BX : min(BX, g.nx - x0), by = FULL ? BY : min(BY, g.ny - y0),
            bz = FULL ? BZ : min(BZ, g.nz - z0);            // FULL: whole bricks only
  const int tx = bx + 1, ty = by + 1, tz = bz + 1;          // staged node tile
  const int tid = threadIdx.x;
  constexpr int nt = BX * BY * BZ;
  const int ntile = tx * ty * tz;
  for (int i = tid; i < ntile; i += nt) {
    const int lx = i % tx, ly = (i / tx) % ty, lz = i / (tx * ty);
    const long long n = lin(g, wrap(x0 + lx, g.nx), wrap(y0 + ly, g.ny), wrap(z0 + lz, g.nz));
    double r[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = A.u[c * g.N + n];
      r[3 + c] = A.v[c * g.N + n];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      su[c][i] = r[c];
      sv[c][i] = r[3 + c];
    }
  }
  __syncthreads();
  double red[TRI_NV];
#pragma unroll
  for (int k = 0; k < TRI_NV; ++k) red[k] = 0.0;
  const int ex = tid % BX, ey = (tid / BX) % BY, ez = tid / (BX * BY);
  if (ex < bx && ey < by && ez < bz) {
    const long long eg = lin(g, x0 + ex, y0 + ey, z0 + ez);
    const int ph = A.phase[eg];
    const unsigned soft = A.soft[eg];
    const double lam = A.mat.lam[ph], mu = A.mat.mu[ph];
    const int t0 = ex + tx * (ey + ty * ez);
    const int sy = tx, sz = tx * ty;
#pragma unroll 1
    for (int q = 0; q < 8; ++q) {
      // the point's state first, so that its loads overlap the gradients:
      // kappa_hist, a and, at a softening point, w = sqrt(c') s
      const bool sq = (soft >> q) & 1u;
      const double kh = A.khist[q * g.N + eg];
      const double ao = A.a[q * g.N + eg];
      Sym w, wn;
#pragma unroll
      for (int k = 0; k < 6; ++k) w.v[k] = wn.v[k] = 0.0;
      if (sq) {
#pragma unroll
        for (int k = 0; k < 6; ++k) w.v[k] = A.sw[(q * 6 + k) * g.N + eg];
        if (TENS) {
#pragma unroll
          for (int k = 0; k < 6; ++k) wn.v[k] = A.sn[(q * 6 + k) * g.N + eg];
        }
      }
      double H[3][3], p[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          H[i][j] = A.E[3 * i + j];
          p[i][j] = A.Pu ? A.Pu[3 * i + j] : 0.0;   // the step's uniform part (mean-stress control)
        }
      tile_grad<kTile>(su, q, t0, sy, sz, H);
      tile_grad<kTile>(sv, q, t0, sy, sz, p);
      double Ht[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Ht[i][j] = H[i][j] + p[i][j];
      const PointLaw P = eval_law<TENS>(eval_strain<3>(Ht, A.mat, ph), lam, mu, A.mat.E[ph],
                                        A.mat.damage[ph], A.mat.k0[ph], A.mat.kf[ph], kh);
      Sym tau;
#pragma unroll
      for (int k = 0; k < 6; ++k) tau.v[k] = P.a * P.s.v[k];
      const Sym ps = sym_of<3>(p);
      const Sym so = c_contract(eval_strain<3>(H, A.mat, ph), lam, mu);
      const double s_p = sym_dot(so, ps);
      const double trp = ps.v[0] + ps.v[1] + ps.v[2];
      const double pCp = lam * trp * trp + 2.0 * mu * sym_dot(ps, ps);
      double pp = 0.0, hh = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          pp += p[i][j] * p[i][j];
          hh += Ht[i][j] * Ht[i][j];
        }
      red[TRI_SP] += ao * s_p;
      // c' (n:p)(s:p) = (w_n:p)(w:p)
      double soft_pp = 0.0;
      if (sq) {
        const double wp = sym_dot(w, ps);
        soft_pp = TENS ? sym_dot(wn, ps) * wp : wp * wp;
      }
      red[TRI_PBP] += ao * pCp - soft_pp;
      red[TRI_STP] += sym_dot(tau, ps);
      red[TRI_PP] += pp;
      red[TRI_HH] += hh;
    }
  }
  block_reduce_store<TRI_NV>(red, A.red.partials);
}

// Hessian K v = D^T B D v at the state, in FP64 (R = double) or, for the
// mixed-precision CG, FP32 (R = float) with the reduction terms {v.Kv, |D v|^2}
// accumulated in FP64. The same brick scheme as k_brick, with the direction
// staged on the tile. The gradient of v and the divergence are
// sum-factorised. The tangent at a point is a C minus the rank-one softening
// term, which the residual pass stored as w = sqrt(c') s at the points where
// c' != 0 (bit q of the element's soft mask): B : e = a C : e - (w : e) w.
// NS (a tensile-masking phase is present): the tangent is not symmetric and
// the residual pass also stored w_n = sqrt(c') n, so B : e = a C : e -
// (w_n : e) w. The state displacement is not read.
// FP32: at most 128 VGPRs (4 waves per SIMD), which the FP32 kernel fits
// without spills; FP64 keeps the compiler's choice.
template <typename R> constexpr int hessian_waves_per_eu() { return sizeof(R) == 4 ? 4 : 1; }

// Forces of one element under the Hessian: the sum-factorised gradient of
// the staged direction, the tangent at the 8 points (a C : e minus the
// rank-one softening term at the points of the element's mask), and the
// sum-factorised divergence into f[c][corner]. tile(c, i) reads component c
// of staged node i; corner a = ax + 2 ay + 4 az sits at t0 + ax + ay sy + az sz.
// dd receives sum |D v|^2 over the element's points if `owned` (else 0).
// MS (mean-stress control): the uniform U (3x3) is added to D v at every
// point, and tv receives the element's point sums of the tangent's output
// (Voigt xx yy zz yz xz xy) if `owned`.
template <typename R, bool NS, bool MS = false, typename Tile>
__device__ __forceinline__ void hess_element(const Tile& tile, int t0, int sy, int sz, R lam, R mu,
                                             const R (&aq)[8], unsigned soft,
                                             const double* __restrict__ w_e,
                                             const double* __restrict__ n_e, long long N,
                                             R (&f)[3][8], double& dd, bool owned,
                                             const double* __restrict__ U = nullptr,
                                             double* tv = nullptr) {
  R G[3][3][2][2];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R v[8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
      v[a] = tile(c, t0 + (a & 1) + ((a >> 1) & 1) * sy + ((a >> 2) & 1) * sz);
    q1_grad_sf(v, G[c]);
  }
  dd = 0.0;
  if (owned) {
    // |D v|^2 over the points: each G value is the gradient entry of the two
    // points that differ only in the Gauss coordinate along j
    double s2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int k = 0; k < 2; ++k) s2 += (double)G[c][j][m][k] * (double)G[c][j][m][k];
    dd = 2.0 * s2;
  }
  // T[c][j][m][n]: tau_cj summed over the Gauss coordinate along j; an entry
  // is written at the first of its two points and added at the second
  R T[3][3][2][2];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int gx = q & 1, gy = (q >> 1) & 1, gz = (q >> 2) & 1;
    R dH[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dH[c][0] = G[c][0][gy][gz];
      dH[c][1] = G[c][1][gx][gz];
      dH[c][2] = G[c][2][gx][gy];
    }
    if constexpr (MS) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < 3; ++j) dH[c][j] += (R)U[3 * c + j];
    }
    // tau = a C : e - (w : e) w with e = sym(dH); h_ij = 2 e_ij
    const R h01 = dH[0][1] + dH[1][0], h02 = dH[0][2] + dH[2][0], h12 = dH[1][2] + dH[2][1];
    const R al = aq[q] * lam, am = aq[q] * mu;
    const R ltr = al * (dH[0][0] + dH[1][1] + dH[2][2]), am2 = am + am;
    R t00 = ltr + am2 * dH[0][0], t11 = ltr + am2 * dH[1][1], t22 = ltr + am2 * dH[2][2];
    R t01 = am * h01, t02 = am * h02, t12 = am * h12;
    if ((soft >> q) & 1u) {
      R w[6], wn[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) w[k] = (R)w_e[(q * 6 + k) * N];
      if (NS) {
#pragma unroll
        for (int k = 0; k < 6; ++k) wn[k] = (R)n_e[(q * 6 + k) * N];
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) wn[k] = w[k];
      }
      const R we = wn[0] * dH[0][0] + wn[1] * dH[1][1] + wn[2] * dH[2][2] + wn[3] * h01 +
                   wn[4] * h02 + wn[5] * h12;
      t00 -= we * w[0];
      t11 -= we * w[1];
      t22 -= we * w[2];
      t01 -= we * w[3];
      t02 -= we * w[4];
      t12 -= we * w[5];
    }
    const R tau[3][3] = {{t00, t01, t02}, {t01, t11, t12}, {t02, t12, t22}};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (gx == 0) T[c][0][gy][gz] = tau[c][0]; else T[c][0][gy][gz] += tau[c][0];
      if (gy == 0) T[c][1][gx][gz] = tau[c][1]; else T[c][1][gx][gz] += tau[c][1];
      if (gz == 0) T[c][2][gx][gy] = tau[c][2]; else T[c][2][gx][gy] += tau[c][2];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) q1_div_sf(T[c], f[c]);
  if constexpr (MS) {
    if (owned) {
      // sum over the 8 points of tau_ij: T[i][j] already sums along j
      auto total = [&](int i, int j) {
        return (double)T[i][j][0][0] + (double)T[i][j][0][1] + (double)T[i][j][1][0] +
               (double)T[i][j][1][1];
      };
      tv[0] += total(0, 0);
      tv[1] += total(1, 1);
      tv[2] += total(2, 2);
      tv[3] += total(1, 2);
      tv[4] += total(0, 2);
      tv[5] += total(0, 1);
    }
  }
}

// The element state the Hessian reads: phase and softening mask from the
// mask word, a at the 8 points (1 without a load at intact elements).
template <typename R>
__device__ __forceinline__ void hess_state(const HessArgs<R>& A, long long eg, int& ph,
                                           unsigned& soft, R (&aq)[8]) {
  const unsigned m = A.emask[eg];
  ph = (m >> 8) & 7u;
  soft = m & 0xffu;
  if (m & kIntact) {
#pragma unroll
    for (int q = 0; q < 8; ++q) aq[q] = R(1);
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) aq[q] = A.a[q * A.g.N + eg];
  }
}

// The node sum of the assembly has one fixed order in every Hessian kernel:
// the four corners with az = 0 (the element layer of the node), then the
// four with az = 1 (the layer below), each group summed in corner order
// ((f0 + f1) + f2) + f3, then the two group sums added. It is what lets the
// column kernel carry the az = 1 sums from one layer to the next.

// The canonical tile sums of a brick (hfe_internal.h). The values are staged
// by thread: st[t] is d.Kd of node thread t (t = x + bx (y + by z)), and
// st[BX*BY*BZ + k * E + t] value k (|Dd|^2, then the NE - 1 tails) of element
// thread t (t = (x+1) + (bx+1) ((y+1) + (by+1) (z+1)) for the element anchored
// at node x, y, z; E elements per brick). One thread per tile position q adds
// its column in ascending z onto 0.0, the tile's 32 columns are added by
// tile_sum32, and lane q = 31 writes the tile's row: d.Kd and |Dd|^2 to
// rows, the tails to tail_rows (6 per row). The brick's extents are
// multiples of the tile's, so its tiles are whole canonical tiles or those
// the grid cuts.
template <int BX, int BY, int BZ, int NE>
__device__ __forceinline__ void brick_tile_rows(const double* st, int bx, int by, int bz, int x0,
                                                int y0, int z0, const Grid& g, double* rows,
                                                double* tail_rows) {
  static_assert(BX % kTileX == 0 && BY % kTileY == 0 && BZ % kTileZ == 0, "whole tiles");
  static_assert(HES_DKD == 0 && HES_DD == 1 && HES_NV == 2, "row layout");
  constexpr int TX = BX / kTileX, TY = BY / kTileY, TZ = BZ / kTileZ, NV = 1 + NE;
  constexpr int kOwn = BX * BY * BZ, kElems = (BX + 1) * (BY + 1) * (BZ + 1);
  constexpr int nsum = TX * TY * TZ * kTileQ;
  const int tid = threadIdx.x;
  if (tid >= (nsum + 63) / 64 * 64) return;
  const int q = tid & (kTileQ - 1), tl = tid / kTileQ;
  const int ix = tl % TX, iy = (tl / TX) % TY, iz = tl / (TX * TY);
  const int x = ix * kTileX + (q % kTileX), y = iy * kTileY + q / kTileX;
  double c[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) c[k] = 0.0;
  if (tid < nsum && x < bx && y < by) {
#pragma unroll
    for (int zz = 0; zz < kTileZ; ++zz) {
      const int z = iz * kTileZ + zz;
      if (z < bz) {
        c[0] += st[x + bx * (y + by * z)];
        const int e = (x + 1) + (bx + 1) * ((y + 1) + (by + 1) * (z + 1));
#pragma unroll
        for (int k = 0; k < NE; ++k) c[1 + k] += st[kOwn + k * kElems + e];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) c[k] = tile_sum32(c[k]);
  if (tid < nsum && q == kTileQ - 1 && ix * kTileX < bx && iy * kTileY < by && iz * kTileZ < bz) {
    const long long row = tile_row(g, x0 / kTileX + ix, y0 / kTileY + iy, z0 / kTileZ + iz);
    rows[row * HES_NV + HES_DKD] = c[0];
    rows[row * HES_NV + HES_DD] = c[1];
#pragma unroll
    for (int k = 2; k < NV; ++k) tail_rows[row * 6 + (k - 2)] = c[k];
  }
}

template <typename R, int BX, int BY, int BZ, bool FULL, bool NS, bool MS>
__global__ void __launch_bounds__((BrickShape<BX, BY, BZ>::threads), hessian_waves_per_eu<R>())
    k_hessian(HessArgs<R> A) {
  constexpr int kTile = BrickShape<BX, BY, BZ>::tile, kOwn = BrickShape<BX, BY, BZ>::own;
  const Grid& g = A.g;
  if (A.cg && A.cg->done) return;
  // One LDS area serves first as the staged direction tile sv[3][kTile], then
  // as the element forces F[8][3][kElems] (corner, component, element).
  constexpr int kElems = BrickShape<BX, BY, BZ>::elems;
  constexpr int kLds = 3 * kTile > 24 * kElems ? 3 * kTile : 24 * kElems;
  __shared__ __align__(16) R lds[kLds];
  R (*sv)[kTile] = reinterpret_cast<R (*)[kTile]>(lds);
  const int nbx = (g.nx + BX - 1) / BX, nby = (g.ny + BY - 1) / BY;
  const int brick = xcd_brick(blockIdx.x, gridDim.x);
  const int bxi = brick % nbx, byi = (brick / nbx) % nby, bzi = brick / (nbx * nby);
  const int x0 = bxi * BX, y0 = byi * BY, z0 = bzi * BZ;
  // FULL: every brick is whole (the grid is a multiple of the brick), so the
  // brick extents and all index arithmetic on them are compile-time constants
  const int bx = FULL ? BX : min(BX, g.nx - x0), by = FULL ? BY : min(BY, g.ny - y0),
            bz = FULL ? BZ : min(BZ, g.nz - z0);
  const int tx = bx + 2, ty = by + 2, tz = bz + 2;
  const int ex_n = bx + 1, ey_n = by + 1, ez_n = bz + 1;
  const int tid = threadIdx.x;
  constexpr int nt = BrickShape<BX, BY, BZ>::threads;
  const int ntile = tx * ty * tz;
  auto tile_node = [&](int i) {
    const int lx = i % tx, ly = (i / tx) % ty, lz = i / (tx * ty);
    return lin(g, wrap(x0 - 1 + lx, g.nx), wrap(y0 - 1 + ly, g.ny), wrap(z0 - 1 + lz, g.nz));
  };
  constexpr int kIt = (kTile + BrickShape<BX, BY, BZ>::threads - 1) / BrickShape<BX, BY, BZ>::threads;
  auto stage = [&](const R* __restrict__ src, R (*dst)[kTile]) {
    R r[kIt][3];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int i = tid + it * nt;
      if (i < ntile) {
        const long long n = tile_node(i);
#pragma unroll
        for (int c = 0; c < 3; ++c) r[it][c] = src[c * g.N + n];
      }
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int i = tid + it * nt;
      if (i < ntile) {
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[c][i] = r[it][c];
      }
    }
  };
  // this thread's element and its state, loaded before the tile so that all
  // these loads are in flight together
  const int ne = ex_n * ey_n * ez_n;
  const bool active = tid < ne;
  const int ex = tid % ex_n, ey = (tid / ex_n) % ey_n, ez = tid / (ex_n * ey_n);
  long long eg = 0;
  int ph = 0;
  unsigned soft = 0;
  R aq[8];
  if (active) {
    eg = lin(g, wrap(x0 - 1 + ex, g.nx), wrap(y0 - 1 + ey, g.ny), wrap(z0 - 1 + ez, g.nz));
    hess_state(A, eg, ph, soft, aq);
  }
  stage(A.v, sv);
  __syncthreads();
  R f[3][8];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 8; ++a) f[i][a] = R(0);
  double dd = 0.0;
  double tv[MS ? 6 : 1] = {};
  if (active) {
    const R lam = (R)A.mat.lam[ph], mu = (R)A.mat.mu[ph];
    const int t0 = ex + tx * (ey + ty * ez);
    auto tile = [&](int c, int i) { return sv[c][i]; };
    hess_element<R, NS, MS>(tile, t0, tx, tx * ty, lam, mu, aq, soft, A.sw + eg,
                            NS ? A.sn + eg : nullptr, g.N, f, dd, ex >= 1 && ey >= 1 && ez >= 1,
                            A.U, tv);
  }
  // Assembly. Every owned node adds the forces of its 8 elements in the
  // fixed order of corner_sum (the same for every Hessian kernel). The
  // direction at the owned node is read from the tile first (for v.Kv), then
  // the tile's LDS is reused for the element forces.
  static_assert(kOwn <= nt, "one owned node per thread");
  const int nown = bx * by * bz;
  R vn[3] = {R(0), R(0), R(0)};
  int lx = 0, ly = 0, lz = 0;
  if (tid < nown) {
    lx = tid % bx;
    ly = (tid / bx) % by;
    lz = tid / (bx * by);
    const int ti = (lx + 1) + tx * ((ly + 1) + ty * (lz + 1));
#pragma unroll
    for (int c = 0; c < 3; ++c) vn[c] = sv[c][ti];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) lds[(a * 3 + c) * kElems + tid] = f[c][a];
  }
  __syncthreads();
  double dkd = 0.0;
  if (tid < nown) {
    const long long n = lin(g, x0 + lx, y0 + ly, z0 + lz);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // corner order of corner_sum: ((f0 + f1) + f2) + f3, the same for
      // f4..f7, then the two sums added
      R lo = R(0), hi = R(0);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int e = (lx + 1 - (a & 1)) + ex_n * ((ly + 1 - ((a >> 1) & 1)) +
                                                   ey_n * (lz + 1 - ((a >> 2) & 1)));
        const R x = lds[(a * 3 + c) * kElems + e];
        if (a == 0) lo = x; else if (a < 4) lo += x; else if (a == 4) hi = x; else hi += x;
      }
      const R v = lo + hi;
      A.f[c * g.N + n] = v;
      dkd += (double)v * (double)vn[c];
    }
  }
  // the per-tile sums: node and element values staged by thread in the LDS
  // area (its element forces are read), then summed per tile
  constexpr int kNe = MS ? 7 : 1;
  static_assert((kOwn + kNe * kElems) * sizeof(double) <= sizeof(lds), "tile staging fits");
  __syncthreads();
  double* st = reinterpret_cast<double*>(lds);
  if (tid < nown) st[tid] = dkd;
  if (active) {
    st[kOwn + tid] = dd;
    if constexpr (MS) {
#pragma unroll
      for (int k = 0; k < 6; ++k) st[kOwn + (1 + k) * kElems + tid] = tv[k];
    }
  }
  __syncthreads();
  brick_tile_rows<BX, BY, BZ, kNe>(st, bx, by, bz, x0, y0, z0, g, A.red.partials,
                                   A.red_tail.partials);
}

// ---- column-marching Hessian (Q1) -----------------------------------------
//
// One block per column of CX x CY owned nodes and `bz` node layers. The
// block walks the element layers of its column upwards, one per step: the
// (CX+1)(CY+1) elements of a layer (one per thread; a halo of one element
// on the low x and y sides is recomputed by the neighbouring column, one
// halo element layer below the column), their forces through LDS to the
// nodes. A node layer takes the az = 0 corners of the element layer it is
// the bottom of and the az = 1 corners of the layer below: the latter are
// summed one step earlier and carried in registers, so no element is
// computed twice along z. The direction is staged as a ring of two node
// layers; the next node layer and the next element layer's mask word are
// loaded while the current layer is computed. The node sums follow the
// fixed corner order, so the result has the bits of the brick kernels.
template <int CX, int CY> struct ColumnShape {
  static constexpr int tx = CX + 2, ty = CY + 2;
  static constexpr int layer = tx * ty;                     // staged nodes per layer
  static constexpr int ex = CX + 1, ey = CY + 1;
  static constexpr int elems = ex * ey;                     // elements per layer
  static constexpr int threads = (elems + 63) / 64 * 64;
  static constexpr int own = CX * CY;
  static constexpr int pre = (layer + threads - 1) / threads;
};

template <typename R, int CX, int CY, bool NS, bool MS>
__global__ void __launch_bounds__((ColumnShape<CX, CY>::threads), hessian_waves_per_eu<R>())
    k_hessian_col(HessArgs<R> A, int bz) {
  using S = ColumnShape<CX, CY>;
  const Grid& g = A.g;
  if (A.cg && A.cg->done) return;
  __shared__ R sv[3][2][S::layer];       // direction: component, ring slot, node
  __shared__ __align__(16) R F[24][S::elems];   // element forces: corner * 3 + component, element
  const int ncx = g.nx / CX, ncy = g.ny / CY;
  const int blk = xcd_brick(blockIdx.x, gridDim.x);
  const int cxi = blk % ncx, cyi = (blk / ncx) % ncy, czi = blk / (ncx * ncy);
  const int x0 = cxi * CX, y0 = cyi * CY, z0 = czi * bz;
  const int nzl = min(bz, g.nz - z0);    // owned node layers
  const int tid = threadIdx.x;
  const long long N = g.N, nxy = (long long)g.nx * g.ny;
  // staged node positions of this thread within a layer (xy offsets)
  long long sxy[S::pre];
#pragma unroll
  for (int it = 0; it < S::pre; ++it) {
    const int i = tid + it * S::threads;
    const int lx = i % S::tx, ly = i / S::tx;
    sxy[it] = i < S::layer ? wrap(x0 - 1 + lx, g.nx) + (long long)g.nx * wrap(y0 - 1 + ly, g.ny)
                           : 0;
  }
  // local node layer k is the global layer z0 - 1 + k; it sits in ring slot k & 1
  auto load_layer = [&](int k, R (&r)[S::pre][3]) {
    const long long zoff = (long long)wrap(z0 - 1 + k, g.nz) * nxy;
#pragma unroll
    for (int it = 0; it < S::pre; ++it)
      if (tid + it * S::threads < S::layer) {
#pragma unroll
        for (int c = 0; c < 3; ++c) r[it][c] = A.v[c * N + zoff + sxy[it]];
      }
  };
  auto store_layer = [&](int k, const R (&r)[S::pre][3]) {
#pragma unroll
    for (int it = 0; it < S::pre; ++it) {
      const int i = tid + it * S::threads;
      if (i < S::layer) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sv[c][k & 1][i] = r[it][c];
      }
    }
  };
  // this thread's element within a layer, and its owned node
  const bool active = tid < S::elems;
  const int ex = tid % S::ex, ey = tid / S::ex;
  const long long exy = wrap(x0 - 1 + ex, g.nx) + (long long)g.nx * wrap(y0 - 1 + ey, g.ny);
  const bool node = tid < S::own;
  const int lx = tid % CX, ly = tid / CX;
  const long long oxy = (x0 + lx) + (long long)g.nx * (y0 + ly);
  const int ti = (lx + 1) + S::tx * (ly + 1);             // owned node in a staged layer
  // element layer k (local) is the global layer z0 - 1 + k; its mask word
  auto elem_of = [&](int k) { return (long long)wrap(z0 - 1 + k, g.nz) * nxy + exy; };
  unsigned m_next = 0;
  {
    R r[S::pre][3];
    load_layer(0, r);
    store_layer(0, r);
    load_layer(1, r);
    store_layer(1, r);
    if (active) m_next = A.emask[elem_of(0)];
  }
  __syncthreads();
  R top[3] = {R(0), R(0), R(0)};        // az = 1 sums of the layer below, for node layer k
  // column sums of the current tile layer group (canonical tiles, 4 node
  // layers): this thread's node, and its element if the column owns it
  double dkd = 0.0, dd = 0.0;
  double tv[MS ? 6 : 1] = {};
  for (int k = 0; k <= nzl; ++k) {
    // element layer k: nodes k (bottom) and k + 1 (top); this step's loads
    // ahead of the arithmetic: node layer k + 2 and the next mask word
    R rn[S::pre][3];
    const bool more = k + 2 <= nzl + 1;
    if (more) load_layer(k + 2, rn);
    const unsigned m = m_next;
    if (active && k < nzl) m_next = A.emask[elem_of(k + 1)];
    R f[3][8];
    if (active) {
      const long long eg = elem_of(k);
      const int ph = (m >> 8) & 7u;
      const unsigned soft = m & 0xffu;
      R aq[8];
      if (m & kIntact) {
#pragma unroll
        for (int q = 0; q < 8; ++q) aq[q] = R(1);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) aq[q] = A.a[q * N + eg];
      }
      const R lam = (R)A.mat.lam[ph], mu = (R)A.mat.mu[ph];
      const int t0 = (k & 1) * S::layer + ex + S::tx * ey;
      const int sz = (k & 1) ? -S::layer : S::layer;       // to the other ring slot
      auto tile = [&](int c, int i) { return (&sv[c][0][0])[i]; };
      double de = 0.0;
      double te[MS ? 6 : 1] = {};
      hess_element<R, NS, MS>(tile, t0, S::tx, sz, lam, mu, aq, soft, A.sw + eg,
                              NS ? A.sn + eg : nullptr, N, f, de, k >= 1 && ex >= 1 && ey >= 1,
                              A.U, te);
      dd += de;
      if constexpr (MS) {
#pragma unroll
        for (int i = 0; i < 6; ++i) tv[i] += te[i];
      }
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) F[a * 3 + c][tid] = f[c][a];
    }
    // the direction at this thread's node of layer k (read before the ring
    // slot is refilled below)
    R vn[3] = {R(0), R(0), R(0)};
    if (node && k >= 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) vn[c] = sv[c][k & 1][ti];
    }
    __syncthreads();
    if (node) {
      double pn = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        R lo = R(0), hi = R(0);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int e = (lx + 1 - (a & 1)) + S::ex * (ly + 1 - ((a >> 1) & 1));
          const R x = F[a * 3 + c][e];
          if (a == 0) lo = x; else if (a < 4) lo += x; else if (a == 4) hi = x; else hi += x;
        }
        if (k >= 1) {
          // node layer k: the bottom corners (az = 0) of element layer k,
          // then the top sums carried from element layer k - 1
          const R v = lo + top[c];
          A.f[c * N + (long long)(z0 + k - 1) * nxy + oxy] = v;
          pn += (double)v * (double)vn[c];
        }
        top[c] = hi;
      }
      dkd += pn;
    }
    if (more) store_layer(k + 2, rn);    // slot k & 1: node layer k is done
    __syncthreads();
    // node layer z0 + k - 1 ends a canonical tile layer group (z0 is a
    // multiple of 4): the column sums go through F (free until the next
    // element layer) in tile order, and each tile's 32 columns are added as
    // in the brick kernels
    if (k >= 1 && (((k - 1) & (kTileZ - 1)) == kTileZ - 1 || k == nzl)) {
      constexpr int kNe = MS ? 7 : 1, kTx = CX / kTileX;
      static_assert(CX % kTileX == 0 && CY % kTileY == 0, "whole tiles");
      static_assert((S::own + kNe * S::elems) * sizeof(double) <= sizeof(F), "tile staging fits");
      // staged by thread: node thread t = x + CX y, element thread
      // t = (x+1) + (CX+1) (y+1) for the element anchored at node x, y
      double* st = reinterpret_cast<double*>(&F[0][0]);
      if (node) st[tid] = dkd;
      if (active) {
        st[S::own + tid] = dd;
        if constexpr (MS) {
#pragma unroll
          for (int i = 0; i < 6; ++i) st[S::own + (1 + i) * S::elems + tid] = tv[i];
        }
      }
      __syncthreads();
      if (tid < S::own) {     // S::own is a multiple of 64; lane bits 0..4 are q
        const int q = tid & (kTileQ - 1), tl = tid / kTileQ;
        const int x = (tl % kTx) * kTileX + q % kTileX, y = (tl / kTx) * kTileY + q / kTileX;
        double cs[1 + kNe];
        cs[0] = tile_sum32(st[x + CX * y]);
#pragma unroll
        for (int i = 0; i < kNe; ++i)
          cs[1 + i] = tile_sum32(st[S::own + i * S::elems + (x + 1) + S::ex * (y + 1)]);
        if (q == kTileQ - 1) {
          const long long row = tile_row(g, x0 / kTileX + tl % kTx, y0 / kTileY + tl / kTx,
                                         (z0 + k - 1) / kTileZ);
          A.red.partials[row * HES_NV + HES_DKD] = cs[0];
          A.red.partials[row * HES_NV + HES_DD] = cs[1];
          if constexpr (MS) {
#pragma unroll
            for (int i = 0; i < 6; ++i) A.red_tail.partials[row * 6 + i] = cs[2 + i];
          }
        }
      }
      __syncthreads();
      dkd = dd = 0.0;
#pragma unroll
      for (int i = 0; i < (MS ? 6 : 1); ++i) tv[i] = 0.0;
    }
  }
}

template <int MODE, int NV, int BX, int BY, int BZ>
hipError_t launch_brick_shape(const ElemArgs& A, hipStream_t s, int* nblocks) {
  const int nb = ((A.g.nx + BX - 1) / BX) * ((A.g.ny + BY - 1) / BY) * ((A.g.nz + BZ - 1) / BZ);
  *nblocks = nb;
  const bool full = A.g.nx % BX == 0 && A.g.ny % BY == 0 && A.g.nz % BZ == 0;
  const dim3 grid(nb), block(BrickShape<BX, BY, BZ>::threads);
  if (A.tens) {
    if (full) hipLaunchKernelGGL((k_brick<MODE, NV, BX, BY, BZ, true, true>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_brick<MODE, NV, BX, BY, BZ, false, true>), grid, block, 0, s, A);
  } else {
    if (full) hipLaunchKernelGGL((k_brick<MODE, NV, BX, BY, BZ, true, false>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_brick<MODE, NV, BX, BY, BZ, false, false>), grid, block, 0, s, A);
  }
  return hipGetLastError();
}

// Brick shape of the residual pass: 8x8x4 (448 threads) whatever Hessian
// shape is tuned, so that its block sums, and the Newton decisions taken on
// them, are the same under every tuning.
template <int MODE, int NV>
hipError_t launch_brick(const ElemArgs& A, hipStream_t s, int* nblocks) {
  return launch_brick_shape<MODE, NV, 8, 8, 4>(A, s, nblocks);
}

// Events armed for the next Hessian launch of this host thread (profiling).
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

// Launch a Hessian kernel; with events armed, through hipExtLaunchKernelGGL,
// which records them at the kernel's own start and end.
template <typename K, typename... Args>
void launch_hess(K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
  if (g_ev_start && g_ev_stop) {
    const hipEvent_t a = g_ev_start, b = g_ev_stop;
    g_ev_start = g_ev_stop = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
  }
}

template <typename R, int BX, int BY, int BZ>
hipError_t launch_hessian_shape(const HessArgs<R>& A, hipStream_t s, int* nblocks) {
  const int nb = ((A.g.nx + BX - 1) / BX) * ((A.g.ny + BY - 1) / BY) * ((A.g.nz + BZ - 1) / BZ);
  *nblocks = tile_count(A.g);   // partial rows: one per canonical tile
  const bool full = A.g.nx % BX == 0 && A.g.ny % BY == 0 && A.g.nz % BZ == 0;
  const dim3 grid(nb), block(BrickShape<BX, BY, BZ>::threads);
  if constexpr (std::is_same<R, double>::value) {
    if (A.U) {
      // mean-stress control: whole and ragged bricks of either law
      if (A.tens) {
        if (full) launch_hess(k_hessian<R, BX, BY, BZ, true, true, true>, grid, block, s, A);
        else launch_hess(k_hessian<R, BX, BY, BZ, false, true, true>, grid, block, s, A);
      } else {
        if (full) launch_hess(k_hessian<R, BX, BY, BZ, true, false, true>, grid, block, s, A);
        else launch_hess(k_hessian<R, BX, BY, BZ, false, false, true>, grid, block, s, A);
      }
      return hipGetLastError();
    }
  }
  if (A.tens) {
    if (full) launch_hess(k_hessian<R, BX, BY, BZ, true, true, false>, grid, block, s, A);
    else launch_hess(k_hessian<R, BX, BY, BZ, false, true, false>, grid, block, s, A);
  } else {
    if (full) launch_hess(k_hessian<R, BX, BY, BZ, true, false, false>, grid, block, s, A);
    else launch_hess(k_hessian<R, BX, BY, BZ, false, false, false>, grid, block, s, A);
  }
  return hipGetLastError();
}

// Column shapes of the marching Hessian (shape ids kBrickOnly..): owned
// nodes per layer CX x CY and node layers per block.
struct ColShape { int cx, cy, bz; };
constexpr ColShape kColShapes[kHessianShapes - kBrickOnly] = {
    {16, 16, 16}, {16, 16, 8}, {16, 8, 16}, {16, 8, 8}, {8, 8, 8}, {8, 8, 16}, {16, 8, 32},
    {16, 16, 32}};

template <typename R, int CX, int CY>
hipError_t launch_hessian_col(const HessArgs<R>& A, int bz, hipStream_t s, int* nblocks) {
  const Grid& g = A.g;
  if (g.nx % CX != 0 || g.ny % CY != 0 || bz < 1 || bz % kTileZ != 0) return hipErrorInvalidValue;
  const int nb = (g.nx / CX) * (g.ny / CY) * ((g.nz + bz - 1) / bz);
  *nblocks = tile_count(g);   // partial rows: one per canonical tile
  const dim3 grid(nb), block(ColumnShape<CX, CY>::threads);
  if constexpr (std::is_same<R, double>::value) {
    if (A.U) {
      if (A.tens) launch_hess(k_hessian_col<R, CX, CY, true, true>, grid, block, s, A, bz);
      else launch_hess(k_hessian_col<R, CX, CY, false, true>, grid, block, s, A, bz);
      return hipGetLastError();
    }
  }
  if (A.tens) launch_hess(k_hessian_col<R, CX, CY, true, false>, grid, block, s, A, bz);
  else launch_hess(k_hessian_col<R, CX, CY, false, false>, grid, block, s, A, bz);
  return hipGetLastError();
}

// Hessian shapes. Bricks: 0 = 8x8x4 (448 threads), 1 = 8x8x8 (768),
// 2 = 16x8x4 (768), 3 = 16x4x4 (448), 4 = 8x4x4 (256: two blocks share a CU
// at the FP64 kernel's register count, so one block's loads overlap the
// other's arithmetic, for 1.76 instead of 1.58 elements per owned node).
// Columns (kBrickOnly and up): kColShapes, where nx and ny are multiples of
// the column.
template <typename R>
hipError_t launch_hessian_brick(const HessArgs<R>& A, hipStream_t s, int* nblocks) {
  if (!A.v || !A.f || !A.a || !A.sw || !A.emask || !A.E || !A.red.partials ||
      (A.tens && !A.sn) || (A.U && !A.red_tail.partials))
    return hipErrorInvalidValue;
  if (A.brick_shape >= kBrickOnly) {
    if (A.brick_shape >= kHessianShapes) return hipErrorInvalidValue;
    const ColShape c = kColShapes[A.brick_shape - kBrickOnly];
    if (c.cx == 16 && c.cy == 16) return launch_hessian_col<R, 16, 16>(A, c.bz, s, nblocks);
    if (c.cx == 16 && c.cy == 8) return launch_hessian_col<R, 16, 8>(A, c.bz, s, nblocks);
    return launch_hessian_col<R, 8, 8>(A, c.bz, s, nblocks);
  }
  switch (A.brick_shape) {
    case 1: return launch_hessian_shape<R, 8, 8, 8>(A, s, nblocks);
    case 2: return launch_hessian_shape<R, 16, 8, 4>(A, s, nblocks);
    case 3: return launch_hessian_shape<R, 16, 4, 4>(A, s, nblocks);
    case 4: return launch_hessian_shape<R, 8, 4, 4>(A, s, nblocks);
    default: return launch_hessian_shape<R, 8, 8, 4>(A, s, nblocks);
  }
}

template <int MODE, int NV>
hipError_t launch_gather(const ElemArgs& A, hipStream_t s, int* nblocks) {
  const int nb = (int)((A.g.N + kBlock - 1) / kBlock);
  *nblocks = nb;
  if (A.g.element == HFE_Q1)
    hipLaunchKernelGGL((k_gather<HFE_Q1, MODE, NV>), dim3(nb), dim3(kBlock), 0, s, A);
  else
    hipLaunchKernelGGL((k_gather<HFE_P1_PAIR, MODE, NV>), dim3(nb), dim3(kBlock), 0, s, A);
  return hipGetLastError();
}

}  // namespace

void arm_kernel_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}

hipError_t launch_residual(const ElemArgs& A, hipStream_t s, int* nblocks) {
  if (A.g.element != HFE_Q1) return launch_gather<MODE_RESIDUAL, RES_NV>(A, s, nblocks);
  if (!A.u || !A.f || !A.a_out || !A.soft_out || !A.emask_out || !A.sw_out || !A.khist ||
      !A.phase || !A.E || !A.red.partials || (A.tens && !A.sn_out))
    return hipErrorInvalidValue;
  return launch_brick<MODE_RESIDUAL, RES_NV>(A, s, nblocks);
}
hipError_t launch_trial(const ElemArgs& A, hipStream_t s, int* nblocks) {
  if (A.g.element != HFE_Q1) return launch_gather<MODE_TRIAL, TRI_NV>(A, s, nblocks);
  if (!A.u || !A.v || !A.a || !A.soft || !A.sw || !A.khist || !A.phase || !A.E ||
      !A.red.partials || (A.tens && !A.sn))
    return hipErrorInvalidValue;
  constexpr int BX = 8, BY = 8, BZ = 4;
  const int nb = ((A.g.nx + BX - 1) / BX) * ((A.g.ny + BY - 1) / BY) * ((A.g.nz + BZ - 1) / BZ);
  *nblocks = nb;
  const bool full = A.g.nx % BX == 0 && A.g.ny % BY == 0 && A.g.nz % BZ == 0;
  const dim3 grid(nb), block(BX * BY * BZ);
  if (A.tens) {
    if (full) hipLaunchKernelGGL((k_trial<BX, BY, BZ, true, true>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_trial<BX, BY, BZ, false, true>), grid, block, 0, s, A);
  } else {
    if (full) hipLaunchKernelGGL((k_trial<BX, BY, BZ, true, false>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((k_trial<BX, BY, BZ, false, false>), grid, block, 0, s, A);
  }
  return hipGetLastError();
}
bool hessian_shape_valid(const Grid& g, int shape) {
  if (shape < 0 || shape >= kHessianShapes) return false;
  if (shape < kBrickOnly) return true;
  const ColShape c = kColShapes[shape - kBrickOnly];
  return g.element == HFE_Q1 && g.nx % c.cx == 0 && g.ny % c.cy == 0;
}
hipError_t launch_hessian(const ElemArgs& A, hipStream_t s, int* nblocks) {
  if (A.g.element != HFE_Q1) return launch_gather<MODE_HESSIAN, HES_NV>(A, s, nblocks);
  HessArgs<double> H;
  H.g = A.g;
  H.mat = A.mat;
  H.E = A.E;
  H.emask = A.emask;
  H.U = A.U;
  H.red_tail = A.red_tail;
  H.sw = A.sw;
  H.sn = A.sn;
  H.tens = A.tens;
  H.a = A.a;
  H.v = A.v;
  H.f = A.f;
  H.red = A.red;
  H.cg = A.cg;
  H.brick_shape = A.brick_shape;
  return launch_hessian_brick<double>(H, s, nblocks);
}
hipError_t launch_hessian_f32(const HessArgs<float>& A, hipStream_t s, int* nblocks) {
  if (A.g.element != HFE_Q1) return hipErrorInvalidValue;
  return launch_hessian_brick<float>(A, s, nblocks);
}
hipError_t launch_commit(const ElemArgs& A, hipStream_t s) {
  const int nb = (int)((A.g.N + kBlock - 1) / kBlock);
  if (A.g.element == HFE_Q1)
    hipLaunchKernelGGL(k_commit<HFE_Q1>, dim3(nb), dim3(kBlock), 0, s, A);
  else
    hipLaunchKernelGGL(k_commit<HFE_P1_PAIR>, dim3(nb), dim3(kBlock), 0, s, A);
  return hipGetLastError();
}
hipError_t launch_init_history(const ElemArgs& A, hipStream_t s) {
  const int nb = (int)((A.g.N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_init_history, dim3(nb), dim3(kBlock), 0, s, A);
  return hipGetLastError();
}
hipError_t launch_fields(const ElemArgs& A, double* out_h, double* out_s, double* out_d,
                         double* out_k, hipStream_t s) {
  const int nb = (int)((A.g.N + kBlock - 1) / kBlock);
  if (A.g.element == HFE_Q1)
    hipLaunchKernelGGL(k_fields<HFE_Q1>, dim3(nb), dim3(kBlock), 0, s, A, out_h, out_s, out_d,
                       out_k);
  else
    hipLaunchKernelGGL(k_fields<HFE_P1_PAIR>, dim3(nb), dim3(kBlock), 0, s, A, out_h, out_s,
                       out_d, out_k);
  return hipGetLastError();
}

}  // namespace hfe
