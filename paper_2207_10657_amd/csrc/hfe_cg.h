// Device-resident scalar state of the truncated CG (Algorithm 1) in
// displacement coordinates, and the decisions taken on it. The finish kernel
// that completes each reduction of a CG iteration applies the corresponding
// decision, so an iteration needs no host round trip: the host enqueues iterations in
// batches and reads the state once per batch. Once `done` is set, every later
// kernel of the batch returns at entry.
#pragma once

#include <hip/hip_runtime.h>

namespace hfe {

enum { CG_RUN = 0, CG_INTERIOR = 1, CG_BOUNDARY = 2, CG_NEGCURV = 3, CG_MAXITER = 4,
       CG_STALL = 5, CG_NUMERIC = 6 };

// Mean-stress control adds up to kMaxFree uniform unknowns to the CG vectors:
// free macroscopic strain components m with unit tensors B_m (e_i (x) e_i, or
// (e_i (x) e_j + e_j (x) e_i) / sqrt 2 for a shear pair), orthonormal under
// the point sum. Their coordinates ("tails") live in this state: a vector is
// (nodal part, tail), its strain-space field D x + sum_m x_m B_m, the inner
// products gain x.y-type tail terms (the cross terms vanish: the point sum
// of D x is zero), and the preconditioned tail is y_m = g_m / N_qp.
constexpr int kMaxFree = 6;

struct CgState {
  // scalars of the recurrences (strain-space inner products)
  double rr, rr0, rr_new;   // <r,r>, <r0,r0>, <r_{j+1},r_{j+1}>
  double zz, zz_new, zd;    // ||z||^2 (current / after the step), <z,d>
  double dd, kap, rd;       // ||d||^2, <d, G B d>, <r, d>
  double alpha, beta, tau;
  double R, eta_cg;
  double restart_c;         // constant of Powell's reset test (eq. 1)
  double rr_ref;            // stall exit: reference residual (squared)
  int j_ref;                // and the iteration that set it
  int stall;                // stall window in iterations (0: off)
  // mean-stress control: tails of the iterate, direction, gradient,
  // preconditioned gradient and K d, and the direction's uniform part
  // sum_m d_m B_m (row-major 3x3) read by the Hessian
  int ne;                   // free components (0: strain control, tails unused)
  int comp[kMaxFree];       // Voigt index (xx, yy, zz, yz, xz, xy) of each
  double nqp;               // points of the grid (the tails' metric)
  double ze[kMaxFree], de[kMaxFree], ge[kMaxFree], ye[kMaxFree], kde[kMaxFree];
  double dU[9];
  int iters;                // Hessian applications of this solve (CG iterations)
  int jmax;
  int done;                 // 1: stop; the remaining kernels of the batch are no-ops
  int flag;                 // CG_* exit flag (CG_RUN while running)
  int apply_tau;            // the exit step z + tau d is still to be formed
  int restart;              // Powell's test fired: the host recomputes the residual
  int ntrace;               // entries written to the trace
  int trace_cap;            // capacity of the trace (entries)
};

// Copy a CgState between global memory and LDS with the block's lanes, one
// 4-byte word each: copied by one lane, the whole struct (about 130 words)
// would pass through that lane's registers and push the kernel into spills.
// The caller's next barrier completes it.
__device__ __forceinline__ void copy_state_block(CgState* dst, const CgState* src) {
  static_assert(sizeof(CgState) % 4 == 0, "CgState is copied in 4-byte words");
  constexpr int kWords = (int)(sizeof(CgState) / 4);
  const unsigned* s = reinterpret_cast<const unsigned*>(src);
  unsigned* d = reinterpret_cast<unsigned*>(dst);
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) d[i] = s[i];
}

// Roots of ||z + t d||^2 = R^2 with ||z|| < R, without cancellation.
__device__ __forceinline__ void cg_roots(double zz, double zd, double dd, double R, double* tm,
                                         double* tp) {
  const double b = 2.0 * zd, c = zz - R * R;
  const double disc = sqrt(fmax(b * b - 4.0 * dd * c, 0.0));
  const double qq = -0.5 * (b + copysign(disc, b));
  const double t1 = qq / dd;
  const double t2 = qq != 0.0 ? c / qq : -t1;
  *tm = fmin(t1, t2);
  *tp = fmax(t1, t2);
}

// sum_m x_m B_m as a row-major 3x3 (Voigt comp: xx, yy, zz, yz, xz, xy)
__host__ __device__ inline void tail_tensor(const CgState* s, const double* x, double* U) {
  for (int k = 0; k < 9; ++k) U[k] = 0.0;
  const double r = 0.70710678118654752440;   // 1 / sqrt 2
  for (int m = 0; m < s->ne; ++m) {
    const int v = s->comp[m];
    if (v < 3) {
      U[4 * v] += x[m];
    } else {
      const int i = v == 3 ? 1 : 0, j = v == 5 ? 1 : 2;
      U[3 * i + j] += r * x[m];
      U[3 * j + i] += r * x[m];
    }
  }
}

// The pairing sum_q tau : B_m from the point sums of a symmetric tensor in
// Voigt order (xx, yy, zz, yz, xz, xy).
__host__ __device__ inline double tail_pair(int v, const double* voigt) {
  return v < 3 ? voigt[v] : 1.41421356237309504880 * voigt[v];
}

__device__ __forceinline__ void cg_trace(CgState* s, double* trace, double kap, double ratio) {
  if (trace && s->ntrace < s->trace_cap) {
    trace[2 * s->ntrace] = kap;
    trace[2 * s->ntrace + 1] = ratio;
  }
  s->ntrace += 1;
}

// After the Hessian application: curvature test, step length, boundary test.
// kvoigt (mean-stress control): the point sums of B : D d in Voigt order.
__device__ __forceinline__ void cg_decide_curvature(CgState* s, double* trace, double kap,
                                                    double dd, const double* kvoigt = nullptr) {
  if (s->done) return;
  if (s->ne > 0 && kvoigt) {
    for (int m = 0; m < s->ne; ++m) {
      s->kde[m] = tail_pair(s->comp[m], kvoigt);
      kap += s->de[m] * s->kde[m];
      dd += s->nqp * s->de[m] * s->de[m];
    }
  }
  s->kap = kap;
  s->dd = dd;
  s->iters += 1;
  if (!isfinite(kap) || !isfinite(dd)) {
    s->flag = CG_NUMERIC;
    s->done = 1;
    return;
  }
  if (kap <= 0.0) {
    // negative curvature: the root on the sphere with the smaller model value
    double tm, tp;
    cg_roots(s->zz, s->zd, dd, s->R, &tm, &tp);
    const double mm = tm * s->rd + 0.5 * tm * tm * kap;
    const double mp = tp * s->rd + 0.5 * tp * tp * kap;
    s->tau = mm < mp ? tm : tp;
    s->apply_tau = 1;
    for (int m = 0; m < s->ne; ++m) s->ze[m] += s->tau * s->de[m];
    s->flag = CG_NEGCURV;
    s->done = 1;
    cg_trace(s, trace, kap, NAN);
    return;
  }
  const double alpha = s->rr / kap;
  const double zz_new = s->zz + 2.0 * alpha * s->zd + alpha * alpha * dd;
  if (sqrt(zz_new) >= s->R) {
    double tm, tp;
    cg_roots(s->zz, s->zd, dd, s->R, &tm, &tp);
    s->tau = tp;
    s->apply_tau = 1;
    for (int m = 0; m < s->ne; ++m) s->ze[m] += s->tau * s->de[m];
    s->flag = CG_BOUNDARY;
    s->done = 1;
    cg_trace(s, trace, kap, NAN);
    return;
  }
  s->alpha = alpha;
  s->zz_new = zz_new;
  for (int m = 0; m < s->ne; ++m) {
    s->ze[m] += alpha * s->de[m];
    s->ge[m] += alpha * s->kde[m];
  }
}

// After the residual update: convergence, restart test, beta.
__device__ __forceinline__ void cg_decide_residual(CgState* s, double* trace, double rr_new,
                                                   double pw) {
  if (s->done) return;
  // tails: <r_{j+1}, r_{j+1}> gains |g_e|^2 / N_qp, the Powell numerator
  // y_e(old) . g_e(new); then y_e = g_e / N_qp
  for (int m = 0; m < s->ne; ++m) {
    pw += s->ye[m] * s->ge[m];
    s->ye[m] = s->ge[m] / s->nqp;
    rr_new += s->ge[m] * s->ye[m];
  }
  cg_trace(s, trace, s->kap, sqrt(fmax(rr_new, 0.0) / s->rr0));
  s->rr_new = rr_new;
  if (sqrt(fmax(rr_new, 0.0)) <= s->eta_cg * sqrt(s->rr0)) {
    s->flag = CG_INTERIOR;
    s->done = 1;
    return;
  }
  // stall exit: the residual norm has not halved within `stall` iterations
  if (rr_new <= 0.25 * s->rr_ref) {
    s->rr_ref = rr_new;
    s->j_ref = s->iters;
  } else if (s->stall > 0 && s->iters - s->j_ref >= s->stall) {
    s->flag = CG_STALL;
    s->done = 1;
    return;
  }
  if (fabs(pw) > s->restart_c * rr_new) {
    s->restart = 1;
    s->done = 1;
    return;
  }
  s->beta = rr_new / s->rr;
}

// The tail of the next direction, d_e = -y_e + beta d_e (beta as decided,
// 0 after a restart), and its uniform tensor for the next Hessian; taken
// where the nodal direction update is.
__device__ __forceinline__ void cg_tail_direction(CgState* s) {
  if (s->done || s->ne == 0) return;
  for (int m = 0; m < s->ne; ++m) s->de[m] = -s->ye[m] + s->beta * s->de[m];
  tail_tensor(s, s->de, s->dU);
}

// After the direction update: <z,d>, ||z||^2 and <r,r> for the next iteration.
__device__ __forceinline__ void cg_decide_direction(CgState* s, double gd, double zg) {
  if (s->done) return;
  for (int m = 0; m < s->ne; ++m) {
    gd += s->ge[m] * s->de[m];
    zg += s->ze[m] * s->ge[m];
  }
  s->zd = -zg + s->beta * (s->zd + s->alpha * s->dd);
  s->zz = s->zz_new;
  s->rr = s->rr_new;
  s->rd = gd;
  if (s->iters >= s->jmax) {
    s->flag = CG_MAXITER;
    s->done = 1;
  }
}

}  // namespace hfe
