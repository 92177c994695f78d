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
  int iters;                // Hessian applications of this solve (CG iterations)
  int jmax;
  int done;                 // 1: stop; the remaining kernels of the batch are no-ops
  int flag;                 // CG_* exit flag (CG_RUN while running)
  int apply_tau;            // the exit step z + tau d is still to be formed
  int restart;              // Powell's test fired: the host recomputes the residual
  int ntrace;               // entries written to the trace
  int trace_cap;            // capacity of the trace (entries)
};

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

__device__ __forceinline__ void cg_trace(CgState* s, double* trace, double kap, double ratio) {
  if (trace && s->ntrace < s->trace_cap) {
    trace[2 * s->ntrace] = kap;
    trace[2 * s->ntrace + 1] = ratio;
  }
  s->ntrace += 1;
}

// After the Hessian application: curvature test, step length, boundary test.
__device__ __forceinline__ void cg_decide_curvature(CgState* s, double* trace, double kap,
                                                    double dd) {
  if (s->done) return;
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
    s->flag = CG_BOUNDARY;
    s->done = 1;
    cg_trace(s, trace, kap, NAN);
    return;
  }
  s->alpha = alpha;
  s->zz_new = zz_new;
}

// After the residual update: convergence, restart test, beta.
__device__ __forceinline__ void cg_decide_residual(CgState* s, double* trace, double rr_new,
                                                   double pw) {
  if (s->done) return;
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

// After the direction update: <z,d>, ||z||^2 and <r,r> for the next iteration.
__device__ __forceinline__ void cg_decide_direction(CgState* s, double gd, double zg) {
  if (s->done) return;
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
