/*
 * hfe.h - C ABI of the MI355X FE-projection homogenization solver.
 *
 * The library solves the periodic cell problem of small-strain homogenization
 * (Sec. 2: strain split into a prescribed macroscopic strain E and a periodic
 * fluctuation, eq. strain_decomp; equilibrium and compatibility, eq.
 * equilibrium / eq. compatibility) with the FE-projection scheme of Sec. 2.1
 * (projector built from the discrete derivative of linear finite elements,
 * eq. proj_operator) and the trust-region Newton solver of Sec. 2.2 with the
 * first-order approximate incremental energy (eq. incr_energy_func, eq.
 * rho_bar; Algorithm 2) around Steihaug's truncated CG with restart
 * (Algorithm 1, eq. 1).
 *
 * Conventions shared by every entry point:
 *   - Grid: nx x ny (x nz) unit voxels, periodic. Node and element indices
 *     are n = x + nx*(y + ny*z) (x fastest). Nodes sit at voxel corners, so
 *     there are as many nodes as voxels.
 *   - Elements: HFE_Q1 = trilinear hexahedron, 2x2x2 Gauss points
 *     (1/2 -+ 1/(2 sqrt 3)), point index q = qx + 2 qy + 4 qz (3D only);
 *     HFE_P1_PAIR = two linear triangles per pixel, one point each,
 *     T1 = corners (0,0),(1,0),(0,1), T2 = (1,1),(0,1),(1,0) (2D only,
 *     plane strain).
 *   - Tensors crossing the ABI are 3x3 row-major doubles (9 values).
 *   - Host pointers are owned by the caller and only read or written during
 *     the call. Device pointers (the workspace, and the device arguments of
 *     the operator entry points) are borrowed: the caller keeps them alive
 *     for as long as the context, or the call, uses them.
 *   - Every call returns an hfe_status; nothing throws across the ABI. A
 *     negative status is an error and leaves the context as it was (its
 *     text is available from hfe_last_error). Calls out of the documented
 *     order return HFE_ESTATE.
 *   - All device work is enqueued on the stream given at creation; calls
 *     that return host data synchronise with that stream before returning.
 */
#ifndef HFE_H
#define HFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hfe_ctx hfe_ctx;

typedef enum {
  HFE_OK = 0,
  HFE_EINVAL = -1,    /* invalid argument (grid, phase id, material, size) */
  HFE_ENOMEM = -2,    /* workspace too small */
  HFE_EDEVICE = -3,   /* a HIP call failed */
  HFE_ENUMERIC = -4,  /* non-finite values in the state */
  HFE_ESTATE = -5     /* call out of order */
} hfe_status;

/* Positive outcome codes of hfe_solve_increment (stored in report.status). */
enum { HFE_CONVERGED = 0, HFE_NOT_CONVERGED = 1 };

enum { HFE_P1_PAIR = 1, HFE_Q1 = 2 };
enum { HFE_ELASTIC = 0, HFE_DAMAGE_ENERGY_NORM = 1, HFE_DAMAGE_TENSILE = 2 };
enum { HFE_MAX_PHASES = 8 };
/* Arithmetic of the CG inside hfe_solve_increment (hfe_solver_params.precision). */
enum { HFE_FP64 = 0, HFE_MIXED = 1 };

/* Fields readable through hfe_get_field (sizes per entry). */
enum {
  HFE_FIELD_U = 0,       /* nodal fluctuation displacement, [dim][N]            */
  HFE_FIELD_GRAD = 1,    /* full gradient H = E + D u at points, [N][nq][dim][dim] */
  HFE_FIELD_STRESS = 2,  /* stress at points, [N][nq][dim][dim]                  */
  HFE_FIELD_DAMAGE = 3,  /* committed damage d(kappa_hist), [N][nq]              */
  HFE_FIELD_KAPPA = 4,   /* committed history kappa_hist, [N][nq]                */
  HFE_FIELD_SOFTENING = 5 /* 1 where the tangent of the evaluated state carries the
                           * softening term (loading with 0 < d < 1), else 0, [N][nq] */
};

/* Exit flags of the truncated CG (Algorithm 1), as logged per Newton step.
 * HFE_CG_STALL: the optional stall exit (hfe_solver_params.cg_stall). */
enum { HFE_CG_INTERIOR = 1, HFE_CG_BOUNDARY = 2, HFE_CG_NEGCURV = 3, HFE_CG_MAXITER = 4,
       HFE_CG_STALL = 5 };

typedef struct {
  int dim;       /* 2 or 3 */
  int n[3];      /* nx, ny, nz (nz = 1 in 2D); every n even-or-odd as below   */
  int element;   /* HFE_P1_PAIR (dim 2) or HFE_Q1 (dim 3)                       */
} hfe_grid;
/* Supported sizes: nx even; nx/2, ny and nz each in
 * {1,2,3,4,6,8,12,16,24,32,48,64,96,128}; (nx/2+1)*ny*16 bytes <= 160 KiB
 * (one spectral plane fits in LDS); nz = 1 exactly when dim = 2. */

typedef struct {
  int kind;        /* HFE_ELASTIC, HFE_DAMAGE_ENERGY_NORM or HFE_DAMAGE_TENSILE */
  double E, nu;    /* Young's modulus > 0, Poisson ratio in (-1, 1/2)          */
  double kappa0;   /* damage threshold of the equivalent strain (damage only) */
  double kappaf;   /* equivalent strain at full damage, > kappa0             */
} hfe_material;
/* Damage law (per point): kappa_t = sqrt(eps : C : eps / E),
 * loading iff kappa_t > kappa_hist, d = clamp(kf/k (k - k0)/(kf - k0), 0, 1)
 * with k = kappa_t when loading else kappa_hist, sigma = (1 - d) C : eps.
 * Consistent tangent B = (1-d) C - c' (C:eps) (x) (C:eps),
 * c' = d'(kappa_t)/(E kappa_t) while loading with 0 < d < 1, else 0.
 * HFE_DAMAGE_TENSILE, the tensile-masking law of Appendix A (eqs.
 * strain_measure, stress_contributions_maksing_matrices, Mask_matrices_t,
 * our_model_damage_variable): the same d(kappa) and sigma, with
 * kappa_t = |eps_t|, eps_t = sum_i max(e_i, 0) q_i (x) q_i over the
 * eigenpairs of eps; the appendix's relative softening slope alpha is
 * kappaf = kappa0 (1 + alpha) / alpha. Tangent B = (1-d) C - c' (C:eps) (x) eps_t,
 * c' = d'(kappa_t)/kappa_t, which is not symmetric: the CG of Algorithm 1
 * runs on it unchanged (3D Q1: the state keeps a second factor per softening
 * point). */

typedef struct {
  double eta_eq;   /* equilibrium tolerance on ||G sigma|| / ||sigma||        */
  double eta_nr;   /* Newton tolerance on ||delta eps|| / ||eps||             */
  double eta_cg;   /* CG tolerance relative to the initial model gradient    */
  double eta_up;   /* step accepted iff rho_bar > eta_up                       */
  double R0;       /* initial trust radius (<= 0: 10 sqrt(N_qp) ||dE_1||_F)   */
  double Rmax;     /* maximum trust radius (<= 0: 1000 sqrt(N_qp) ||dE_1||_F)  */
  int i_nr_max;    /* maximum Newton iterations per load step                */
  int j_cg_max;    /* maximum CG iterations per Newton step                  */
  int precision;   /* HFE_FP64: everything in FP64. HFE_MIXED (3D only): the
                    * Hessian, the FFT / Green's operator and the CG vectors
                    * inside Algorithm 1 in FP32 (CG inner products summed in
                    * FP64); the residual D^T sigma, the trial evaluation and
                    * the energy terms of the ratio rho_bar, the history and
                    * the state stay FP64, so each Newton step starts from an
                    * FP64 residual and the tolerances keep their meaning.   */
  double restart;  /* constant c of the reset test of Algorithm 1 (eq. 1):
                    * after a CG step, if |<r_{j+1}, r_j>| > c <r_{j+1}, r_{j+1}>
                    * the residual is recomputed as A z_{j+1} + g and the
                    * next direction is -r_{j+1} (beta = 0). The paper's value
                    * is 0.2 (the default). Any c < 0 restarts after every
                    * step (steepest descent with exact line search); +inf
                    * never restarts. HFE_EINVAL if NaN. */
  int cg_stall;    /* stall exit of the CG, an addition to Algorithm 1 (0, the
                    * default, switches it off): the CG returns its current
                    * iterate as an interior step (flag HFE_CG_STALL) once
                    * cg_stall iterations have passed without the residual
                    * norm falling to half of its last reference value (the
                    * reference starts at ||r_0|| and is replaced by every
                    * residual at or below half of it). At damaged states the
                    * residual of Algorithm 1 can plateau far above eta_cg
                    * for thousands of iterations (in FP64 and FP32 alike);
                    * this ends such solves. HFE_EINVAL if negative. */
} hfe_solver_params;

typedef struct {
  int status;          /* HFE_CONVERGED or HFE_NOT_CONVERGED                       */
  int newton_iters, rejected, cg_iters, restarts, boundary_exits, negcurv_exits;
  int matvecs;         /* projected-Hessian applications (CG + restarts)          */
  int stall_exits;     /* Newton steps whose CG ended at the stall exit           */
  double r_eq, r_nr, R, rho_last;
  double time_ms;      /* wall time of the call                                    */
} hfe_solve_report;

/* Per-Newton-step record (lockstep logs against the oracle). p_norm is the
 * step's strain-space norm ||p|| summed directly over the points by the trial
 * pass (the CG tracks it by recurrences; on a boundary or negative-curvature
 * exit it equals R_before). */
typedef struct {
  int flag, cg_iters, restarts, accepted;
  double dm, dW, rho, R_before, p_norm;
} hfe_newton_record;

/* Bytes of device workspace needed for a grid; 0 if the grid is unsupported. */
size_t hfe_workspace_bytes(const hfe_grid* grid);

/* Create a context on the current HIP device. `workspace` is a device buffer of
 * at least hfe_workspace_bytes(grid) bytes, 256-byte aligned; `hip_stream` is a
 * hipStream_t (NULL = default stream). Both are borrowed. On success *out
 * holds the new context. Sec. 2 (cell problem), Algorithm 2 (initialisation). */
hfe_status hfe_create(const hfe_grid* grid, void* workspace, size_t ws_bytes,
                      void* hip_stream, hfe_ctx** out);
hfe_status hfe_destroy(hfe_ctx* ctx);

/* Phase id per voxel (host array of N bytes, x fastest), ids < n_phases <=
 * HFE_MAX_PHASES. Resets the state (u = 0, E = 0, history = kappa0). */
hfe_status hfe_set_microstructure(hfe_ctx* ctx, const uint8_t* phase, int n_phases);

/* Material of one phase (Sec. 3, Appendix A; call once per phase before the
 * first load step). The struct is copied. Errors: HFE_EINVAL for a null
 * material, a phase outside [0, n_phases), an unknown kind, E <= 0, nu outside
 * (-1, 1/2), or a damage kind without 0 < kappa0 < kappaf; HFE_ESTATE before
 * the microstructure is set or once loading has started. */
hfe_status hfe_set_material(hfe_ctx* ctx, int phase, const hfe_material* mat);

/* Eigenstrain of a phase (host, 3x3 row-major; its symmetric part is used, in
 * 2D only the in-plane block). Algorithm 2 adds it to the strain of every
 * point of the phase before each evaluation of the law (the eps_eval lines),
 * trial evaluations included. It may change between load steps (a growing
 * eigenstrain, as for expanding inclusions): the next hfe_apply_load_step
 * (with dE = 0 for a load by eigenstrain alone) evaluates the state with
 * it. When the first increment is zero, the default trust radii take the
 * scale of the largest phase eigenstrain instead of ||dE_1||. */
hfe_status hfe_set_eigenstrain(hfe_ctx* ctx, int phase, const double eig[9]);

/* Mean-stress control (Sec. 3.3 holds its cell's mean stress at zero, free
 * expansion, through a modified projector). Bit v of free_mask (Voigt order
 * v = 0..5: xx, yy, zz, yz, xz, xy) makes that macroscopic strain component
 * an unknown whose mean stress must vanish; the others stay prescribed.
 * The projector becomes G + M, M the projection onto uniform fields in the
 * free components (a free shear pair (i, j) as (e_i e_j + e_j e_i) / sqrt 2),
 * an orthogonal projector that G annihilates: Algorithm 1 runs on fields
 * D u + sum_m e_m B_m, the trust-region ratio is unchanged, and an accepted
 * step moves E by its uniform part. The residual r_eq measures
 * ||(G + M) sigma|| / ||sigma||. 0 restores strain control. Takes effect at
 * the next solve (hfe_get_state returns E with the solved components).
 * 3D and FP64 only: HFE_EINVAL for a mask outside 0..63, a non-zero mask on a
 * 2D grid, and later for HFE_MIXED solves or the L-BFGS increment while a
 * component is free. */
hfe_status hfe_set_mean_stress_control(hfe_ctx* ctx, int free_mask);

/* Algorithm 2, start of a load increment: E <- E + dE (dE a host 3x3,
 * symmetric; in 2D only the in-plane block is used), keep the fluctuation of
 * the previous step as initial guess, evaluate sigma and B with the history
 * frozen, the right-hand side -G sigma and its relative norm. Errors:
 * HFE_EINVAL for a NULL or non-finite dE; HFE_ESTATE before the
 * microstructure and every material are set; HFE_ENUMERIC if the stress or
 * the residual at the new E is not finite (E and the evaluated state are
 * then those before the call). */
hfe_status hfe_apply_load_step(hfe_ctx* ctx, const double dE[9]);

/* Algorithm 2 (Newton / trust-region loop with Algorithm 1 inside) for the
 * current increment. Commits the damage history iff it converges. `params`
 * may be NULL (defaults: eta_eq = eta_nr = 1e-8, eta_cg = 1e-6, eta_up = 0.15,
 * i_nr_max = 50, j_cg_max = 2000, radii from the first increment, restart
 * = 0.2, cg_stall = 0). `out` may be NULL. */
hfe_status hfe_solve_increment(hfe_ctx* ctx, const hfe_solver_params* params,
                               hfe_solve_report* out);

/* Quasi-Newton alternative to hfe_solve_increment for the same increment:
 * L-BFGS on the approximate incremental energy. Sec. 2.2 notes that the
 * first-order energy increment of eq. incr_energy_func makes quasi-Newton
 * solvers usable; the method below is this library's reading of that remark:
 *   direction p = -H_k g (g = G sigma) by the two-loop recursion over the
 *   last m pairs (s, y), H_0 = gamma I, gamma = s.y / y.y of the newest pair,
 *   before any pair 1 / max over phases of (lambda + 2 mu); a direction with
 *   sigma:p >= 0 is replaced by -gamma g and the pairs dropped;
 *   step: alpha = 1, halved up to max_backtracks times, until
 *   DeltaW_bar(alpha p) = (sigma + sigma(u + alpha p)) : alpha p / 2
 *   <= c1 alpha sigma:p (history frozen);
 *   a pair is kept iff s.y > 1e-12 |s| |y|;
 *   convergence and commit of the history as Algorithm 2 (r_eq <= eta_eq, or
 *   r_NR <= eta_nr after an accepted step).
 * Inner products are those of strain space (s.y = du . dg0 with g0 = D^T sigma).
 * FP64. `workspace`: device buffer of hfe_lbfgs_workspace_bytes(grid, m)
 * bytes (borrowed; it holds the pairs and work vectors). HFE_EINVAL for
 * m < 1 or m > HFE_LBFGS_MAX_M or a small workspace; `params` may be NULL
 * (defaults below), `out` may be NULL. */
#define HFE_LBFGS_MAX_M 32
typedef struct {
  double eta_eq;       /* 1e-8 */
  double eta_nr;       /* 1e-8 */
  int max_iters;       /* 500 quasi-Newton iterations */
  int m;               /* 5 pairs */
  double c1;           /* 1e-4 */
  int max_backtracks;  /* 30 */
} hfe_lbfgs_params;
typedef struct {
  int status;          /* HFE_CONVERGED or HFE_NOT_CONVERGED                      */
  int iters;           /* quasi-Newton iterations (directions formed)            */
  int trials;          /* energy evaluations of the line search                  */
  int pairs_skipped;   /* pairs failing the curvature test                       */
  int resets;          /* non-descent directions replaced by -gamma g            */
  double r_eq, r_nr, time_ms;
} hfe_lbfgs_report;
size_t hfe_lbfgs_workspace_bytes(const hfe_grid* grid, int m);
hfe_status hfe_solve_increment_lbfgs(hfe_ctx* ctx, const hfe_lbfgs_params* params,
                                     void* workspace, size_t ws_bytes, hfe_lbfgs_report* out);

/* Mean stress over all quadrature points (3x3; in 2D includes sigma_zz of
 * plane strain) at the last evaluated state. */
hfe_status hfe_homogenized_stress(const hfe_ctx* ctx, double out[9]);

/* Relative equilibrium residual of the last evaluated state, Algorithm 2's
 * r_eq = ||G sigma|| / ||sigma|| (G_M under mean-stress control; 0 when
 * sigma = 0), as the convergence test uses it. Lets a caller compare initial
 * guesses (hfe_set_displacement) before solving. *out (host) receives it;
 * HFE_ESTATE before a state is evaluated. */
hfe_status hfe_residual(const hfe_ctx* ctx, double* out);

/* Copy a field (HFE_FIELD_*) to host memory; n = number of doubles in out. */
hfe_status hfe_get_field(const hfe_ctx* ctx, int which, double* host_out, size_t n);

/* Per-Newton-step records of the last solve; *count receives the number
 * written (at most max). */
hfe_status hfe_get_newton_log(const hfe_ctx* ctx, hfe_newton_record* out, int max, int* count);

/* Checkpoint and restart: the solver state is the nodal fluctuation u
 * ([dim][N]), the committed history kappa_hist ([N][nq], point order as the
 * fields), the macroscopic strain E (3x3) and the trust radius with its cap
 * (radius[0] = R, radius[1] = Rmax; Algorithm 2 carries R from one load step
 * to the next). All host arrays. hfe_set_state re-evaluates the state at the
 * restored point without committing; after it a solve continues exactly as
 * the run the state was taken from (up to rounding). */
hfe_status hfe_get_state(const hfe_ctx* ctx, double* u, double* kappa_hist, double E[9],
                         double radius[2]);
hfe_status hfe_set_state(hfe_ctx* ctx, const double* u, const double* kappa_hist,
                         const double E[9], const double radius[2]);

/* Trace of the truncated CG of the last solve, two doubles per iteration:
 * {d.Ad, ||r_{j+1}|| / ||r_0||} (the second is NaN on a boundary or
 * negative-curvature exit). Used to certify that a decision that differs
 * from the oracle's sits on a stopping threshold. */
hfe_status hfe_get_cg_trace(const hfe_ctx* ctx, double* out, int max, int* count);

/* Replace the nodal fluctuation u (host, [dim][N]) and re-evaluate the state
 * at the current E without committing (operator tests and restarts).
 * HFE_EINVAL (nothing changed) if an entry is not finite. */
hfe_status hfe_set_displacement(hfe_ctx* ctx, const double* host_u);

/* Projected Hessian in displacement coordinates at the current state
 * (eq. project_stress_linear): out = L^+ K d with K = D^T B D and
 * L = D^T D (the FE Green's operator of eq. proj_operator), so that
 * D out = G : B : (D d). `dev_in`, `dev_out` are device arrays [dim][N]
 * (distinct). dots (host, may be NULL) receives {d.Kd, sum |D d|^2}. */
hfe_status hfe_apply_projected_hessian(hfe_ctx* ctx, const double* dev_in,
                                       double* dev_out, double dots[2]);

/* The projected Hessian of hfe_apply_projected_hessian in the FP32 arithmetic
 * of the HFE_MIXED CG (3D only): the tangent scalars 1-d rounded to FP32
 * (the rank-one softening factors are read in FP64 and rounded on use), FP32
 * Hessian and FFT, dots summed in FP64. `dev_in`, `dev_out` are
 * distinct device float arrays [dim][N]. HFE_EINVAL in 2D. */
hfe_status hfe_apply_projected_hessian_f32(hfe_ctx* ctx, const float* dev_in, float* dev_out,
                                           double dots[2]);

/* Solve one load increment (as hfe_solve_increment) on each of n distinct
 * contexts at once: several load cases or cells on one GPU, one host thread
 * per context. The work of contexts created on distinct streams overlaps on
 * the device, which fills the chip where one cell cannot. `params` (may be
 * NULL) applies to all; reports[i] (host, n entries) receives context i's
 * report. Returns the first non-OK status (every solve still runs). */
hfe_status hfe_solve_batch(hfe_ctx* const* ctxs, int n, const hfe_solver_params* params,
                           hfe_solve_report* reports);

/* Effective stiffness of a cell (the six columns of C-bar, Voigt order xx,
 * yy, zz, yz, xz, xy with engineering shears) from six contexts of the same
 * grid, microstructure and materials, each in the state to linearise about
 * (fresh, or restarted with hfe_set_state, e.g. u = 0, E = 0 and a damaged
 * history: loads below the history unload, which gives the secant stiffness
 * of the damaged cell). Context J gets the increment `strain` times the J-th
 * unit strain (shears: E_ij = E_ji = strain / 2) and the six increments are
 * solved as one batch (hfe_solve_batch); column J is the change of the
 * homogenized stress divided by `strain`. 3D only. C (host, 36 doubles,
 * row-major) receives C-bar; reports (host, 6, may be NULL) the solves. The
 * contexts keep the solved increments. */
hfe_status hfe_effective_stiffness(hfe_ctx* const* ctxs, double strain,
                                   const hfe_solver_params* params, double C[36],
                                   hfe_solve_report* reports);

/* Launch shapes of the hot kernels, per context. FP64 fields serve the FP64
 * path, *32 fields the FP32 kernels of the HFE_MIXED CG. */
typedef struct {
  int plane_threads;    /* threads of an x-y plane FFT block (64..1024, multiple of 64) */
  int pencil_cols;      /* z columns per pencil block (1..64)                       */
  int pencil_threads;   /* threads of a pencil block (64..256, multiple of 64)      */
  int brick_shape;      /* Q1 Hessian launch shape. Bricks of nodes (any grid): 0 = 8x8x4,
                           1 = 8x8x8, 2 = 16x8x4, 3 = 16x4x4, 4 = 8x4x4. Columns of
                           CX x CY nodes marching over BZ node layers (nx a multiple
                           of CX, ny of CY): 5 = 16x16x16, 6 = 16x16x8, 7 = 16x8x16,
                           8 = 16x8x8, 9 = 8x8x8, 10 = 8x8x16, 11 = 16x8x32,
                           12 = 16x16x32. Every shape gives the same K d bits,
                           and the same sums (formed per canonical tile). */
  int plane_threads32, pencil_cols32, pencil_threads32, brick_shape32;
} hfe_tuning;

/* Current launch shapes (defaults at creation). */
hfe_status hfe_get_tuning(const hfe_ctx* ctx, hfe_tuning* out);
/* Set launch shapes; HFE_EINVAL (context unchanged) if one does not fit the
 * grid: a plane block must stage (nx/2+1) ny values at 15 per thread, a
 * pencil block pencil_cols * nz values at 15 per thread in 64 KiB of LDS, a
 * Hessian column must divide nx and ny. */
hfe_status hfe_set_tuning(hfe_ctx* ctx, const hfe_tuning* in);
/* Autotuner: times every valid plane / pencil shape and, once a load step
 * has been applied, every valid Hessian shape at the current state (FP64 and
 * FP32); keeps the fastest and returns them in `out` (may be NULL). With a 3D
 * state, the FP64 plane / pencil shapes are timed on CG iterations of a probe
 * solve started at that state (the fused passes the solver runs), otherwise
 * (2D, no state, or a probe that stops on negative curvature) on the Green's
 * operator; the FP32 ones on the FP32 Green's operator. The probe overwrites
 * the CG work vectors, which every solve initialises itself. Results do not
 * depend on the shapes (every value and every sum is formed in the same
 * order), only the time does. */
hfe_status hfe_autotune(hfe_ctx* ctx, hfe_tuning* out);

/* The two halves of the matvec, for operator tests: out = K d (device
 * arrays [dim][N]), and out = L^+ f (zero mean; the k = 0 mode removed). */
hfe_status hfe_apply_stiffness(hfe_ctx* ctx, const double* dev_in, double* dev_out);
hfe_status hfe_apply_green(hfe_ctx* ctx, const double* dev_in, double* dev_out);

/* 3D real-to-complex FFT of dim fields (device in [dim][N]) to the half
 * spectrum, device out [dim][nz][ny][nx/2+1] complex (interleaved doubles),
 * unscaled, exponent sign -1; and its inverse (unscaled, sign +1). The
 * transforms of eq. conv_to_fourier. */
hfe_status hfe_fft_forward(hfe_ctx* ctx, const double* dev_in, double* dev_out_spec);
hfe_status hfe_fft_inverse(hfe_ctx* ctx, const double* dev_in_spec, double* dev_out);

/* Kernel timing: when on, every launch is bracketed with HIP events on the
 * context's stream. hfe_kernel_stats writes, for up to max kernels, the name
 * pointer, launch count and total milliseconds since the last reset. */
hfe_status hfe_set_profiling(hfe_ctx* ctx, int on);

/* Softening points of a Q1 state: points where the damage law of Appendix A
 * is loading with 0 < d < 1, so that its consistent tangent carries the
 * rank-one term c' (C:eps) (x) (C:eps) besides (1-d) C. *current gets the
 * count of the evaluated state; *mean_per_hessian the mean of that count over
 * the Hessian launches timed since the last hfe_set_profiling (0 if none).
 * Either pointer may be null. Host pointers; 0 for P1 pairs. */
hfe_status hfe_soft_points(hfe_ctx* ctx, double* current, double* mean_per_hessian);
hfe_status hfe_kernel_stats(hfe_ctx* ctx, const char** names, int* counts, double* total_ms,
                            int max, int* n_kernels);

/* Text of the last error on this context (never NULL). */
const char* hfe_last_error(const hfe_ctx* ctx);

/* ---- learned warm start (BF16 3D convolutions and their training) ----------
 *
 * A small convolutional network on the periodic voxel grid predicts the
 * displacement increment of a load step from the cell's state; the solve
 * then starts from it (the initial guess of Algorithm 2's load loop) and
 * refines it to the same tolerance. These entry points are its building
 * blocks. Fields are device arrays, channels-major [C][nz][ny][nx] (x
 * fastest), n = {nx, ny, nz}; filter banks [cout][cin][27] with tap
 * (dz+1)*9 + (dy+1)*3 + (dx+1); the grid is periodic. BF16 values are
 * uint16_t (the upper half of an IEEE binary32, round to nearest even).
 * Channel counts: 1 to 512. Layers whose counts are both among 1, 2, 3, 4,
 * 6, 8, 16 and 32 hold their filter bank in LDS; the others (the 64-channel
 * levels of a widening network) read it from global memory in tiles of 16
 * channels. `stream` is a hipStream_t (NULL:
 * the default stream); the calls are asynchronous on it. HFE_EINVAL for bad
 * arguments, HFE_EDEVICE if a launch fails. */

/* out = conv(in; w) + bias (bias may be NULL), ReLU if relu != 0; FP32 out,
 * and its BF16 copy in out_bf16 when not NULL. Products accumulate in FP32. */
hfe_status hfe_nn_conv3d(const uint16_t* in, int cin, const uint16_t* w, const float* bias,
                         int cout, const int n[3], int relu, float* out, uint16_t* out_bf16,
                         void* stream);
/* gin = the adjoint convolution of gout (masked by act > 0 when act, the
 * layer's ReLU output, is not NULL): the gradient with respect to the input. */
hfe_status hfe_nn_conv3d_backward_data(const float* gout, int cout, const float* act,
                                       const uint16_t* w, int cin, const int n[3], float* gin,
                                       void* stream);
/* Weight and bias gradients (gb may be NULL) of the layer, with the same
 * masking; sums over all voxels in FP64 in a fixed order. */
hfe_status hfe_nn_conv3d_backward_weights(const float* gout, int cout, const float* act,
                                          const uint16_t* in, int cin, const int n[3], float* gw,
                                          float* gb, void* stream);
/* Mean squared error over n values: grad = 2 (pred - target) / n, *loss
 * (device) = mean (pred - target)^2; partials: device scratch of
 * hfe_nn_mse_partials(n) doubles. */
size_t hfe_nn_mse_partials(long long n);
hfe_status hfe_nn_mse(const float* pred, const float* target, long long n, float* grad,
                      double* partials, double* loss, void* stream);
/* hfe_nn_mse for callers that cannot allocate device memory (code under HIP
 * graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the partial sums in a
 * library-owned array of 4096 doubles (32 KiB) per device, held until the
 * process ends; any n >= 1 fits (the loss kernel's grid never exceeds 4096
 * blocks). No allocation of any kind. The first call on a device resolves the
 * array's address (do not make that first call inside a graph capture).
 * Every call on a device shares the array: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 * Each call rewrites every row it reads. HFE_EINVAL for null pointers or
 * n < 1, HFE_EDEVICE if the address or a launch fails. */
hfe_status hfe_nn_mse_noalloc(const float* pred, const float* target, long long n, float* grad,
                              double* loss, void* stream);
/* One Adam step (step = 1, 2, ...) on FP32 master weights w with moments m,
 * v; writes the BF16 copy when w_bf16 is not NULL. */
hfe_status hfe_nn_adam(float* w, float* m, float* v, const float* g, long long n, float lr,
                       float beta1, float beta2, float eps, int step, uint16_t* w_bf16,
                       void* stream);
/* y = BF16(x). */
hfe_status hfe_nn_to_bf16(const float* x, long long n, uint16_t* y, void* stream);
/* Levels of the encoder-decoder. hfe_nn_pool2: the mean over 2x2x2 blocks of
 * c FP32 channels on the fine grid n (all even) into FP32 out and / or its
 * BF16 copy (either may be NULL, not both); hfe_nn_pool2_backward ADDS its
 * adjoint (gout / 8 to each child) to the fine gin. hfe_nn_upsample2: nearest
 * doubling of every axis of the coarse grid m into out / out_bf16;
 * hfe_nn_upsample2_backward writes its adjoint (the sum over the 8 children)
 * to the coarse gin. Device pointers, layout [c][z][y][x]. */
hfe_status hfe_nn_pool2(const float* in, int c, const int n[3], float* out, uint16_t* out_bf16,
                        void* stream);
hfe_status hfe_nn_pool2_backward(const float* gout, int c, const int n[3], float* gin,
                                 void* stream);
hfe_status hfe_nn_upsample2(const float* in, int c, const int m[3], float* out,
                            uint16_t* out_bf16, void* stream);
hfe_status hfe_nn_upsample2_backward(const float* gout, int c, const int m[3], float* gin,
                                     void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HFE_H */
