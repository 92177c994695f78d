// Internal declarations shared by the kernel translation units and the host
// driver. Not part of the public ABI (include/hfe.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/hfe.h"
#include "hfe_cg.h"

namespace hfe {

constexpr int kMaxPhases = HFE_MAX_PHASES;
constexpr int kBlock = 256;        // threads per block of the element / vector kernels
constexpr int kMaxPartials = 16;   // doubles per block in a partial-sum row

// Per-phase constants, passed by value to the kernels (no __constant__ state,
// so several contexts can live on one device).
struct MatTable {
  double lam[kMaxPhases], mu[kMaxPhases], E[kMaxPhases];
  double k0[kMaxPhases], kf[kMaxPhases];
  double eig[kMaxPhases][6];   // eigenstrain (xx, yy, zz, xy, xz, yz), added before the law
  int damage[kMaxPhases];
};

struct Grid {
  int nx, ny, nz;     // nz = 1 in 2D
  int dim, nq, na;    // displacement components, points and nodes per element
  int element;        // HFE_Q1 or HFE_P1_PAIR
  long long N;        // nodes = elements
};

// Canonical tiles of the node grid (3D): 8 x 4 x 4 nodes from the origin,
// cut by the grid at its far faces. The Hessian sums over nodes (and over the
// elements, each counted at its anchor node, the one with the lowest x, y,
// z) per tile in one fixed order and writes one partial row per tile:
// row = tx + ntx (ty + nty tz). Every Hessian launch shape covers whole
// tiles, so the rows, and every total formed from them, have the same bits
// under every shape.
constexpr int kTileX = 8, kTileY = 4, kTileZ = 4, kTileQ = kTileX * kTileY;
__host__ __device__ inline int tiles_x(const Grid& g) { return (g.nx + kTileX - 1) / kTileX; }
__host__ __device__ inline int tiles_y(const Grid& g) { return (g.ny + kTileY - 1) / kTileY; }
__host__ __device__ inline int tiles_z(const Grid& g) { return (g.nz + kTileZ - 1) / kTileZ; }
__host__ __device__ inline int tile_count(const Grid& g) {
  return tiles_x(g) * tiles_y(g) * tiles_z(g);
}
__host__ __device__ inline int tile_row(const Grid& g, int tx, int ty, int tz) {
  return tx + tiles_x(g) * (ty + tiles_y(g) * tz);
}

struct Macro {        // macroscopic strain E, full 3x3 row-major
  double e[9];
};

// Every reducing kernel writes one row of partial sums per block; a
// single-block finish kernel then adds the rows in a fixed order and acts on
// the totals (writes them out, or takes the CG decision). The kernel boundary
// between the two orders the memory accesses, so no device-wide fences are
// needed (on a part with one L2 per XCD such fences write the L2 back).
struct Reducer {
  double* partials;        // [blocks][nv]
};

// ---- element kernels (k_element.hip) -------------------------------------

// Partial-sum layouts written by the element kernels (one row per block).
// RES_NSOFT: number of softening points (c' != 0) of the state, Q1 only.
enum {
  RES_S0 = 0 /* 6 stress sums xx,yy,zz,xy,xz,yz */, RES_SS = 6, RES_HH = 7, RES_NSOFT = 8,
  RES_NV = 9
};
enum { TRI_SP = 0, TRI_PBP = 1, TRI_STP = 2, TRI_PP = 3, TRI_HH = 4, TRI_NV = 5 };
enum { HES_DKD = 0, HES_DD = 1, HES_NV = 2 };

struct ElemArgs {
  Grid g;
  MatTable mat;
  const double* E;       // macroscopic strain, 3x3 row-major (device)
  const uint8_t* phase;
  const double* khist;   // [nq][N]
  const double* a;       // [nq][N] current tangent scalars a = 1 - d
  const double* cp;      // [nq][N] c' (P1 pairs; Q1 keeps w below instead)
  double* a_out;         // [nq][N] written by the residual
  double* cp_out;        // (P1 pairs)
  const double* u;       // [dim][N]
  const double* v;       // second nodal input: z (trial) or the direction (Hessian)
  double* f;             // nodal output [dim][N]
  // Q1: the softening term c' (s:e) s of the tangent as (w:e) w with
  // w = sqrt(c') s, s = C : eps (c' >= 0). soft[e] has bit q set iff c' != 0
  // at point q of element e; w [nq][6][N] (xx,yy,zz,xy,xz,yz) is written, and
  // read, only at those points. Both come from the residual pass.
  const uint8_t* soft;
  uint8_t* soft_out;
  // Q1: the Hessian's per-element mask word (bits 0-7 the soft mask, 8-10 the
  // phase, 15 a = 1 at all 8 points), written by the residual pass
  const uint16_t* emask;
  uint16_t* emask_out;
  const double* sw;
  double* sw_out;
  // tens != 0: some phase follows the tensile-masking law, whose tangent
  // a C - c' (n:e) s is not symmetric (n = eps_t): the residual pass also
  // writes w_n = sqrt(c') n [nq][6][N] at the softening points (n = s at
  // energy-norm points), read by the trial and Hessian passes.
  int tens;
  const double* sn;
  double* sn_out;
  Reducer red;
  CgState* cg;           // Hessian in a CG iteration: skipped once cg->done
  int brick_shape;       // brick shape of the Q1 element passes (see launch_brick)
  // mean-stress control (Q1, FP64): U (device, 3x3) is the uniform part of the
  // Hessian's direction, added to D v at every point, and the Hessian writes
  // the point sums of B : (D v + U) (Voigt xx yy zz yz xz xy) to red_tail;
  // Pu (device, 3x3) is the uniform part of the trial step. Null: none.
  const double* U;
  Reducer red_tail;
  const double* Pu;
};

// Residual: f = D^T sigma(E + D u), writes a_out and cp_out (P1 pairs) or
// soft_out and sw_out (Q1), partial rows RES_*.
hipError_t launch_residual(const ElemArgs& A, hipStream_t s, int* nblocks);
// Trial at u + v: sums over points only (rows TRI_*), no nodal or point output.
hipError_t launch_trial(const ElemArgs& A, hipStream_t s, int* nblocks);
// Hessian: f = D^T B D v at the state (a and the softening term), rows HES_*
// (no-op once A.cg->done when A.cg is set).
hipError_t launch_hessian(const ElemArgs& A, hipStream_t s, int* nblocks);
// Profiling: a start / stop event pair that the next Hessian launch on this
// host thread records around the kernel itself (hipExtLaunchKernelGGL), so
// that their interval is the kernel's execution without its dispatch. The
// launch consumes the pair; (nullptr, nullptr) disarms it.
void arm_kernel_events(hipEvent_t start, hipEvent_t stop);
// Hessian operands in one precision (the FP32 copies of the state serve the
// mixed-precision CG; Q1 only).
template <typename R>
struct HessArgs {
  Grid g;
  MatTable mat;
  const double* E;       // macroscopic strain (device, FP64)
  const uint16_t* emask; // [N] mask word of each element (soft mask, phase, intact), as in ElemArgs
  const double* sw;      // [nq][6][N] w = sqrt(c') s at the softening points (FP64)
  int tens;              // as in ElemArgs: sn holds w_n = sqrt(c') n (FP64)
  const double* sn;
  const R* a;            // [nq][N] tangent scalars of the state
  const R* v;            // [dim][N] direction
  R* f;                  // [dim][N] K v
  Reducer red;           // rows HES_* (FP64)
  CgState* cg;           // skipped once cg->done when set
  int brick_shape;
  const double* U;       // mean-stress control (FP64 only): as in ElemArgs, or null
  Reducer red_tail;
};
// Hessian launch shapes: bricks 0..kBrickOnly-1, marching columns up to
// kHessianShapes-1 (valid where the grid's nx, ny are multiples of the column).
constexpr int kBrickOnly = 5;
constexpr int kHessianShapes = 13;
bool hessian_shape_valid(const Grid& g, int shape);
// FP32 Hessian f = D^T B D v (rows HES_* in FP64), 3D Q1 only.
hipError_t launch_hessian_f32(const HessArgs<float>& A, hipStream_t s, int* nblocks);
// Commit: khist <- max(khist, kappa_t(E + D u)) on damage points (khist is
// written through the const-cast pointer a_out).
hipError_t launch_commit(const ElemArgs& A, hipStream_t s);
// khist := kappa0 on damage points, 0 elsewhere (written through a_out).
hipError_t launch_init_history(const ElemArgs& A, hipStream_t s);
// Fields at points: grad (H) and stress into out_h / out_s ([N][nq][dim][dim]),
// damage and kappa into out_d / out_k ([N][nq]); any may be null.
hipError_t launch_fields(const ElemArgs& A, double* out_h, double* out_s, double* out_d,
                         double* out_k, hipStream_t s);

// ---- FFT / Green kernels (k_fft.hip) ---------------------------------------

// Complex type of a real type: double2 for double, float2 for float.
template <typename R> struct Complex;
template <> struct Complex<double> { using T = double2; };
template <> struct Complex<float> { using T = float2; };
template <typename R> using C2 = typename Complex<R>::T;

// Twiddle and symbol tables of one precision (R = double or float).
template <typename R>
struct FftTablesT {
  const C2<R>* tw;        // concatenated twiddle tables, see offsets
  int off_x, off_y, off_z, off_post;   // offsets (in complex values) of the Lx=nx/2, ny,
                                       // nz tables and of e^{-2 pi i k/nx}, k <= nx/2
  const R* sx;            // 4 sin^2(pi k / n) per axis (the 1D FE Laplacian symbol)
  const R* sy;
  const R* sz;
  // launch shape: threads of a plane block, columns and threads of a pencil block
  int plane_threads, pencil_cols, pencil_threads;
};
using FftTables = FftTablesT<double>;

bool fft_length_supported(int L);
// Launch shapes: whether one fits the grid (threads, staged values, LDS of a
// pencil block for reals of `real_bytes`), and the default one.
bool fft_launch_valid(const Grid& g, int plane_threads, int pencil_cols, int pencil_threads,
                      size_t real_bytes);
void fft_default_launch(const Grid& g, int* plane_threads, int* pencil_cols, int* pencil_threads);
template <typename R> size_t fft_plane_lds_bytes(const Grid& g);
// Raise the dynamic-LDS limit of the plane kernels a grid needs above 64 KiB
// (once per device; call on the context's device before any capture).
hipError_t fft_prepare(const Grid& g);
// The plane passes of this grid fit one block (LDS and staged values).
template <typename R> bool fft_plane_fits(const Grid& g);
// Pipeline entry points, R = double or float. `in`/`out` are [dim][N] reals,
// `spec` is the [dim][nz][ny][nx/2+1] complex work buffer.
// Green's operator: out = L^+ in (3D: three passes, 2D: one).
template <typename R>
hipError_t green_apply(const Grid& g, const FftTablesT<R>& t, const R* in, R* out, C2<R>* spec,
                       hipStream_t s, const CgState* skip = nullptr);
// The three passes of green_apply (3D) and the single 2D pass, launched
// separately so that each can be timed.
template <typename R>
hipError_t fft_plane_forward(const Grid& g, const FftTablesT<R>& t, const R* in, C2<R>* spec,
                             hipStream_t s, const CgState* skip = nullptr);
template <typename R>
hipError_t fft_pencil_green(const Grid& g, const FftTablesT<R>& t, C2<R>* spec, hipStream_t s,
                            const CgState* skip = nullptr);
template <typename R>
hipError_t fft_plane_inverse(const Grid& g, const FftTablesT<R>& t, C2<R>* spec, R* out,
                             hipStream_t s, const CgState* skip = nullptr);
template <typename R>
hipError_t fft_plane_green2d(const Grid& g, const FftTablesT<R>& t, const R* in, R* out,
                             C2<R>* spec, hipStream_t s, const CgState* skip = nullptr);

// CG iteration passes with the vector updates and decisions fused in (3D):
//  forward plane pass of Kd: every block adds the rows of the previous
//  direction update {g.d, z.g} (rows_dir) and of the Hessian {d.Kd, |Dd|^2}
//  (rows_hes) in a fixed order and takes the direction and curvature
//  decisions on its own copy of st_in (block (0,0) stores the result in
//  st_out and writes the trace); then z += alpha d, g += alpha Kd (or, when
//  the CG has just stopped on the sphere, z += tau d);
//  inverse plane pass (state st_in): instead of writing w = L^+ Kd, y +=
//  alpha w and partial rows {y_new.g, y_old.g} (one row per plane block,
//  accumulated in FP64 in either precision).
template <typename R>
struct CgFuse {
  const CgState* st_in;
  CgState* st_out;          // forward pass only
  const double* rows_dir;   // forward pass only
  int nb_dir;
  const double* rows_hes;   // forward pass only
  int nb_hes;
  const double* rows_tail;  // forward pass, mean-stress control: the Hessian's rows of the
                            // point sums of B : D d (Voigt, 6 per row), else null
  double* trace;            // forward pass only
  const R* d;
  R* z;
  R* g;
  R* y;
  double* partials;
};
template <typename R>
hipError_t fft_plane_forward_cg(const Grid& g, const FftTablesT<R>& t, const R* Kd, C2<R>* spec,
                                const CgFuse<R>& f, hipStream_t s);
template <typename R>
hipError_t fft_plane_inverse_cg(const Grid& g, const FftTablesT<R>& t, C2<R>* spec,
                                const CgFuse<R>& f, hipStream_t s, int* nblocks);
// Plain transforms (FP64): forward R2C and unscaled inverse C2R (times N).
hipError_t fft_forward(const Grid& g, const FftTables& t, const double* in, double2* spec,
                       hipStream_t s);
hipError_t fft_inverse(const Grid& g, const FftTables& t, double2* spec, double* out,
                       hipStream_t s);

// ---- vector kernels (k_vec.hip) --------------------------------------------

// x += alpha * y over n doubles
hipError_t vec_axpy(long long n, double alpha, const double* y, double* x, hipStream_t s);
// out = x + alpha * y
hipError_t vec_axpy_to(long long n, const double* x, double alpha, const double* y, double* out,
                       hipStream_t s);
// rows of x . y
// out = alpha x + beta y (out may alias x or y; with beta = 0 pass y = x)
hipError_t vec_lincomb(long long n, double alpha, const double* x, double beta, const double* y,
                       double* out, hipStream_t s);
hipError_t vec_dot(long long n, const double* x, const double* y, const Reducer& r,
                   hipStream_t s, int* nblocks);
// CG, after the curvature decision: z += alpha d ; g += alpha Kd, or, when the
// CG has just stopped on the trust-region sphere, z += tau d.
hipError_t cg_step_zg(long long n, const double* d, const double* Kd, double* z, double* g,
                      CgState* st, hipStream_t s);
// CG: y += alpha w, rows {y_new.g, y_old.g}
hipError_t cg_step_y(long long n, const double* w, double* y, const double* g, const Reducer& r,
                     const CgState* st, hipStream_t s, int* nblocks);
// CG: d = -y + beta d, rows {g.d, z.g} (R = double or float; sums in FP64).
// With rows_res set, every block first adds the nb_res rows {y_new.g,
// y_old.g} of the inverse plane pass and takes the residual decision on its
// own copy of st (block 0 stores it in st_out and writes the trace);
// otherwise it reads beta from st.
// Start of a CG solve (FP64): z = 0, g = g0, y = y0, d0 = -y0, with the rows
// {g.d, z.g = 0} of the first direction decision (the sums of cg_step_d at
// beta = 0, in the same order).
hipError_t cg_start(long long n, const double* g0, const double* y0, double* z, double* g,
                    double* y, double* d, const Reducer& r, hipStream_t s, int* nblocks);
template <typename R>
hipError_t cg_step_d(long long n, const R* y, R* d, const R* g, const R* z, const Reducer& r,
                     const CgState* st, hipStream_t s, int* nblocks,
                     const double* rows_res = nullptr, int nb_res = 0, CgState* st_out = nullptr,
                     double* trace = nullptr);
// Mixed precision: rows of x . y over FP32 vectors (FP64 sums); y = (float) x;
// y = (double) x; out = (float)(x + y).
hipError_t vec_dot_f32(long long n, const float* x, const float* y, const Reducer& r,
                       hipStream_t s, int* nblocks);
hipError_t vec_to_f32(long long n, const double* x, float* y, hipStream_t s);
hipError_t vec_to_f64(long long n, const float* x, double* y, hipStream_t s);
hipError_t vec_add_f32(long long n, const float* x, const double* y, float* out, hipStream_t s);
// After the host recomputed the residual of a restart: beta = 0, run again.
hipError_t cg_resume(CgState* st, hipStream_t s);

// Finish kernels (one block): add `nblocks` rows of `nv` partials in a fixed
// order, then
enum { FIN_OUT = 0,          // write the nv totals to out (device or host-mapped)
       FIN_CURVATURE = 1,    // CG curvature decision on {d.Kd, |Dd|^2}
       FIN_RESIDUAL = 2,     // CG residual decision on {y_new.g, y_old.g}
       FIN_DIRECTION = 3 };  // CG direction update on {g.d, z.g}
hipError_t finish(int kind, const Reducer& r, int nblocks, int nv, double* out, CgState* st,
                  double* trace, hipStream_t s);
// Direction update (rows rd of {g.d, z.g}) then curvature decision (rows rc of
// {d.Kd, |Dd|^2}), one block.
hipError_t finish_direction_curvature(const Reducer& rd, int nbd, const Reducer& rc, int nbc,
                                      CgState* st, double* trace, hipStream_t s);

}  // namespace hfe
