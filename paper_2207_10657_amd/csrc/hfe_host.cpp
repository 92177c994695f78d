// Host side of the library: context and workspace management, the C ABI, and
// the scalar logic of the trust-region Newton solver (Algorithm 2) and of the
// truncated CG (Algorithm 1). Every vector operation runs in the kernels of
// k_element.hip, k_fft.hip and k_vec.hip; the host only sees reduced scalars.
//
// Displacement coordinates. The paper iterates on compatible strain fields
// with the projector G = D (D^T D)^+ D^T (Sec. 2.1). Every such field is D u
// for a nodal field u, so the CG of Algorithm 1 is run on nodal vectors:
//   model gradient  G sigma          <->  g = D^T sigma (nodal), y = L^+ g
//   Hessian action  G B (D d)        <->  K d = D^T B D d, then L^+ (K d)
//   <r, r>                           =    y . g
//   <d, G B d>                       =    d . K d
//   <r_{j+1}, r_j>  (restart test)   =    y_j . g_{j+1}
//   <r, d>                           =    g . d
//   ||d||^2                          =    sum over points of |D d|^2
// with L = D^T D the FE Laplacian. <z, d> and ||z||^2 follow from
// L d_{j+1} = -g_{j+1} + beta L d_j:
//   <z_{j+1}, d_{j+1}> = -z_{j+1}.g_{j+1} + beta (<z_j, d_j> + alpha ||d_j||^2)
//   ||z_{j+1}||^2      = ||z_j||^2 + 2 alpha <z_j, d_j> + alpha^2 ||d_j||^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hfe_internal.h"

using hfe::Grid;

namespace {

constexpr size_t kAlign = 256;
constexpr int kTraceCap = 1 << 16;    // CG trace entries kept per solve
constexpr int kCgBatch = 8;           // the longest batch of CG iterations between host polls
constexpr int kCgSlots = 4;           // captured batches of 1, 2, 4, 8 iterations

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t u, z, d, g, y, Kd, w, g0, y0, tmp;          // nodal [dim][N]
  size_t a, cp, kh;                                   // per point [nq][N]
  size_t sw;                                          // per point [nq][6][N] (Q1)
  size_t sn;                                          // per point [nq][6][N] (Q1)
  size_t phase;                                       // N bytes
  size_t soft;                                        // N bytes: element softens
  size_t emask;                                       // N uint16: Hessian mask word
  size_t spec;                                        // dim*nz*ny*(nx/2+1) double2
  size_t partials;                                    // rows * 16 doubles
  size_t partials2;                                   // second row buffer (direction sums)
  size_t partials3;                                   // rows of 6 (mean-stress tail sums)
  size_t Udev, Pudev;                                 // 3x3 uniform parts (mean-stress control)
  size_t cgstate;                                     // device CgState
  size_t cgmid;                                       // its copy between the fused passes
  size_t trace;                                       // CG trace, 2 doubles per entry
  size_t Edev;                                        // macroscopic strain (9 doubles)
  size_t tw;                                          // twiddles
  size_t stab;                                        // sin^2 tables
  // FP32 copies for the mixed-precision CG
  size_t z32, d32, g32, y32, Kd32, tmp32;             // nodal [dim][N] floats
  size_t a32;                                         // per point [nq][N] floats
  size_t spec32;                                      // dim*nz*ny*(nx/2+1) float2
  size_t tw32, stab32;                                // tables
  size_t total;
  int partial_rows;
  int n_tw, n_stab;
};

bool grid_ok(const hfe_grid* gr, std::string* why) {
  if (!gr) { *why = "grid is NULL"; return false; }
  const int nx = gr->n[0], ny = gr->n[1], nz = gr->n[2];
  if (gr->dim == 2) {
    if (gr->element != HFE_P1_PAIR) { *why = "2D grids use the HFE_P1_PAIR element"; return false; }
    if (nz != 1) { *why = "2D grids have nz = 1"; return false; }
  } else if (gr->dim == 3) {
    if (gr->element != HFE_Q1) { *why = "3D grids use the HFE_Q1 element"; return false; }
  } else {
    *why = "dim must be 2 or 3";
    return false;
  }
  if (nx < 2 || ny < 1 || nz < 1 || (nx & 1)) { *why = "nx must be even and >= 2, ny, nz >= 1"; return false; }
  if (!hfe::fft_length_supported(nx / 2) || !hfe::fft_length_supported(ny) ||
      !hfe::fft_length_supported(nz)) {
    *why = "nx/2, ny and nz must each be one of 1,2,3,4,6,8,12,16,24,32,48,64,96,128";
    return false;
  }
  if (((size_t)(nx / 2 + 1) * ny + nx + 1 + ny) * 16 > 159 * 1024) {
    *why = "a spectral x-y plane (with its twiddles) must fit in 160 KiB of LDS";
    return false;
  }
  return true;
}

Grid make_grid(const hfe_grid* gr) {
  Grid g;
  g.nx = gr->n[0];
  g.ny = gr->n[1];
  g.nz = gr->n[2];
  g.dim = gr->dim;
  g.element = gr->element;
  g.nq = gr->element == HFE_Q1 ? 8 : 2;
  g.na = gr->element == HFE_Q1 ? 8 : 4;
  g.N = (long long)g.nx * g.ny * g.nz;
  return g;
}

Layout make_layout(const Grid& g) {
  Layout L;
  size_t off = 0;
  const size_t nod = (size_t)g.dim * g.N * sizeof(double);
  const size_t pts = (size_t)g.nq * g.N * sizeof(double);
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  L.u = take(nod); L.z = take(nod); L.d = take(nod); L.g = take(nod); L.y = take(nod);
  L.Kd = take(nod); L.w = take(nod); L.g0 = take(nod); L.y0 = take(nod);
  L.tmp = take(nod);
  L.a = take(pts); L.cp = take(pts); L.kh = take(pts);
  L.sw = take(g.element == HFE_Q1 ? 6 * pts : 0);
  L.sn = take(g.element == HFE_Q1 ? 6 * pts : 0);
  L.phase = take((size_t)g.N);
  L.soft = take((size_t)g.N);
  L.emask = take((size_t)g.N * sizeof(uint16_t));
  L.spec = take((size_t)g.dim * g.nz * g.ny * (g.nx / 2 + 1) * sizeof(double2));
  // rows of partial sums: one per block of the element and vector kernels,
  // one per canonical tile of the Hessian
  L.partial_rows = (int)std::max<long long>(
      std::max<long long>((g.N + hfe::kBlock - 1) / hfe::kBlock, 1024), hfe::tile_count(g));
  L.partials = take((size_t)L.partial_rows * hfe::kMaxPartials * sizeof(double));
  L.partials2 = take((size_t)L.partial_rows * 2 * sizeof(double));
  L.partials3 = take((size_t)L.partial_rows * 6 * sizeof(double));
  L.Udev = take(9 * sizeof(double));
  L.Pudev = take(9 * sizeof(double));
  L.cgstate = take(sizeof(hfe::CgState));
  L.cgmid = take(sizeof(hfe::CgState));
  L.trace = take((size_t)2 * kTraceCap * sizeof(double));
  L.Edev = take(9 * sizeof(double));
  L.n_tw = g.nx / 2 + g.ny + g.nz + (g.nx / 2 + 1);
  L.tw = take((size_t)L.n_tw * sizeof(double2));
  L.n_stab = (g.nx / 2 + 1) + g.ny + g.nz;
  L.stab = take((size_t)L.n_stab * sizeof(double));
  const size_t nod32 = (size_t)g.dim * g.N * sizeof(float);
  const size_t pts32 = (size_t)g.nq * g.N * sizeof(float);
  L.z32 = take(nod32); L.d32 = take(nod32); L.g32 = take(nod32);
  L.y32 = take(nod32); L.Kd32 = take(nod32); L.tmp32 = take(nod32);
  L.a32 = take(pts32);
  L.spec32 = take((size_t)g.dim * g.nz * g.ny * (g.nx / 2 + 1) * sizeof(float2));
  L.tw32 = take((size_t)L.n_tw * sizeof(float2));
  L.stab32 = take((size_t)L.n_stab * sizeof(float));
  L.total = off;
  return L;
}

// e^{-2 pi i k / n} and 4 sin^2(pi k / n), evaluated in long double.
void twiddles(int n, int count, std::vector<double2>& out) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < count; ++k) {
    const long double a = 2.0L * pi * (long double)k / (long double)n;
    out.push_back(make_double2((double)cosl(a), (double)(-sinl(a))));
  }
}
void sin2_table(int n, int count, std::vector<double>& out) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < count; ++k) {
    const long double s = sinl(pi * (long double)k / (long double)n);
    out.push_back((double)(4.0L * s * s));
  }
}

struct ProfEvent { int kernel; hipEvent_t start, stop; };

// A captured batch of CG iterations and the timing events inside it.
struct CgGraph {
  hipGraphExec_t exec = nullptr;
  int iters = 0;
  bool profiled = false;
  std::vector<ProfEvent> ev;
};

}  // namespace

struct hfe_ctx {
  Grid g;
  Layout L;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // device views
  double *u, *z, *d, *gv, *y, *Kd, *w, *g0, *y0, *tmp;
  double *a, *cp, *kh;
  double* sw;                // Q1: w = sqrt(c') s at the softening points
  double* sn;                // Q1, tensile-masking phases present: w_n = sqrt(c') n
  bool tens = false;         // some phase follows the tensile-masking law
  uint8_t* phase;
  uint8_t* soft;             // per element: bit q set iff c' != 0 at point q (Q1)
  uint16_t* emask;           // per element: soft mask, phase, intact bit (Q1 Hessian)
  double n_soft = 0.0;       // softening points of the state (Q1)
  double prof_soft_sum = 0.0;  // profiling: n_soft summed over the Hessian launches
  long long prof_soft_n = 0;
  double2* spec;
  double* partials;
  double* partials2;
  double* partials3;         // the Hessian's tail rows (mean-stress control)
  double* Udev;              // uniform part of an operator input (mean-stress control)
  double* Pudev;             // uniform part of the trial step (mean-stress control)
  int nb_dir = 0;            // rows of the pending direction sums in partials2
  hfe::CgState* cg;          // device CG state (after each iteration)
  hfe::CgState* cg_mid;      // the state after the forward plane pass's decisions (3D)
  double* Edev;              // device copy of E
  double* trace;             // device CG trace
  hfe::FftTables tabs;
  // mixed precision: FP32 CG vectors, FP32 copies of the state, FP32 tables
  float *z32, *d32, *g32, *y32, *Kd32, *tmp32, *a32;
  float2* spec32;
  hfe::FftTablesT<float> tabs32;
  bool state32_fresh = false;  // a32 matches a
  double* hscal = nullptr;   // pinned, device-mapped: reduction totals land here
  double* dscal = nullptr;   // device alias of hscal
  hfe::CgState* hcg = nullptr;  // pinned host copy of the CG state
  // host state
  hfe::MatTable mat;
  bool mat_set[hfe::kMaxPhases] = {};
  int n_phases = 0;
  bool have_micro = false, have_state = false, history_ready = false;
  double E[9] = {0};
  bool R_init = false;
  double R = 0, Rmax = 0, R0_default = 0, Rmax_default = 0;
  double r_eq = 0, sig_norm2 = 0, rr0 = 0;
  double rr0_nodal = 0;      // y0 . g0 (rr0 adds the tails of mean-stress control)
  // mean-stress control: free macroscopic strain components (Voigt index)
  int ne = 0;
  int comp[hfe::kMaxFree] = {};
  double g0e[hfe::kMaxFree] = {};   // tails of the residual: sum_q sigma : B_m
  double ze[hfe::kMaxFree] = {};    // tail of the last CG step
  double sigma_sum[6] = {0};
  std::vector<hfe_newton_record> log;
  std::vector<double> cg_trace;
  std::string err;
  // profiling
  bool profiling = false;
  std::vector<std::string> knames;
  std::vector<int> kcount;
  std::vector<double> kms;
  std::vector<ProfEvent> pending;
  std::vector<hipEvent_t> pool;
  std::vector<ProfEvent>* prof_sink = nullptr;   // events recorded while capturing
  // CG iteration graphs of 1, 2, 4 and 8 iterations (slot s holds 2^s)
  hipStream_t cap_stream = nullptr;
  CgGraph graphs[kCgSlots];
  int cg_predict = 2;        // CG iterations of the previous solve (first batch size)
  int graph_precision = HFE_FP64;   // precision the captured graphs run
  bool use_graphs = true;
  int brick_shape = 0;       // Q1 Hessian brick shape, FP64 (HFE_BRICK_SHAPE=0..4 overrides)
  int brick_shape32 = 0;     // and FP32
};

namespace {

hfe_status fail(hfe_ctx* c, hfe_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

#define HIPCHK(ctx, call)                                                          \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, HFE_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int kernel_id(hfe_ctx* c, const char* name) {
  for (size_t i = 0; i < c->knames.size(); ++i)
    if (c->knames[i] == name) return (int)i;
  c->knames.push_back(name);
  c->kcount.push_back(0);
  c->kms.push_back(0.0);
  return (int)c->knames.size() - 1;
}

hipEvent_t take_event(hfe_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket a group of launches with events when profiling is on.
struct Prof {
  hfe_ctx* c;
  int id = -1;
  hipEvent_t s = nullptr;
  Prof(hfe_ctx* ctx, const char* name) : c(ctx) {
    if (!c->profiling) return;
    id = kernel_id(c, name);
    s = take_event(c);
    if (s) hipEventRecord(s, c->stream);
  }
  ~Prof() {
    if (!c->profiling || !s) return;
    hipEvent_t e = take_event(c);
    if (!e) return;
    hipEventRecord(e, c->stream);
    (c->prof_sink ? c->prof_sink : &c->pending)->push_back({id, s, e});
  }
};

// Profiling of a Hessian launch. In 3D the launch records the events at the
// kernel's own start and end (hfe::arm_kernel_events), so the interval is
// the kernel's execution; events recorded on the stream around a launch
// (Prof) also hold its dispatch, a few microseconds per launch at 64^3. The
// 2D Hessian is timed as Prof does.
struct ProfKernel {
  hfe_ctx* c;
  int id = -1;
  hipEvent_t s = nullptr, e = nullptr;
  bool armed = false;
  ProfKernel(hfe_ctx* ctx, const char* name) : c(ctx) {
    if (!c->profiling) return;
    id = kernel_id(c, name);
    c->prof_soft_sum += c->n_soft;
    ++c->prof_soft_n;
    s = take_event(c);
    e = s ? take_event(c) : nullptr;
    if (!e) {
      if (s) c->pool.push_back(s);
      s = nullptr;
      return;
    }
    if (c->g.dim == 3) {
      hfe::arm_kernel_events(s, e);
      armed = true;
    } else {
      hipEventRecord(s, c->stream);
    }
  }
  ~ProfKernel() {
    if (!c->profiling || !s || !e) return;
    if (armed) hfe::arm_kernel_events(nullptr, nullptr);   // if the launch did not happen
    else hipEventRecord(e, c->stream);
    (c->prof_sink ? c->prof_sink : &c->pending)->push_back({id, s, e});
  }
};

// Collect finished event pairs (call after a stream synchronisation).
void prof_drain(hfe_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      c->kcount[p.kernel] += 1;
      c->kms[p.kernel] += ms;
    }
    c->pool.push_back(p.start);
    c->pool.push_back(p.stop);
  }
  c->pending.clear();
}

// Wait for the stream; reduction totals are then visible in hscal.
// Accumulate the timings of the events inside a replayed graph.
void prof_drain_graph(hfe_ctx* c, const CgGraph& G) {
  for (const auto& p : G.ev) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      c->kcount[p.kernel] += 1;
      c->kms[p.kernel] += ms;
    }
  }
}

void destroy_graphs(hfe_ctx* c) {
  for (auto& G : c->graphs) {
    if (G.exec) hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
    for (auto& p : G.ev) {
      c->pool.push_back(p.start);
      c->pool.push_back(p.stop);
    }
    G.ev.clear();
  }
}

hfe_status sync(hfe_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->profiling) prof_drain(c);
  return HFE_OK;
}

hfe::Reducer reducer(hfe_ctx* c) {
  hfe::Reducer r;
  r.partials = c->partials;
  return r;
}

// Complete a reduction of nb rows of nv partials: totals to `out`, or a CG decision.
hfe_status finish(hfe_ctx* c, int kind, int nb, int nv, double* out) {
  Prof p(c, "finish");
  HIPCHK(c, hfe::finish(kind, reducer(c), nb, nv, out, c->cg, c->trace, c->stream));
  return HFE_OK;
}

hfe::ElemArgs elem_args(hfe_ctx* c) {
  hfe::ElemArgs A;
  A.g = c->g;
  A.mat = c->mat;
  A.E = c->Edev;
  A.phase = c->phase;
  A.khist = c->kh;
  A.a = c->a;
  A.cp = c->cp;
  A.a_out = nullptr;
  A.cp_out = nullptr;
  A.u = c->u;
  A.v = nullptr;
  A.f = nullptr;
  A.soft = c->soft;
  A.soft_out = nullptr;
  A.emask = c->emask;
  A.emask_out = nullptr;
  A.sw = c->sw;
  A.sw_out = nullptr;
  A.tens = c->tens;
  A.sn = c->sn;
  A.sn_out = nullptr;
  A.red = reducer(c);
  A.cg = nullptr;
  A.brick_shape = c->brick_shape;
  A.U = nullptr;
  A.red_tail.partials = c->partials3;
  A.Pu = nullptr;
  return A;
}

long long ndof(const hfe_ctx* c) { return (long long)c->g.dim * c->g.N; }

// Offsets of the reduction totals in hscal.
enum { S_HES = 0, S_RES = 8, S_RR0 = 24, S_TRI = 32, S_DOT = 48, S_ESTAGE = 56, S_TAIL = 72,
       S_USTAGE = 80, S_COUNT = 96 };

// y = L^+ x (the passes are skipped once skip->done is set)
hfe_status green(hfe_ctx* c, const double* x, double* y, const hfe::CgState* skip = nullptr) {
  if (c->g.dim == 2) {
    Prof p(c, "fft_green2d");
    HIPCHK(c, hfe::fft_plane_green2d(c->g, c->tabs, x, y, c->spec, c->stream, skip));
    return HFE_OK;
  }
  {
    Prof p(c, "fft_plane_fwd");
    HIPCHK(c, hfe::fft_plane_forward(c->g, c->tabs, x, c->spec, c->stream, skip));
  }
  {
    Prof p(c, "fft_pencil_green");
    HIPCHK(c, hfe::fft_pencil_green(c->g, c->tabs, c->spec, c->stream, skip));
  }
  {
    Prof p(c, "fft_plane_inv");
    HIPCHK(c, hfe::fft_plane_inverse(c->g, c->tabs, c->spec, y, c->stream, skip));
  }
  return HFE_OK;
}

// out = K v at the current state. Totals (d.Kd, |Dd|^2) to hscal[S_HES..], or,
// inside the CG, the curvature decision on the device state.
// U (device 3x3, may be null): the uniform part of v under mean-stress
// control; its point sums of B : (D v + U) go to hscal[S_TAIL..] (Voigt).
hfe_status stiffness(hfe_ctx* c, const double* v, double* out, bool in_cg,
                     const double* U = nullptr) {
  hfe::ElemArgs A = elem_args(c);
  A.v = v;
  A.f = out;
  A.U = U;
  if (in_cg) A.cg = c->cg;
  int nb = 0;
  {
    ProfKernel p(c, "stiffness");
    HIPCHK(c, hfe::launch_hessian(A, c->stream, &nb));
  }
  if (U && !in_cg) {
    hfe::Reducer r;
    r.partials = c->partials3;
    Prof p(c, "finish");
    HIPCHK(c, hfe::finish(hfe::FIN_OUT, r, nb, 6, c->dscal + S_TAIL, c->cg, c->trace, c->stream));
  }
  return in_cg ? finish(c, hfe::FIN_CURVATURE, nb, hfe::HES_NV, nullptr)
               : finish(c, hfe::FIN_OUT, nb, hfe::HES_NV, c->dscal + S_HES);
}

// x . y into a device (or host-mapped) address
hfe_status dot(hfe_ctx* c, const double* x, const double* y, double* dev_out) {
  int nb = 0;
  {
    Prof p(c, "cg_vec");
    HIPCHK(c, hfe::vec_dot(ndof(c), x, y, reducer(c), c->stream, &nb));
  }
  return finish(c, hfe::FIN_OUT, nb, 1, dev_out);
}

// Copy E to the device (through the pinned staging area; synchronous, rare).
hfe_status upload_E(hfe_ctx* c) {
  double* stage = c->hscal + S_ESTAGE;
  for (int k = 0; k < 9; ++k) stage[k] = c->E[k];
  HIPCHK(c, hipMemcpyAsync(c->Edev, stage, 9 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HFE_OK;
}

// Tails of the residual under mean-stress control, g0_m = sum_q sigma : B_m
// (from the stress sums), and r_eq = ||G_M sigma|| / ||sigma|| with
// ||G_M sigma||^2 = y0 . g0 + sum_m g0_m^2 / N_qp.
void refresh_tails(hfe_ctx* c) {
  // stress sums are (xx, yy, zz, xy, xz, yz); tails use Voigt (xx, yy, zz, yz, xz, xy)
  const double* s = c->sigma_sum;
  const double voigt[6] = {s[0], s[1], s[2], s[5], s[4], s[3]};
  const double nqp = (double)c->g.N * c->g.nq;
  c->rr0 = c->rr0_nodal;
  for (int m = 0; m < c->ne; ++m) {
    c->g0e[m] = hfe::tail_pair(c->comp[m], voigt);
    c->rr0 += c->g0e[m] * c->g0e[m] / nqp;
  }
  c->r_eq = c->sig_norm2 > 0.0 ? std::sqrt(std::max(c->rr0, 0.0)) / std::sqrt(c->sig_norm2) : 0.0;
}

// Upload a 3x3 (a uniform field) to the device through the pinned staging
// area (synchronous, rare).
hfe_status upload_3x3(hfe_ctx* c, const double* U, double* dev) {
  double* stage = c->hscal + S_USTAGE;
  for (int k = 0; k < 9; ++k) stage[k] = U[k];
  HIPCHK(c, hipMemcpyAsync(dev, stage, 9 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HFE_OK;
}

// Residual at (u, E) with E already on the device: g0 = D^T sigma, tangent
// scalars, y0 = L^+ g0, the stress sums and r_eq.
hfe_status evaluate_residual(hfe_ctx* c) {
  hfe::ElemArgs A = elem_args(c);
  A.a_out = c->a;
  A.cp_out = c->cp;
  A.soft_out = c->soft;
  A.emask_out = c->emask;
  A.sw_out = c->sw;
  A.sn_out = c->sn;
  A.f = c->g0;
  int nb = 0;
  {
    Prof p(c, "residual");
    HIPCHK(c, hfe::launch_residual(A, c->stream, &nb));
  }
  hfe_status st = finish(c, hfe::FIN_OUT, nb, hfe::RES_NV, c->dscal + S_RES);
  if (st) return st;
  st = green(c, c->g0, c->y0);
  if (st) return st;
  st = dot(c, c->y0, c->g0, c->dscal + S_RR0);
  if (st) return st;
  st = sync(c);
  if (st) return st;
  const double* h = c->hscal;
  for (int k = 0; k < 6; ++k) c->sigma_sum[k] = h[S_RES + k];
  c->sig_norm2 = h[S_RES + hfe::RES_SS];
  c->n_soft = h[S_RES + hfe::RES_NSOFT];
  c->rr0_nodal = h[S_RR0];
  if (!std::isfinite(c->rr0_nodal) || !std::isfinite(c->sig_norm2))
    return fail(c, HFE_ENUMERIC, "non-finite stress or residual");
  refresh_tails(c);
  c->have_state = true;
  c->state32_fresh = false;
  return HFE_OK;
}

hfe_status evaluate_state(hfe_ctx* c) {
  hfe_status st = upload_E(c);
  if (st) return st;
  return evaluate_residual(c);
}

struct CgInfo { int iters = 0, restarts = 0, matvecs = 0; };

// d = -y + beta d with <r, d> and z.g into the second row buffer; the
// direction update of the state is applied by the next iteration's finish.
hfe_status direction(hfe_ctx* c) {
  hfe::Reducer r;
  r.partials = c->partials2;
  Prof p(c, "cg_vec");
  HIPCHK(c, hfe::cg_step_d(ndof(c), c->y, c->d, c->gv, c->z, r, c->cg, c->stream, &c->nb_dir));
  return HFE_OK;
}

// ---- mixed precision: the CG of Algorithm 1 on FP32 vectors ----------------

// FP32 copy of the tangent scalars a read by the FP32 Hessian (the softening
// factors w are read in FP64).
hfe_status refresh_state32(hfe_ctx* c) {
  if (c->state32_fresh) return HFE_OK;
  const long long np = (long long)c->g.nq * c->g.N;
  {
    Prof p(c, "convert");
    HIPCHK(c, hfe::vec_to_f32(np, c->a, c->a32, c->stream));
  }
  c->state32_fresh = true;
  return HFE_OK;
}

hfe::HessArgs<float> hess_args32(hfe_ctx* c, const float* v, float* out, bool in_cg) {
  hfe::HessArgs<float> H;
  H.g = c->g;
  H.mat = c->mat;
  H.E = c->Edev;
  H.emask = c->emask;
  H.a = c->a32;
  H.sw = c->sw;
  H.tens = c->tens;
  H.sn = c->sn;
  H.v = v;
  H.f = out;
  H.red = reducer(c);
  H.cg = in_cg ? c->cg : nullptr;
  H.brick_shape = c->brick_shape32;
  H.U = nullptr;                 // mean-stress control runs in FP64 only
  H.red_tail.partials = nullptr;
  return H;
}

// out = K v in FP32 (state copies must be fresh); totals as in stiffness().
hfe_status stiffness32(hfe_ctx* c, const float* v, float* out, bool in_cg) {
  int nb = 0;
  {
    ProfKernel p(c, "stiffness_f32");
    HIPCHK(c, hfe::launch_hessian_f32(hess_args32(c, v, out, in_cg), c->stream, &nb));
  }
  return in_cg ? finish(c, hfe::FIN_CURVATURE, nb, hfe::HES_NV, nullptr)
               : finish(c, hfe::FIN_OUT, nb, hfe::HES_NV, c->dscal + S_HES);
}

// y = L^+ x in FP32 (3D)
hfe_status green32(hfe_ctx* c, const float* x, float* y) {
  {
    Prof p(c, "fft_plane_fwd_f32");
    HIPCHK(c, hfe::fft_plane_forward(c->g, c->tabs32, x, c->spec32, c->stream));
  }
  {
    Prof p(c, "fft_pencil_green_f32");
    HIPCHK(c, hfe::fft_pencil_green(c->g, c->tabs32, c->spec32, c->stream));
  }
  {
    Prof p(c, "fft_plane_inv_f32");
    HIPCHK(c, hfe::fft_plane_inverse(c->g, c->tabs32, c->spec32, y, c->stream));
  }
  return HFE_OK;
}

hfe_status dot32(hfe_ctx* c, const float* x, const float* y, double* dev_out) {
  int nb = 0;
  {
    Prof p(c, "cg_vec_f32");
    HIPCHK(c, hfe::vec_dot_f32(ndof(c), x, y, reducer(c), c->stream, &nb));
  }
  return finish(c, hfe::FIN_OUT, nb, 1, dev_out);
}

hfe_status direction32(hfe_ctx* c) {
  hfe::Reducer r;
  r.partials = c->partials2;
  Prof p(c, "cg_vec_f32");
  HIPCHK(c, hfe::cg_step_d<float>(ndof(c), c->y32, c->d32, c->g32, c->z32, r, c->cg, c->stream,
                                  &c->nb_dir));
  return HFE_OK;
}

// Operands of the fused CG passes of a 3D iteration: the forward pass reads
// the state after the previous iteration (cg) with the pending direction rows
// (partials2) and the Hessian rows (partials, nb_hes), and stores its
// decisions in cg_mid.
template <typename R>
hfe::CgFuse<R> fuse_args(hfe_ctx* c, int nb_hes, const R* d, R* z, R* g, R* y) {
  hfe::CgFuse<R> f;
  f.st_in = c->cg;
  f.st_out = c->cg_mid;
  f.rows_dir = c->partials2;
  f.nb_dir = c->nb_dir;
  f.rows_hes = c->partials;
  f.nb_hes = nb_hes;
  f.rows_tail = c->ne > 0 ? c->partials3 : nullptr;
  f.trace = c->trace;
  f.d = d;
  f.z = z;
  f.g = g;
  f.y = y;
  f.partials = c->partials;
  return f;
}

// The FP64 iteration below with FP32 vectors, Hessian and FFT (3D).
hfe_status cg_iteration32(hfe_ctx* c) {
  int nb = 0;
  {
    ProfKernel p(c, "stiffness_f32");
    HIPCHK(c, hfe::launch_hessian_f32(hess_args32(c, c->d32, c->Kd32, true), c->stream, &nb));
  }
  hfe::CgFuse<float> f = fuse_args<float>(c, nb, c->d32, c->z32, c->g32, c->y32);
  {
    Prof p(c, "fft_plane_fwd_cg_f32");
    HIPCHK(c, hfe::fft_plane_forward_cg(c->g, c->tabs32, (const float*)c->Kd32, c->spec32, f,
                                        c->stream));
  }
  {
    Prof p(c, "fft_pencil_green_f32");
    HIPCHK(c, hfe::fft_pencil_green(c->g, c->tabs32, c->spec32, c->stream, c->cg_mid));
  }
  f.st_in = c->cg_mid;
  {
    Prof p(c, "fft_plane_inv_cg_f32");
    HIPCHK(c, hfe::fft_plane_inverse_cg(c->g, c->tabs32, c->spec32, f, c->stream, &nb));
  }
  hfe::Reducer r;
  r.partials = c->partials2;
  Prof p(c, "cg_vec_f32");
  HIPCHK(c, hfe::cg_step_d<float>(ndof(c), c->y32, c->d32, c->g32, c->z32, r, c->cg_mid, c->stream,
                                  &c->nb_dir, c->partials, nb, c->cg, c->trace));
  return HFE_OK;
}

// One CG iteration, all decisions on the device (no host synchronisation):
// K d, [direction update of the previous iteration + curvature decision],
// z/g update + forward FFT, Green z-pass, inverse FFT + y update + residual
// sums, [residual decision], new direction. In 3D the bracketed decisions
// are taken inside the neighbouring passes (5 launches per iteration).
hfe_status cg_iteration(hfe_ctx* c) {
  const long long n = ndof(c);
  hfe::ElemArgs A = elem_args(c);
  A.v = c->d;
  A.f = c->Kd;
  A.cg = c->cg;
  // mean-stress control: the direction's uniform part, kept in the CG state
  if (c->ne > 0) A.U = c->cg->dU;
  int nb = 0;
  {
    ProfKernel p(c, "stiffness");
    HIPCHK(c, hfe::launch_hessian(A, c->stream, &nb));
  }
  if (c->g.dim == 3) {
    // 3D: five launches, the decisions fused into the forward plane pass
    // (direction + curvature) and into the direction update (residual)
    hfe::CgFuse<double> f = fuse_args<double>(c, nb, c->d, c->z, c->gv, c->y);
    {
      Prof p(c, "fft_plane_fwd_cg");
      HIPCHK(c, hfe::fft_plane_forward_cg(c->g, c->tabs, (const double*)c->Kd, c->spec, f,
                                          c->stream));
    }
    {
      Prof p(c, "fft_pencil_green");
      HIPCHK(c, hfe::fft_pencil_green(c->g, c->tabs, c->spec, c->stream, c->cg_mid));
    }
    f.st_in = c->cg_mid;
    {
      Prof p(c, "fft_plane_inv_cg");
      HIPCHK(c, hfe::fft_plane_inverse_cg(c->g, c->tabs, c->spec, f, c->stream, &nb));
    }
    hfe::Reducer r;
    r.partials = c->partials2;
    Prof p(c, "cg_vec");
    HIPCHK(c, hfe::cg_step_d<double>(n, c->y, c->d, c->gv, c->z, r, c->cg_mid, c->stream,
                                     &c->nb_dir, c->partials, nb, c->cg, c->trace));
    return HFE_OK;
  }
  // 2D: separate passes and finish kernels
  {
    hfe::Reducer rd;
    rd.partials = c->partials2;
    Prof p(c, "finish");
    HIPCHK(c, hfe::finish_direction_curvature(rd, c->nb_dir, reducer(c), nb, c->cg, c->trace,
                                              c->stream));
  }
  {
    Prof p(c, "cg_vec");
    HIPCHK(c, hfe::cg_step_zg(n, c->d, c->Kd, c->z, c->gv, c->cg, c->stream));
  }
  hfe_status st = green(c, c->Kd, c->w, c->cg);
  if (st) return st;
  {
    Prof p(c, "cg_vec");
    HIPCHK(c, hfe::cg_step_y(n, c->w, c->y, c->gv, reducer(c), c->cg, c->stream, &nb));
  }
  st = finish(c, hfe::FIN_RESIDUAL, nb, 2, nullptr);
  if (st) return st;
  return direction(c);
}

// Graph capture and instantiation are serialised across the process: the
// contexts of a batch solve on separate host threads, and each captures its
// CG graphs the first time it needs them. Replays stay concurrent.
std::mutex g_capture_mutex;

// Enqueue `k` CG iterations: a replay of a captured graph (captured on a
// private stream, launched on the context's stream), or plain launches.
hfe_status cg_batch(hfe_ctx* c, int slot, int k) {
  // timing events cannot be recorded inside a captured graph on this
  // runtime, so a profiled solve launches the kernels one by one
  auto iteration = [&]() {
    return c->graph_precision == HFE_MIXED ? cg_iteration32(c) : cg_iteration(c);
  };
  if (!c->use_graphs || c->profiling) {
    for (int i = 0; i < k; ++i) {
      hfe_status st = iteration();
      if (st) return st;
    }
    return HFE_OK;
  }
  CgGraph& G = c->graphs[slot];
  if (G.exec && G.profiled != c->profiling) {
    hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
    for (auto& p : G.ev) {
      c->pool.push_back(p.start);
      c->pool.push_back(p.stop);
    }
    G.ev.clear();
  }
  if (!G.exec) {
    std::lock_guard<std::mutex> lock(g_capture_mutex);
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const hipStream_t saved = c->stream;
    c->stream = c->cap_stream;
    c->prof_sink = &G.ev;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    hfe_status st = HFE_OK;
    if (e == hipSuccess)
      for (int i = 0; i < k && st == HFE_OK; ++i) st = iteration();
    hipGraph_t graph = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(c->cap_stream, &graph) : e;
    c->stream = saved;
    c->prof_sink = nullptr;
    if (st) {
      if (graph) hipGraphDestroy(graph);
      return st;
    }
    if (e2 != hipSuccess) return fail(c, HFE_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e2));
    const hipError_t e3 = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
      G.exec = nullptr;
      return fail(c, HFE_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e3));
    }
    G.iters = k;
    G.profiled = c->profiling;
  }
  HIPCHK(c, hipGraphLaunch(G.exec, c->stream));
  return HFE_OK;
}

// Algorithm 1 in displacement coordinates. Result in c->z; returns the exit flag.
// The CG state at the start of a solve at the current residual (rr0, and the
// tails under mean-stress control).
hfe::CgState cg_initial_state(const hfe_ctx* c, double R, double eta_cg, int j_max,
                              double restart_c, int stall) {
  hfe::CgState init;
  std::memset(&init, 0, sizeof(init));
  init.rr = init.rr0 = init.rr_new = c->rr0;
  init.R = R;
  init.eta_cg = eta_cg;
  init.restart_c = restart_c;
  init.rr_ref = c->rr0;
  init.j_ref = 0;
  init.stall = stall;
  // mean-stress control: z_e = 0, g_e = g0_e, y_e = g0_e / N_qp, d_e = -y_e
  init.ne = c->ne;
  init.nqp = (double)c->g.N * c->g.nq;
  for (int m = 0; m < c->ne; ++m) {
    init.comp[m] = c->comp[m];
    init.ge[m] = c->g0e[m];
    init.ye[m] = c->g0e[m] / init.nqp;
    init.de[m] = -init.ye[m];
  }
  hfe::tail_tensor(&init, init.de, init.dU);
  init.jmax = j_max;
  init.flag = hfe::CG_RUN;
  init.trace_cap = kTraceCap;
  return init;
}

hfe_status steihaug(hfe_ctx* c, double R, double eta_cg, int j_max, int prec, double restart_c,
                    int stall, int* flag, CgInfo* info) {
  const long long n = ndof(c);
  const size_t bytes = (size_t)n * sizeof(double);
  const bool mixed = prec == HFE_MIXED;
  *flag = HFE_CG_INTERIOR;
  if (c->rr0 == 0.0) {
    HIPCHK(c, hipMemsetAsync(c->z, 0, bytes, c->stream));
    return HFE_OK;
  }
  if (c->graph_precision != prec) {
    // captured iterations run one precision's kernels and buffers
    destroy_graphs(c);
    c->graph_precision = prec;
  }
  if (mixed) {
    hfe_status st0 = refresh_state32(c);
    if (st0) return st0;
    HIPCHK(c, hipMemsetAsync(c->z, 0, bytes, c->stream));
    HIPCHK(c, hipMemsetAsync(c->z32, 0, (size_t)n * sizeof(float), c->stream));
    HIPCHK(c, hfe::vec_to_f32(n, c->g0, c->g32, c->stream));
    HIPCHK(c, hfe::vec_to_f32(n, c->y0, c->y32, c->stream));
  }
  *c->hcg = cg_initial_state(c, R, eta_cg, j_max, restart_c, stall);
  HIPCHK(c, hipMemcpyAsync(c->cg, c->hcg, sizeof(hfe::CgState), hipMemcpyHostToDevice, c->stream));
  // d0 = -y0 (beta = 0) with <r0, d0> and z.g = 0; in FP64 one kernel also
  // sets z = 0, g = g0 and y = y0
  if (mixed) {
    hfe_status st = direction32(c);
    if (st) return st;
  } else {
    hfe::Reducer r;
    r.partials = c->partials2;
    Prof p(c, "cg_vec");
    HIPCHK(c, hfe::cg_start(n, c->g0, c->y0, c->z, c->gv, c->y, c->d, r, c->stream, &c->nb_dir));
  }
  int restarts = 0;
  int batch = 0;        // batches of this (re)start
  int enq = 0;          // iterations enqueued since the (re)start
  for (;;) {
    // Iterations enqueued after the stop return at entry but still cost
    // their launches, and every host poll costs a round trip. The first
    // batch is the previous solve's iteration count (trust-region solves of
    // one load step are alike), later ones grow 2, 4, 8, 8, ...; a batch of
    // k iterations is replayed from the captured graphs of 8, 4, 2 and 1.
    // A profiled solve polls after every iteration, so no launch of a batch
    // runs after the stop (such launches would bias the per-kernel averages).
    int k = 1;
    if (!c->profiling) {
      k = batch == 0 ? std::min(std::max(c->cg_predict - enq, 1), kCgBatch)
                     : std::min(2 << std::min(batch - 1, 2), kCgBatch);
    }
    hfe_status st = HFE_OK;
    for (int sl = kCgSlots - 1, rem = k; sl >= 0 && st == HFE_OK; --sl)
      while (rem >= (1 << sl) && st == HFE_OK) {
        st = cg_batch(c, sl, 1 << sl);
        rem -= 1 << sl;
      }
    if (st) return st;
    ++batch;
    enq += k;
    HIPCHK(c, hipMemcpyAsync(c->hcg, c->cg, sizeof(hfe::CgState), hipMemcpyDeviceToHost, c->stream));
    st = sync(c);
    if (st) return st;

    const hfe::CgState h = *c->hcg;
    if (!h.done) continue;
    if (h.flag == hfe::CG_NUMERIC) return fail(c, HFE_ENUMERIC, "non-finite curvature in CG");
    if (h.restart) {
      // Powell's test: recompute the true residual at the new iterate and
      // restart along steepest descent (beta = 0)
      restarts += 1;
      if (mixed) {
        st = stiffness32(c, c->z32, c->tmp32, false);
        if (st) return st;
        HIPCHK(c, hfe::vec_add_f32(n, c->tmp32, c->g0, c->g32, c->stream));
        st = green32(c, c->g32, c->y32);
        if (st) return st;
        st = dot32(c, c->y32, c->g32, &c->cg->rr_new);
        if (st) return st;
        HIPCHK(c, hfe::cg_resume(c->cg, c->stream));
        st = direction32(c);
      } else if (c->ne > 0) {
        // with the tails of mean-stress control: K z with z's uniform part,
        // then r = K z + g on both parts, y = L^+ r (nodal) and r_e / N_qp,
        // beta = 0, d_e = -y_e; the resumed state is written from the host
        double Uz[9];
        hfe::tail_tensor(&h, h.ze, Uz);
        st = upload_3x3(c, Uz, c->Udev);
        if (st) return st;
        st = stiffness(c, c->z, c->tmp, false, c->Udev);
        if (st) return st;
        HIPCHK(c, hfe::vec_axpy_to(n, c->tmp, 1.0, c->g0, c->gv, c->stream));
        st = green(c, c->gv, c->y);
        if (st) return st;
        st = dot(c, c->y, c->gv, c->dscal + S_DOT);
        if (st) return st;
        st = sync(c);
        if (st) return st;
        hfe::CgState r = h;
        double rr = c->hscal[S_DOT];
        for (int m = 0; m < c->ne; ++m) {
          r.ge[m] = hfe::tail_pair(c->comp[m], c->hscal + S_TAIL) + c->g0e[m];
          r.ye[m] = r.ge[m] / r.nqp;
          r.de[m] = -r.ye[m];
          rr += r.ge[m] * r.ye[m];
        }
        hfe::tail_tensor(&r, r.de, r.dU);
        r.rr_new = rr;
        r.beta = 0.0;
        r.restart = 0;
        r.done = 0;
        r.flag = hfe::CG_RUN;
        *c->hcg = r;
        HIPCHK(c, hipMemcpyAsync(c->cg, c->hcg, sizeof(hfe::CgState), hipMemcpyHostToDevice,
                                 c->stream));
        st = direction(c);
      } else {
        st = stiffness(c, c->z, c->tmp, false);
        if (st) return st;
        HIPCHK(c, hfe::vec_axpy_to(n, c->tmp, 1.0, c->g0, c->gv, c->stream));
        st = green(c, c->gv, c->y);
        if (st) return st;
        st = dot(c, c->y, c->gv, &c->cg->rr_new);
        if (st) return st;
        HIPCHK(c, hfe::cg_resume(c->cg, c->stream));
        st = direction(c);
      }
      if (st) return st;
      batch = 0;
      enq = h.iters;
      continue;
    }
    for (int m = 0; m < c->ne; ++m) c->ze[m] = h.ze[m];   // the step's tail
    info->iters = h.iters;
    info->restarts = restarts;
    c->cg_predict = std::max(h.iters, 1);
    info->matvecs = h.iters + restarts;
    *flag = h.flag;
    // the step of a mixed-precision solve continues in FP64
    if (mixed) HIPCHK(c, hfe::vec_to_f64(n, c->z32, c->z, c->stream));
    // keep the trace of this solve
    const int nt = std::min(h.ntrace, kTraceCap);
    if (nt > 0) {
      const size_t off = c->cg_trace.size();
      c->cg_trace.resize(off + 2 * (size_t)nt);
      HIPCHK(c, hipMemcpyAsync(c->cg_trace.data() + off, c->trace, 2 * (size_t)nt * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return HFE_OK;
  }
}

hfe_status commit(hfe_ctx* c) {
  hfe::ElemArgs A = elem_args(c);
  A.a_out = c->kh;
  Prof p(c, "commit");
  HIPCHK(c, hfe::launch_commit(A, c->stream));
  return HFE_OK;
}

hfe_status reset_state(hfe_ctx* c) {
  const size_t nod = (size_t)ndof(c) * sizeof(double);
  HIPCHK(c, hipMemsetAsync(c->u, 0, nod, c->stream));
  for (int k = 0; k < 9; ++k) c->E[k] = 0.0;
  {
    hfe_status st = upload_E(c);
    if (st) return st;
  }
  c->R_init = false;
  c->have_state = false;
  c->history_ready = false;
  c->log.clear();
  return HFE_OK;
}

bool materials_ready(const hfe_ctx* c) {
  for (int p = 0; p < c->n_phases; ++p)
    if (!c->mat_set[p]) return false;
  return c->have_micro;
}

hfe_status ensure_history(hfe_ctx* c) {
  if (c->history_ready) return HFE_OK;
  hfe::ElemArgs A = elem_args(c);
  A.a_out = c->kh;
  HIPCHK(c, hfe::launch_init_history(A, c->stream));
  c->history_ready = true;
  return HFE_OK;
}

}  // namespace

extern "C" {

size_t hfe_workspace_bytes(const hfe_grid* grid) {
  std::string why;
  if (!grid_ok(grid, &why)) return 0;
  return make_layout(make_grid(grid)).total;
}

hfe_status hfe_create(const hfe_grid* grid, void* workspace, size_t ws_bytes, void* hip_stream,
                      hfe_ctx** out) {
  if (!out) return HFE_EINVAL;
  *out = nullptr;
  std::string why;
  if (!grid_ok(grid, &why)) return HFE_EINVAL;
  const Grid g = make_grid(grid);
  const Layout L = make_layout(g);
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return HFE_EINVAL;
  if (ws_bytes < L.total) return HFE_ENOMEM;
  hfe_ctx* c = new hfe_ctx();
  c->g = g;
  c->L = L;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;
  c->use_graphs = std::getenv("HFE_NO_GRAPHS") == nullptr;
  if (const char* bs = std::getenv("HFE_BRICK_SHAPE")) {
    const int v = std::atoi(bs);
    if (hfe::hessian_shape_valid(g, v)) c->brick_shape = c->brick_shape32 = v;
  }
  auto D = [&](size_t off) { return (double*)(c->ws + off); };
  c->u = D(L.u); c->z = D(L.z); c->d = D(L.d); c->gv = D(L.g); c->y = D(L.y);
  c->Kd = D(L.Kd); c->w = D(L.w); c->g0 = D(L.g0); c->y0 = D(L.y0);
  c->tmp = D(L.tmp);
  c->a = D(L.a); c->cp = D(L.cp); c->kh = D(L.kh);
  c->sw = c->g.element == HFE_Q1 ? D(L.sw) : nullptr;
  c->sn = c->g.element == HFE_Q1 ? D(L.sn) : nullptr;
  auto F = [&](size_t off) { return (float*)(c->ws + off); };
  c->z32 = F(L.z32); c->d32 = F(L.d32); c->g32 = F(L.g32);
  c->y32 = F(L.y32); c->Kd32 = F(L.Kd32); c->tmp32 = F(L.tmp32);
  c->a32 = F(L.a32);
  c->spec32 = (float2*)(c->ws + L.spec32);
  c->phase = (uint8_t*)(c->ws + L.phase);
  c->soft = (uint8_t*)(c->ws + L.soft);
  c->emask = (uint16_t*)(c->ws + L.emask);
  c->spec = (double2*)(c->ws + L.spec);
  c->partials = D(L.partials);
  c->partials2 = D(L.partials2);
  c->partials3 = D(L.partials3);
  c->Udev = D(L.Udev);
  c->Pudev = D(L.Pudev);
  c->cg = (hfe::CgState*)(c->ws + L.cgstate);
  c->cg_mid = (hfe::CgState*)(c->ws + L.cgmid);
  c->trace = D(L.trace);
  c->Edev = D(L.Edev);
  std::memset(&c->mat, 0, sizeof(c->mat));
  // FFT tables
  std::vector<double2> tw;
  const int M = g.nx / 2;
  c->tabs.off_x = 0;
  twiddles(M, M, tw);
  c->tabs.off_y = (int)tw.size();
  twiddles(g.ny, g.ny, tw);
  c->tabs.off_z = (int)tw.size();
  twiddles(g.nz, g.nz, tw);
  c->tabs.off_post = (int)tw.size();
  twiddles(g.nx, M + 1, tw);
  std::vector<double> st;
  sin2_table(g.nx, M + 1, st);
  sin2_table(g.ny, g.ny, st);
  sin2_table(g.nz, g.nz, st);
  double2* dtw = (double2*)(c->ws + L.tw);
  double* dst = D(L.stab);
  c->tabs.tw = dtw;
  c->tabs.sx = dst;
  c->tabs.sy = dst + (M + 1);
  c->tabs.sz = dst + (M + 1) + g.ny;
  hfe::fft_default_launch(g, &c->tabs.plane_threads, &c->tabs.pencil_cols, &c->tabs.pencil_threads);
  // the same tables rounded to FP32 for the mixed-precision CG
  std::vector<float2> tw32(tw.size());
  for (size_t i = 0; i < tw.size(); ++i) tw32[i] = make_float2((float)tw[i].x, (float)tw[i].y);
  std::vector<float> st32(st.begin(), st.end());
  float2* dtw32 = (float2*)(c->ws + L.tw32);
  float* dst32 = F(L.stab32);
  c->tabs32.tw = dtw32;
  c->tabs32.off_x = c->tabs.off_x;
  c->tabs32.off_y = c->tabs.off_y;
  c->tabs32.off_z = c->tabs.off_z;
  c->tabs32.off_post = c->tabs.off_post;
  c->tabs32.sx = dst32;
  c->tabs32.sy = dst32 + (M + 1);
  c->tabs32.sz = dst32 + (M + 1) + g.ny;
  c->tabs32.plane_threads = c->tabs.plane_threads;
  c->tabs32.pencil_cols = c->tabs.pencil_cols;
  c->tabs32.pencil_threads = c->tabs.pencil_threads;
  hipError_t e = hfe::fft_prepare(g);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->hscal, S_COUNT * sizeof(double),
                      hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->dscal, c->hscal, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->hcg, sizeof(hfe::CgState), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws, 0, L.total, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dtw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dtw32, tw32.data(), tw32.size() * sizeof(float2), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst32, st32.data(), st32.size() * sizeof(float), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    if (c->hscal) hipHostFree(c->hscal);
    if (c->hcg) hipHostFree(c->hcg);
    delete c;
    return HFE_EDEVICE;
  }
  *out = c;
  return HFE_OK;
}

hfe_status hfe_destroy(hfe_ctx* c) {
  if (!c) return HFE_EINVAL;
  hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  for (auto& p : c->pending) {
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  for (auto e : c->pool) hipEventDestroy(e);
  if (c->hscal) hipHostFree(c->hscal);
  if (c->hcg) hipHostFree(c->hcg);
  delete c;
  return HFE_OK;
}

hfe_status hfe_set_microstructure(hfe_ctx* c, const uint8_t* phase, int n_phases) {
  if (!c) return HFE_EINVAL;
  if (!phase) return fail(c, HFE_EINVAL, "phase is NULL");
  if (n_phases < 1 || n_phases > hfe::kMaxPhases) return fail(c, HFE_EINVAL, "n_phases out of range");
  for (long long i = 0; i < c->g.N; ++i)
    if (phase[i] >= n_phases) return fail(c, HFE_EINVAL, "phase id >= n_phases");
  HIPCHK(c, hipMemcpyAsync(c->phase, phase, (size_t)c->g.N, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  destroy_graphs(c);
  c->n_phases = n_phases;
  for (int p = 0; p < hfe::kMaxPhases; ++p) c->mat_set[p] = false;
  std::memset(c->mat.eig, 0, sizeof(c->mat.eig));
  c->have_micro = true;
  return reset_state(c);
}

hfe_status hfe_set_material(hfe_ctx* c, int phase, const hfe_material* m) {
  if (!c) return HFE_EINVAL;
  if (!c->have_micro) return fail(c, HFE_ESTATE, "set the microstructure first");
  if (c->have_state) return fail(c, HFE_ESTATE, "materials are fixed once loading started");
  if (!m || phase < 0 || phase >= c->n_phases) return fail(c, HFE_EINVAL, "bad phase or material");
  if (!(m->E > 0.0) || !(m->nu > -1.0 && m->nu < 0.5)) return fail(c, HFE_EINVAL, "E > 0 and -1 < nu < 1/2 required");
  if (m->kind != HFE_ELASTIC && m->kind != HFE_DAMAGE_ENERGY_NORM && m->kind != HFE_DAMAGE_TENSILE)
    return fail(c, HFE_EINVAL, "unknown material kind");
  if (m->kind != HFE_ELASTIC && !(m->kappa0 > 0.0 && m->kappaf > m->kappa0))
    return fail(c, HFE_EINVAL, "damage needs 0 < kappa0 < kappaf");
  const double E = m->E, nu = m->nu;
  c->mat.lam[phase] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  c->mat.mu[phase] = E / (2.0 * (1.0 + nu));
  c->mat.E[phase] = E;
  c->mat.damage[phase] = m->kind;   // the law: 0 elastic, else the damage kind
  c->mat.k0[phase] = c->mat.damage[phase] ? m->kappa0 : 0.0;
  c->mat.kf[phase] = c->mat.damage[phase] ? m->kappaf : 1.0;
  c->mat_set[phase] = true;
  c->tens = false;
  for (int p = 0; p < c->n_phases; ++p)
    c->tens = c->tens || (c->mat_set[p] && c->mat.damage[p] == HFE_DAMAGE_TENSILE);
  destroy_graphs(c);
  c->history_ready = false;  // kappa0 may have changed: re-initialise before the first step
  return HFE_OK;
}

hfe_status hfe_set_eigenstrain(hfe_ctx* c, int phase, const double eig[9]) {
  if (!c) return HFE_EINVAL;
  if (!c->have_micro) return fail(c, HFE_ESTATE, "set the microstructure first");
  if (!eig || phase < 0 || phase >= c->n_phases) return fail(c, HFE_EINVAL, "bad phase or eigenstrain");
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(eig[k])) return fail(c, HFE_EINVAL, "non-finite eigenstrain");
  const int D = c->g.dim;
  // (xx, yy, zz, xy, xz, yz) of the symmetric part; 2D keeps the in-plane block
  double v[6] = {eig[0], eig[4], eig[8], 0.5 * (eig[1] + eig[3]), 0.5 * (eig[2] + eig[6]),
                 0.5 * (eig[5] + eig[7])};
  if (D == 2) v[2] = v[4] = v[5] = 0.0;
  hfe_status st = sync(c);
  if (st) return st;
  destroy_graphs(c);   // captured kernels hold the material table by value
  for (int k = 0; k < 6; ++k) c->mat.eig[phase][k] = v[k];
  return HFE_OK;
}

hfe_status hfe_set_mean_stress_control(hfe_ctx* c, int free_mask) {
  if (!c) return HFE_EINVAL;
  if (free_mask < 0 || free_mask > 63) return fail(c, HFE_EINVAL, "free_mask has bits 0..5");
  if (free_mask != 0 && c->g.dim != 3)
    return fail(c, HFE_EINVAL, "mean-stress control is implemented for 3D grids");
  hfe_status st = sync(c);
  if (st) return st;
  destroy_graphs(c);   // captured iterations hold the tail buffers (or none)
  c->ne = 0;
  for (int v = 0; v < 6; ++v)
    if (free_mask & (1 << v)) c->comp[c->ne++] = v;
  if (c->have_state) refresh_tails(c);
  return HFE_OK;
}

hfe_status hfe_apply_load_step(hfe_ctx* c, const double dE[9]) {
  if (!c) return HFE_EINVAL;
  if (!dE) return fail(c, HFE_EINVAL, "dE is NULL");
  if (!materials_ready(c)) return fail(c, HFE_ESTATE, "microstructure and every material must be set");
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(dE[k])) return fail(c, HFE_EINVAL, "non-finite dE");
  const int D = c->g.dim;
  double inc[9] = {0};
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) inc[3 * i + j] = dE[3 * i + j];
  hfe_status st = ensure_history(c);
  if (st) return st;
  const double Eold[9] = {c->E[0], c->E[1], c->E[2], c->E[3], c->E[4], c->E[5], c->E[6], c->E[7], c->E[8]};
  for (int k = 0; k < 9; ++k) c->E[k] += inc[k];
  if (!c->R_init) {
    double nrm = 0.0;
    for (int k = 0; k < 9; ++k) nrm += inc[k] * inc[k];
    if (nrm == 0.0) {
      // a load by eigenstrain alone: the scale of the largest phase eigenstrain
      for (int p = 0; p < c->n_phases; ++p) {
        const double* e = c->mat.eig[p];
        const double n2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2] +
                          2.0 * (e[3] * e[3] + e[4] * e[4] + e[5] * e[5]);
        nrm = std::max(nrm, n2);
      }
    }
    const double s = std::sqrt((double)c->g.N * c->g.nq) * std::sqrt(nrm);
    c->R0_default = 10.0 * s;
    c->Rmax_default = 1000.0 * s;
  }
  const bool had_state = c->have_state;
  st = evaluate_state(c);
  if (st) {
    // back to the previous increment: E and, if there was one, the evaluated
    // state (stress, tangent, residual) at it
    const std::string why = c->err;
    for (int k = 0; k < 9; ++k) c->E[k] = Eold[k];
    c->have_state = false;
    if (had_state && evaluate_state(c) != HFE_OK)
      return fail(c, st, why + "; the previous state could not be re-evaluated");
    c->err = why;
    return st;
  }
  c->log.clear();
  return HFE_OK;
}

hfe_status hfe_solve_increment(hfe_ctx* c, const hfe_solver_params* prm, hfe_solve_report* out) {
  if (!c) return HFE_EINVAL;
  if (!c->have_state) return fail(c, HFE_ESTATE, "apply a load step first");
  const auto t0 = std::chrono::steady_clock::now();
  hfe_solver_params p;
  p.eta_eq = 1e-8; p.eta_nr = 1e-8; p.eta_cg = 1e-6; p.eta_up = 0.15;
  p.R0 = 0.0; p.Rmax = 0.0; p.i_nr_max = 50; p.j_cg_max = 2000; p.precision = HFE_FP64;
  p.restart = 0.2; p.cg_stall = 0;
  if (prm) p = *prm;
  if (std::isnan(p.restart)) return fail(c, HFE_EINVAL, "restart constant is NaN");
  if (p.cg_stall < 0) return fail(c, HFE_EINVAL, "cg_stall must be >= 0");
  if (p.precision != HFE_FP64 && p.precision != HFE_MIXED)
    return fail(c, HFE_EINVAL, "precision must be HFE_FP64 or HFE_MIXED");
  if (p.precision == HFE_MIXED && c->g.dim != 3)
    return fail(c, HFE_EINVAL, "HFE_MIXED is implemented for 3D grids");
  if (p.precision == HFE_MIXED && c->ne > 0)
    return fail(c, HFE_EINVAL, "mean-stress control runs in FP64 (HFE_FP64)");
  refresh_tails(c);   // the free components may have changed since the evaluation
  if (!c->R_init) {
    c->R = p.R0 > 0.0 ? p.R0 : c->R0_default;
    c->Rmax = p.Rmax > 0.0 ? p.Rmax : c->Rmax_default;
    c->R_init = true;
  } else if (p.Rmax > 0.0) {
    c->Rmax = p.Rmax;
  }
  hfe_solve_report rep;
  std::memset(&rep, 0, sizeof(rep));
  rep.status = HFE_NOT_CONVERGED;
  c->log.clear();
  c->cg_trace.clear();
  const long long n = ndof(c);
  hfe_status st = HFE_OK;
  bool converged = false;
  if (c->r_eq <= p.eta_eq) {
    converged = true;
  } else {
    for (int it = 0; it < p.i_nr_max && !converged; ++it) {
      rep.newton_iters = it + 1;
      int flag = 0;
      CgInfo info;
      st = steihaug(c, c->R, p.eta_cg, p.j_cg_max, p.precision, p.restart, p.cg_stall, &flag,
                    &info);
      if (st) return st;
      rep.cg_iters += info.iters;
      rep.restarts += info.restarts;
      rep.matvecs += info.matvecs;
      if (flag == HFE_CG_BOUNDARY) rep.boundary_exits++;
      if (flag == HFE_CG_NEGCURV) rep.negcurv_exits++;
      if (flag == HFE_CG_STALL) rep.stall_exits++;
      // trial evaluation at u + z (Algorithm 2: model change, trial stress, FAIEF)
      hfe::ElemArgs A = elem_args(c);
      A.v = c->z;
      double Pu[9] = {0};
      if (c->ne > 0) {
        // the step's uniform part moves the free macroscopic strain
        hfe::CgState t;
        t.ne = c->ne;
        for (int m = 0; m < c->ne; ++m) t.comp[m] = c->comp[m];
        hfe::tail_tensor(&t, c->ze, Pu);
        st = upload_3x3(c, Pu, c->Pudev);
        if (st) return st;
        A.Pu = c->Pudev;
      }
      int nb = 0;
      {
        Prof pr(c, "trial");
        HIPCHK(c, hfe::launch_trial(A, c->stream, &nb));
      }
      st = finish(c, hfe::FIN_OUT, nb, hfe::TRI_NV, c->dscal + S_TRI);
      if (st) return st;
      st = sync(c);
      if (st) return st;
      double h[hfe::TRI_NV];
      for (int k = 0; k < hfe::TRI_NV; ++k) h[k] = c->hscal[S_TRI + k];
      const double sp = h[hfe::TRI_SP], pbp = h[hfe::TRI_PBP], stp = h[hfe::TRI_STP];
      const double dm = sp + 0.5 * pbp;
      const double dW = 0.5 * (sp + stp);
      double rho = -INFINITY;
      if (dm < 0.0 && std::isfinite(dm) && std::isfinite(dW)) rho = dW / dm;
      if (!std::isfinite(rho)) rho = -INFINITY;
      hfe_newton_record rec;
      rec.flag = flag;
      rec.cg_iters = info.iters;
      rec.restarts = info.restarts;
      rec.dm = dm;
      rec.dW = dW;
      rec.rho = rho;
      rec.R_before = c->R;
      rec.p_norm = std::sqrt(std::max(h[hfe::TRI_PP], 0.0));
      rec.accepted = 0;
      rep.rho_last = rho;
      const bool on_boundary = flag == HFE_CG_BOUNDARY || flag == HFE_CG_NEGCURV;
      if (rho < 0.25) c->R = 0.25 * c->R;
      else if (rho > 0.75 && on_boundary) c->R = std::min(2.0 * c->R, c->Rmax);
      if (rho > p.eta_up) {
        rec.accepted = 1;
        // the state moves to u + z; its stress, tangent scalars and residual
        // (g0 = D^T sigma, y0 = L^+ g0) are evaluated there in FP64, in
        // place, so captured CG graphs stay valid
        HIPCHK(c, hfe::vec_axpy(n, 1.0, c->z, c->u, c->stream));
        if (c->ne > 0) {
          for (int k = 0; k < 9; ++k) c->E[k] += Pu[k];
          st = evaluate_state(c);
        } else {
          st = evaluate_residual(c);
        }
        if (st) return st;
        const double pp = h[hfe::TRI_PP], hh = h[hfe::TRI_HH];
        const double r_nr = hh > 0.0 ? std::sqrt(pp) / std::sqrt(hh) : 0.0;
        rep.r_nr = r_nr;
        if (!on_boundary && (c->r_eq <= p.eta_eq || r_nr <= p.eta_nr)) converged = true;
      } else {
        rep.rejected++;
      }
      c->log.push_back(rec);
    }
  }
  if (converged) {
    st = commit(c);
    if (st) return st;
    rep.status = HFE_CONVERGED;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->profiling) prof_drain(c);
  rep.r_eq = c->r_eq;
  rep.R = c->R;
  rep.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = rep;
  return HFE_OK;
}

size_t hfe_lbfgs_workspace_bytes(const hfe_grid* grid, int m) {
  std::string why;
  if (!grid_ok(grid, &why) || m < 1 || m > HFE_LBFGS_MAX_M) return 0;
  const Grid g = make_grid(grid);
  const size_t vec = align_up((size_t)g.dim * g.N * sizeof(double));
  return (3 * ((size_t)m + 1) + 4) * vec;
}

// L-BFGS on the approximate energy increment (the quasi-Newton use of eq.
// incr_energy_func that Sec. 2.2 proposes); the steps are those documented
// with hfe_solve_increment_lbfgs. The strain-space vectors are held in
// displacement coordinates: a strain D x is stored as x, and since
// L = D^T D, (D x):(D y) = x . L y. The gradient G sigma is D y0 with
// L y0 = g0 = D^T sigma; a pair keeps s (du), y (dy0) and L y (dg0), and the
// first loop keeps q both as qd and as L qd, so that every inner product is a
// plain dot of two stored vectors and no operator is applied.
hfe_status hfe_solve_increment_lbfgs(hfe_ctx* c, const hfe_lbfgs_params* prm, void* workspace,
                                     size_t ws_bytes, hfe_lbfgs_report* out) {
  if (!c) return HFE_EINVAL;
  if (!c->have_state) return fail(c, HFE_ESTATE, "apply a load step first");
  if (c->ne > 0) return fail(c, HFE_EINVAL, "the L-BFGS increment runs under strain control");
  const auto t0 = std::chrono::steady_clock::now();
  hfe_lbfgs_params p;
  p.eta_eq = 1e-8; p.eta_nr = 1e-8; p.max_iters = 500; p.m = 5; p.c1 = 1e-4;
  p.max_backtracks = 30;
  if (prm) p = *prm;
  if (p.m < 1 || p.m > HFE_LBFGS_MAX_M || p.max_iters < 0 || p.max_backtracks < 0 ||
      !(p.c1 > 0.0 && p.c1 < 1.0))
    return fail(c, HFE_EINVAL, "bad L-BFGS parameters");
  const long long n = ndof(c);
  const size_t vec = align_up((size_t)n * sizeof(double));
  if (!workspace || ws_bytes < (3 * ((size_t)p.m + 1) + 4) * vec || ((uintptr_t)workspace & 255))
    return fail(c, HFE_EINVAL, "L-BFGS workspace too small or misaligned");
  char* w = (char*)workspace;
  auto V = [&](size_t k) { return (double*)(w + k * vec); };
  const int m = p.m;
  // m + 1 pair slots (a new pair is formed before the oldest one is dropped):
  // slot k holds su (du), sy (dy0), sg (dg0); then qd, qf, rd, v
  const int ns = m + 1;
  double* qd = V(3 * ns);
  double* qf = V(3 * ns + 1);
  double* rd = V(3 * ns + 2);
  double* v = V(3 * ns + 3);
  std::vector<int> order;            // slots of the kept pairs, oldest first
  std::vector<double> rho(ns, 0.0), yy(ns, 0.0);
  double lpm = 0.0;                  // max over phases of lambda + 2 mu
  for (int ph = 0; ph < c->n_phases; ++ph) lpm = std::max(lpm, c->mat.lam[ph] + 2.0 * c->mat.mu[ph]);
  const double gamma0 = 1.0 / lpm;
  // host value of x . y
  auto dotv = [&](const double* x, const double* y, double* res) -> hfe_status {
    hfe_status st = dot(c, x, y, c->dscal + S_DOT);
    if (st) return st;
    st = sync(c);
    if (st) return st;
    *res = c->hscal[S_DOT];
    return HFE_OK;
  };
  hfe_lbfgs_report rep;
  std::memset(&rep, 0, sizeof(rep));
  rep.status = HFE_NOT_CONVERGED;
  hfe_status st = HFE_OK;
  bool converged = c->r_eq <= p.eta_eq;
  for (int it = 0; it < p.max_iters && !converged; ++it) {
    rep.iters = it + 1;
    // two-loop recursion: rd = H_k (G sigma), displacement coordinates
    double gamma = gamma0;
    if (!order.empty()) gamma = 1.0 / (rho[order.back()] * yy[order.back()]);
    HIPCHK(c, hipMemcpyAsync(qd, c->y0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(qf, c->g0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    std::vector<double> alpha(ns, 0.0);
    for (int k = (int)order.size() - 1; k >= 0; --k) {
      const int j = order[k];
      double sq;
      st = dotv(V(3 * j), qf, &sq);
      if (st) return st;
      alpha[j] = rho[j] * sq;
      HIPCHK(c, hfe::vec_axpy(n, -alpha[j], V(3 * j + 1), qd, c->stream));
      HIPCHK(c, hfe::vec_axpy(n, -alpha[j], V(3 * j + 2), qf, c->stream));
    }
    HIPCHK(c, hfe::vec_lincomb(n, gamma, qd, 0.0, qd, rd, c->stream));
    for (size_t k = 0; k < order.size(); ++k) {
      const int j = order[k];
      double yr;
      st = dotv(V(3 * j + 2), rd, &yr);
      if (st) return st;
      const double b = rho[j] * yr;
      HIPCHK(c, hfe::vec_axpy(n, alpha[j] - b, V(3 * j), rd, c->stream));
    }
    // p = -rd; sigma:p = g0 . p
    double sp;
    st = dotv(c->g0, rd, &sp);
    if (st) return st;
    sp = -sp;
    if (!(sp < 0.0)) {
      order.clear();
      rep.resets++;
      HIPCHK(c, hfe::vec_lincomb(n, gamma0, c->y0, 0.0, c->y0, rd, c->stream));
      st = dotv(c->g0, rd, &sp);
      if (st) return st;
      sp = -sp;
    }
    // backtracking on the approximate energy increment
    double a = 1.0;
    bool found = false;
    double h[hfe::TRI_NV];
    for (int bt = 0; bt <= p.max_backtracks; ++bt) {
      HIPCHK(c, hfe::vec_lincomb(n, -a, rd, 0.0, rd, v, c->stream));
      hfe::ElemArgs A = elem_args(c);
      A.v = v;
      int nb = 0;
      {
        Prof pr(c, "trial");
        HIPCHK(c, hfe::launch_trial(A, c->stream, &nb));
      }
      st = finish(c, hfe::FIN_OUT, nb, hfe::TRI_NV, c->dscal + S_TRI);
      if (st) return st;
      st = sync(c);
      if (st) return st;
      rep.trials++;
      for (int k = 0; k < hfe::TRI_NV; ++k) h[k] = c->hscal[S_TRI + k];
      const double dW = 0.5 * (h[hfe::TRI_SP] + h[hfe::TRI_STP]);
      if (dW <= p.c1 * a * sp) {
        found = true;
        break;
      }
      a *= 0.5;
    }
    if (!found) break;
    // accept u + v; a free slot gets s = v and the old y0, g0
    int j = 0;
    while (std::find(order.begin(), order.end(), j) != order.end()) ++j;
    HIPCHK(c, hipMemcpyAsync(V(3 * j), v, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(V(3 * j + 1), c->y0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(V(3 * j + 2), c->g0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hfe::vec_axpy(n, 1.0, v, c->u, c->stream));
    st = evaluate_residual(c);
    if (st) return st;
    HIPCHK(c, hfe::vec_lincomb(n, 1.0, c->y0, -1.0, V(3 * j + 1), V(3 * j + 1), c->stream));
    HIPCHK(c, hfe::vec_lincomb(n, 1.0, c->g0, -1.0, V(3 * j + 2), V(3 * j + 2), c->stream));
    double sy, yyj;
    st = dotv(V(3 * j), V(3 * j + 2), &sy);
    if (st) return st;
    st = dotv(V(3 * j + 1), V(3 * j + 2), &yyj);
    if (st) return st;
    const double ss = h[hfe::TRI_PP];        // |D v|^2 over the points
    if (sy > 1e-12 * std::sqrt(ss * yyj)) {
      rho[j] = 1.0 / sy;
      yy[j] = yyj;
      order.push_back(j);
      if ((int)order.size() > m) order.erase(order.begin());
    } else {
      rep.pairs_skipped++;
    }
    const double hh = h[hfe::TRI_HH];
    const double r_nr = hh > 0.0 ? std::sqrt(ss) / std::sqrt(hh) : 0.0;
    rep.r_nr = r_nr;
    if (c->r_eq <= p.eta_eq || r_nr <= p.eta_nr) converged = true;
  }
  if (converged) {
    st = commit(c);
    if (st) return st;
    rep.status = HFE_CONVERGED;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->profiling) prof_drain(c);
  rep.r_eq = c->r_eq;
  rep.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = rep;
  return HFE_OK;
}

hfe_status hfe_solve_batch(hfe_ctx* const* ctxs, int n, const hfe_solver_params* params,
                           hfe_solve_report* reports) {
  if (!ctxs || !reports || n < 1) return HFE_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return HFE_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return HFE_EINVAL;
  }
  std::vector<hfe_status> st(n, HFE_OK);
  std::vector<std::thread> pool;
  pool.reserve(n > 1 ? n - 1 : 0);
  for (int i = 1; i < n; ++i)
    pool.emplace_back([&, i]() { st[i] = hfe_solve_increment(ctxs[i], params, &reports[i]); });
  st[0] = hfe_solve_increment(ctxs[0], params, &reports[0]);
  for (auto& t : pool) t.join();
  for (int i = 0; i < n; ++i)
    if (st[i] != HFE_OK) return st[i];
  return HFE_OK;
}

hfe_status hfe_effective_stiffness(hfe_ctx* const* ctxs, double strain,
                                   const hfe_solver_params* params, double C[36],
                                   hfe_solve_report* reports) {
  if (!ctxs || !C || !(strain > 0.0) || !std::isfinite(strain)) return HFE_EINVAL;
  for (int i = 0; i < 6; ++i) {
    if (!ctxs[i]) return HFE_EINVAL;
    if (ctxs[i]->g.dim != 3 || ctxs[i]->g.nx != ctxs[0]->g.nx || ctxs[i]->g.ny != ctxs[0]->g.ny ||
        ctxs[i]->g.nz != ctxs[0]->g.nz)
      return fail(ctxs[i], HFE_EINVAL, "the six contexts need one 3D grid");
  }
  // Voigt order xx, yy, zz, yz, xz, xy; index pairs of the 3x3 tensor
  static const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
  double before[6][9];
  for (int J = 0; J < 6; ++J) {
    hfe_ctx* c = ctxs[J];
    double dE[9] = {0};
    const double e = vi[J] == vj[J] ? strain : 0.5 * strain;
    dE[3 * vi[J] + vj[J]] = e;
    dE[3 * vj[J] + vi[J]] = e;
    if (c->have_state) {
      hfe_status st = hfe_homogenized_stress(c, before[J]);
      if (st) return st;
    } else {
      for (int k = 0; k < 9; ++k) before[J][k] = 0.0;   // a fresh cell is stress free
    }
    hfe_status st = hfe_apply_load_step(c, dE);
    if (st) return st;
  }
  hfe_solve_report rep[6];
  hfe_status st = hfe_solve_batch(ctxs, 6, params, rep);
  if (st) return st;
  for (int J = 0; J < 6; ++J) {
    double after[9];
    st = hfe_homogenized_stress(ctxs[J], after);
    if (st) return st;
    for (int I = 0; I < 6; ++I) {
      const int k = 3 * vi[I] + vj[I];
      C[6 * I + J] = (after[k] - before[J][k]) / strain;
    }
    if (reports) reports[J] = rep[J];
  }
  return HFE_OK;
}

hfe_status hfe_residual(const hfe_ctx* cc, double* out) {
  hfe_ctx* c = const_cast<hfe_ctx*>(cc);
  if (!c || !out) return HFE_EINVAL;
  if (!c->have_state) return fail(c, HFE_ESTATE, "no evaluated state");
  *out = c->r_eq;
  return HFE_OK;
}

hfe_status hfe_homogenized_stress(const hfe_ctx* cc, double out[9]) {
  hfe_ctx* c = const_cast<hfe_ctx*>(cc);
  if (!c || !out) return HFE_EINVAL;
  if (!c->have_state) return fail(c, HFE_ESTATE, "no evaluated state");
  const double inv = 1.0 / ((double)c->g.N * c->g.nq);
  const double* s = c->sigma_sum;
  // (xx, yy, zz, xy, xz, yz) -> 3x3
  out[0] = s[0] * inv; out[4] = s[1] * inv; out[8] = s[2] * inv;
  out[1] = out[3] = s[3] * inv;
  out[2] = out[6] = s[4] * inv;
  out[5] = out[7] = s[5] * inv;
  return HFE_OK;
}

hfe_status hfe_get_field(const hfe_ctx* cc, int which, double* host_out, size_t n) {
  hfe_ctx* c = const_cast<hfe_ctx*>(cc);
  if (!c || !host_out) return HFE_EINVAL;
  if (!c->have_micro) return fail(c, HFE_ESTATE, "no microstructure");
  const Grid& g = c->g;
  size_t need = 0;
  switch (which) {
    case HFE_FIELD_U: need = (size_t)g.dim * g.N; break;
    case HFE_FIELD_GRAD: case HFE_FIELD_STRESS: need = (size_t)g.N * g.nq * g.dim * g.dim; break;
    case HFE_FIELD_DAMAGE: case HFE_FIELD_KAPPA: case HFE_FIELD_SOFTENING:
      need = (size_t)g.N * g.nq;
      break;
    default: return fail(c, HFE_EINVAL, "unknown field");
  }
  if (n < need) return fail(c, HFE_EINVAL, "output buffer too small");
  if (which == HFE_FIELD_SOFTENING) {
    if (!c->have_state) return fail(c, HFE_ESTATE, "no evaluated state");
    if (g.element == HFE_Q1) {
      // the element masks: bit q set iff c' != 0 at point q
      std::vector<uint8_t> m((size_t)g.N);
      HIPCHK(c, hipMemcpyAsync(m.data(), c->soft, (size_t)g.N, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      for (long long e = 0; e < g.N; ++e)
        for (int q = 0; q < g.nq; ++q) host_out[e * g.nq + q] = (m[e] >> q) & 1 ? 1.0 : 0.0;
    } else {
      std::vector<double> cp((size_t)g.nq * g.N);
      HIPCHK(c, hipMemcpyAsync(cp.data(), c->cp, cp.size() * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      for (long long e = 0; e < g.N; ++e)
        for (int q = 0; q < g.nq; ++q) host_out[e * g.nq + q] = cp[(size_t)q * g.N + e] != 0.0 ? 1.0 : 0.0;
    }
    return HFE_OK;
  }
  if (which == HFE_FIELD_U) {
    HIPCHK(c, hipMemcpyAsync(host_out, c->u, need * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HFE_OK;
  }
  hfe_status st = ensure_history(c);
  if (st) return st;
  double* tmp = nullptr;
  HIPCHK(c, hipMalloc((void**)&tmp, need * sizeof(double)));
  hfe::ElemArgs A = elem_args(c);
  hipError_t e = hfe::launch_fields(A, which == HFE_FIELD_GRAD ? tmp : nullptr,
                                    which == HFE_FIELD_STRESS ? tmp : nullptr,
                                    which == HFE_FIELD_DAMAGE ? tmp : nullptr,
                                    which == HFE_FIELD_KAPPA ? tmp : nullptr, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(host_out, tmp, need * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(tmp);
  if (e != hipSuccess) return fail(c, HFE_EDEVICE, std::string("get_field: ") + hipGetErrorString(e));
  return HFE_OK;
}

hfe_status hfe_get_newton_log(const hfe_ctx* c, hfe_newton_record* out, int max, int* count) {
  if (!c || !count || (max > 0 && !out)) return HFE_EINVAL;
  const int n = std::min<int>(max, (int)c->log.size());
  for (int i = 0; i < n; ++i) out[i] = c->log[i];
  *count = n;
  return HFE_OK;
}

hfe_status hfe_get_cg_trace(const hfe_ctx* c, double* out, int max, int* count) {
  if (!c || !count || (max > 0 && !out)) return HFE_EINVAL;
  const int n = std::min<int>(max, (int)(c->cg_trace.size() / 2));
  for (int i = 0; i < 2 * n; ++i) out[i] = c->cg_trace[i];
  *count = n;
  return HFE_OK;
}

hfe_status hfe_get_state(const hfe_ctx* cc, double* u, double* kappa_hist, double E[9],
                         double radius[2]) {
  hfe_ctx* c = const_cast<hfe_ctx*>(cc);
  if (!c || !u || !kappa_hist || !E || !radius) return HFE_EINVAL;
  if (!c->have_micro) return fail(c, HFE_ESTATE, "no microstructure");
  hfe_status st = ensure_history(c);
  if (st) return st;
  const long long N = c->g.N;
  const int nq = c->g.nq;
  std::vector<double> kh((size_t)nq * N);
  HIPCHK(c, hipMemcpyAsync(u, c->u, (size_t)ndof(c) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(kh.data(), c->kh, kh.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (long long e = 0; e < N; ++e)
    for (int q = 0; q < nq; ++q) kappa_hist[e * nq + q] = kh[(size_t)q * N + e];
  for (int k = 0; k < 9; ++k) E[k] = c->E[k];
  radius[0] = c->R_init ? c->R : 0.0;
  radius[1] = c->R_init ? c->Rmax : 0.0;
  return HFE_OK;
}

hfe_status hfe_set_state(hfe_ctx* c, const double* u, const double* kappa_hist, const double E[9],
                         const double radius[2]) {
  if (!c || !u || !kappa_hist || !E || !radius) return HFE_EINVAL;
  if (!materials_ready(c)) return fail(c, HFE_ESTATE, "microstructure and every material must be set");
  const long long N = c->g.N;
  const int nq = c->g.nq;
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(E[k])) return fail(c, HFE_EINVAL, "non-finite E");
  std::vector<double> kh((size_t)nq * N);
  for (long long e = 0; e < N; ++e)
    for (int q = 0; q < nq; ++q) {
      const double v = kappa_hist[e * nq + q];
      if (!(v >= 0.0) || !std::isfinite(v)) return fail(c, HFE_EINVAL, "kappa_hist must be finite and >= 0");
      kh[(size_t)q * N + e] = v;
    }
  HIPCHK(c, hipMemcpyAsync(c->u, u, (size_t)ndof(c) * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->kh, kh.data(), kh.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->history_ready = true;
  const int D = c->g.dim;
  for (int k = 0; k < 9; ++k) c->E[k] = 0.0;
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) c->E[3 * i + j] = E[3 * i + j];
  if (radius[0] > 0.0) {
    c->R = radius[0];
    c->Rmax = radius[1] > 0.0 ? radius[1] : radius[0];
    c->R_init = true;
  } else {
    c->R_init = false;
  }
  c->log.clear();
  c->cg_trace.clear();
  return evaluate_state(c);
}

hfe_status hfe_set_displacement(hfe_ctx* c, const double* host_u) {
  if (!c || !host_u) return HFE_EINVAL;
  if (!materials_ready(c)) return fail(c, HFE_ESTATE, "microstructure and every material must be set");
  for (long long i = 0; i < ndof(c); ++i)
    if (!std::isfinite(host_u[i])) return fail(c, HFE_EINVAL, "non-finite displacement");
  hfe_status st = ensure_history(c);
  if (st) return st;
  HIPCHK(c, hipMemcpyAsync(c->u, host_u, (size_t)ndof(c) * sizeof(double), hipMemcpyHostToDevice, c->stream));
  return evaluate_state(c);
}

hfe_status hfe_apply_projected_hessian(hfe_ctx* c, const double* in, double* out, double dots[2]) {
  if (!c || !in || !out || in == out) return HFE_EINVAL;
  if (!c->have_state) return fail(c, HFE_ESTATE, "no evaluated state");
  hfe_status st = stiffness(c, in, c->Kd, false);
  if (st) return st;
  st = green(c, c->Kd, out);
  if (st) return st;
  if (dots) {
    st = sync(c);
    if (st) return st;
    dots[0] = c->hscal[S_HES];
    dots[1] = c->hscal[S_HES + 1];
  }
  return HFE_OK;
}

hfe_status hfe_apply_projected_hessian_f32(hfe_ctx* c, const float* in, float* out,
                                           double dots[2]) {
  if (!c || !in || !out || in == out) return HFE_EINVAL;
  if (c->g.dim != 3) return fail(c, HFE_EINVAL, "the FP32 operator is implemented for 3D grids");
  if (!c->have_state) return fail(c, HFE_ESTATE, "no evaluated state");
  hfe_status st = refresh_state32(c);
  if (st) return st;
  st = stiffness32(c, in, c->Kd32, false);
  if (st) return st;
  st = green32(c, c->Kd32, out);
  if (st) return st;
  if (dots) {
    st = sync(c);
    if (st) return st;
    dots[0] = c->hscal[S_HES];
    dots[1] = c->hscal[S_HES + 1];
  }
  return HFE_OK;
}

hfe_status hfe_get_tuning(const hfe_ctx* c, hfe_tuning* out) {
  if (!c || !out) return HFE_EINVAL;
  out->plane_threads = c->tabs.plane_threads;
  out->pencil_cols = c->tabs.pencil_cols;
  out->pencil_threads = c->tabs.pencil_threads;
  out->brick_shape = c->brick_shape;
  out->plane_threads32 = c->tabs32.plane_threads;
  out->pencil_cols32 = c->tabs32.pencil_cols;
  out->pencil_threads32 = c->tabs32.pencil_threads;
  out->brick_shape32 = c->brick_shape32;
  return HFE_OK;
}

hfe_status hfe_set_tuning(hfe_ctx* c, const hfe_tuning* in) {
  if (!c || !in) return HFE_EINVAL;
  if (!hfe::fft_launch_valid(c->g, in->plane_threads, in->pencil_cols, in->pencil_threads, 8) ||
      !hfe::fft_launch_valid(c->g, in->plane_threads32, in->pencil_cols32, in->pencil_threads32, 4))
    return fail(c, HFE_EINVAL, "an FFT launch shape does not fit this grid");
  if ((c->g.dim == 3 && (!hfe::hessian_shape_valid(c->g, in->brick_shape) ||
                         !hfe::hessian_shape_valid(c->g, in->brick_shape32))) ||
      (c->g.dim == 2 && (in->brick_shape < 0 || in->brick_shape >= hfe::kHessianShapes ||
                         in->brick_shape32 < 0 || in->brick_shape32 >= hfe::kHessianShapes)))
    return fail(c, HFE_EINVAL, "brick_shape is not a Hessian shape of this grid");
  hfe_status st = sync(c);
  if (st) return st;
  destroy_graphs(c);
  c->tabs.plane_threads = in->plane_threads;
  c->tabs.pencil_cols = in->pencil_cols;
  c->tabs.pencil_threads = in->pencil_threads;
  c->brick_shape = in->brick_shape;
  c->tabs32.plane_threads = in->plane_threads32;
  c->tabs32.pencil_cols = in->pencil_cols32;
  c->tabs32.pencil_threads = in->pencil_threads32;
  c->brick_shape32 = in->brick_shape32;
  return HFE_OK;
}

// A CG solve started only to time its iterations, at the current state: a
// radius and tolerance that never stop it (a negative curvature still can),
// the reset constant of the defaults. The next solve starts its own.
hfe_status cg_probe_start(hfe_ctx* c) {
  *c->hcg = cg_initial_state(c, 1e150, 0.0, 1 << 30, 0.2, 0);
  HIPCHK(c, hipMemcpyAsync(c->cg, c->hcg, sizeof(hfe::CgState), hipMemcpyHostToDevice, c->stream));
  hfe::Reducer r;
  r.partials = c->partials2;
  HIPCHK(c, hfe::cg_start(ndof(c), c->g0, c->y0, c->z, c->gv, c->y, c->d, r, c->stream, &c->nb_dir));
  return HFE_OK;
}

// Whether the probe solve was still running (its timed iterations all did
// their work).
bool cg_probe_running(hfe_ctx* c) {
  int done = 1;
  if (hipMemcpyAsync(&c->hcg->done, &c->cg->done, sizeof(int), hipMemcpyDeviceToHost,
                     c->stream) != hipSuccess)
    return false;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return false;
  done = c->hcg->done;
  return done == 0;
}

hfe_status hfe_autotune(hfe_ctx* c, hfe_tuning* out) {
  if (!c) return HFE_EINVAL;
  if (c->profiling) return fail(c, HFE_ESTATE, "switch profiling off before tuning");
  hfe_status st = sync(c);
  if (st) return st;
  destroy_graphs(c);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(c, HFE_EDEVICE, "hipEventCreate");
  }
  constexpr int kReps = 4, kTrials = 3;
  // best over kTrials of the average of kReps calls, after one untimed call;
  // +inf on failure
  auto time_us = [&](auto&& call) -> double {
    if (call() != HFE_OK) return INFINITY;
    double best = INFINITY;
    for (int t = 0; t < kTrials; ++t) {
      if (hipEventRecord(e0, c->stream) != hipSuccess) return INFINITY;
      for (int r = 0; r < kReps; ++r)
        if (call() != HFE_OK) return INFINITY;
      if (hipEventRecord(e1, c->stream) != hipSuccess) return INFINITY;
      if (hipEventSynchronize(e1) != hipSuccess) return INFINITY;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return INFINITY;
      best = std::min(best, 1e3 * ms / kReps);
    }
    return best;
  };
  // a candidate replaces the current choice only if it is clearly faster, so
  // that timing noise does not flip the choice between runs; the default
  // shape is timed first
  constexpr double kMargin = 0.97;
  int dp = 0, dc = 0, dt = 0;
  hfe::fft_default_launch(c->g, &dp, &dc, &dt);
  const int planes[] = {dp, 256, 512, 1024};
  const int pencils[][2] = {{dc, dt}, {4, 64}, {4, 128}, {8, 64}, {8, 128}, {8, 256}, {16, 128},
                            {16, 256}, {32, 256}};
  const bool q1 = c->g.dim == 3;
  // The FP64 shapes of a 3D cell with a state are timed on the CG iteration
  // itself (the Hessian and the fused passes, whose best shapes differ from
  // those of the plain Green's operator), each from a fresh probe solve. If
  // a probe stops (negative curvature) the FP64 shapes are timed again on
  // the Green's operator.
  bool iter_timing = q1 && c->have_state && c->rr0 > 0.0;
  for (int prec = 0; prec < (q1 ? 2 : 1); ++prec) {
    const size_t rb = prec ? 4 : 8;
    double best = INFINITY;
    int bp = 0, bc = 0, bt = 0;
    bool stopped = false;
    for (int pt : planes)
      for (const auto& pc : pencils) {
        if (!hfe::fft_launch_valid(c->g, pt, pc[0], pc[1], rb)) continue;
        double t;
        if (prec == 0) {
          c->tabs.plane_threads = pt;
          c->tabs.pencil_cols = pc[0];
          c->tabs.pencil_threads = pc[1];
          if (iter_timing) {
            t = cg_probe_start(c) == HFE_OK ? time_us([&]() { return cg_iteration(c); })
                                            : INFINITY;
            if (!cg_probe_running(c)) stopped = true;
          } else {
            t = time_us([&]() { return green(c, c->g0, c->w); });
          }
        } else {
          c->tabs32.plane_threads = pt;
          c->tabs32.pencil_cols = pc[0];
          c->tabs32.pencil_threads = pc[1];
          t = time_us([&]() { return green32(c, c->Kd32, c->tmp32); });
        }
        if (t < kMargin * best) {
          best = t;
          bp = pt;
          bc = pc[0];
          bt = pc[1];
        }
      }
    if (prec == 0 && iter_timing && stopped) {
      iter_timing = false;
      --prec;            // the FP64 shapes again, on the Green's operator
      continue;
    }
    if (!(best < INFINITY)) {
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      return fail(c, HFE_EDEVICE, "autotune: no FFT launch shape ran");
    }
    hfe::FftTablesT<double>* t64 = &c->tabs;
    if (prec == 0) {
      t64->plane_threads = bp;
      t64->pencil_cols = bc;
      t64->pencil_threads = bt;
    } else {
      c->tabs32.plane_threads = bp;
      c->tabs32.pencil_cols = bc;
      c->tabs32.pencil_threads = bt;
    }
  }
  if (q1 && c->have_state) {
    st = refresh_state32(c);
    if (st == HFE_OK) {
      double best = INFINITY, best32 = INFINITY;
      int bs = 0, bs32 = 0;
      for (int shape = 0; shape < hfe::kHessianShapes; ++shape) {
        if (!hfe::hessian_shape_valid(c->g, shape)) continue;
        c->brick_shape = c->brick_shape32 = shape;
        {
          const double t = time_us([&]() { return stiffness(c, c->g0, c->Kd, false); });
          if (t < kMargin * best) { best = t; bs = shape; }
        }
        const double t32 = time_us([&]() { return stiffness32(c, c->Kd32, c->tmp32, false); });
        if (t32 < kMargin * best32) { best32 = t32; bs32 = shape; }
      }
      c->brick_shape = bs;
      c->brick_shape32 = bs32;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  st = sync(c);
  if (st) return st;
  return out ? hfe_get_tuning(c, out) : HFE_OK;
}

hfe_status hfe_apply_stiffness(hfe_ctx* c, const double* in, double* out) {
  if (!c || !in || !out || in == out) return HFE_EINVAL;
  if (!c->have_state) return fail(c, HFE_ESTATE, "no evaluated state");
  return stiffness(c, in, out, false);
}

hfe_status hfe_apply_green(hfe_ctx* c, const double* in, double* out) {
  if (!c || !in || !out) return HFE_EINVAL;
  return green(c, in, out);
}

hfe_status hfe_fft_forward(hfe_ctx* c, const double* in, double* out_spec) {
  if (!c || !in || !out_spec) return HFE_EINVAL;
  HIPCHK(c, hfe::fft_forward(c->g, c->tabs, in, c->spec, c->stream));
  const size_t bytes = (size_t)c->g.dim * c->g.nz * c->g.ny * (c->g.nx / 2 + 1) * sizeof(double2);
  HIPCHK(c, hipMemcpyAsync(out_spec, c->spec, bytes, hipMemcpyDeviceToDevice, c->stream));
  return HFE_OK;
}

hfe_status hfe_fft_inverse(hfe_ctx* c, const double* in_spec, double* out) {
  if (!c || !in_spec || !out) return HFE_EINVAL;
  const size_t bytes = (size_t)c->g.dim * c->g.nz * c->g.ny * (c->g.nx / 2 + 1) * sizeof(double2);
  HIPCHK(c, hipMemcpyAsync(c->spec, in_spec, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hfe::fft_inverse(c->g, c->tabs, c->spec, out, c->stream));
  return HFE_OK;
}

hfe_status hfe_set_profiling(hfe_ctx* c, int on) {
  if (!c) return HFE_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_drain(c);
  c->profiling = on != 0;
  for (size_t i = 0; i < c->kcount.size(); ++i) {
    c->kcount[i] = 0;
    c->kms[i] = 0.0;
  }
  c->prof_soft_sum = 0.0;
  c->prof_soft_n = 0;
  return HFE_OK;
}

hfe_status hfe_soft_points(hfe_ctx* c, double* current, double* mean_per_hessian) {
  if (!c) return HFE_EINVAL;
  if (current) *current = c->n_soft;
  if (mean_per_hessian)
    *mean_per_hessian = c->prof_soft_n ? c->prof_soft_sum / (double)c->prof_soft_n : 0.0;
  return HFE_OK;
}

hfe_status hfe_kernel_stats(hfe_ctx* c, const char** names, int* counts, double* total_ms, int max,
                            int* n_kernels) {
  if (!c || !n_kernels) return HFE_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_drain(c);
  const int n = std::min<int>(max, (int)c->knames.size());
  for (int i = 0; i < n; ++i) {
    if (names) names[i] = c->knames[i].c_str();
    if (counts) counts[i] = c->kcount[i];
    if (total_ms) total_ms[i] = c->kms[i];
  }
  *n_kernels = n;
  return HFE_OK;
}

const char* hfe_last_error(const hfe_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

}  // extern "C"
