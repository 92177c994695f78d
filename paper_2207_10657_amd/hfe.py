"""ctypes binding of libhfe.so (the C ABI declared in include/hfe.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides the device workspace and the stream. Importing this module
without the built library raises ImportError (there is no fallback path).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfe.so")

HFE_P1_PAIR, HFE_Q1 = 1, 2
HFE_ELASTIC, HFE_DAMAGE_ENERGY_NORM, HFE_DAMAGE_TENSILE = 0, 1, 2
FIELD_U, FIELD_GRAD, FIELD_STRESS, FIELD_DAMAGE, FIELD_KAPPA, FIELD_SOFTENING = range(6)
CG_INTERIOR, CG_BOUNDARY, CG_NEGCURV, CG_MAXITER, CG_STALL = 1, 2, 3, 4, 5
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENUMERIC", -5: "ESTATE"}


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("element", ctypes.c_int)]


class _Material(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("E", ctypes.c_double), ("nu", ctypes.c_double),
                ("kappa0", ctypes.c_double), ("kappaf", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("eta_eq", ctypes.c_double), ("eta_nr", ctypes.c_double),
                ("eta_cg", ctypes.c_double), ("eta_up", ctypes.c_double),
                ("R0", ctypes.c_double), ("Rmax", ctypes.c_double),
                ("i_nr_max", ctypes.c_int), ("j_cg_max", ctypes.c_int),
                ("precision", ctypes.c_int), ("restart", ctypes.c_double),
                ("cg_stall", ctypes.c_int)]


class _Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in (
        "plane_threads", "pencil_cols", "pencil_threads", "brick_shape",
        "plane_threads32", "pencil_cols32", "pencil_threads32", "brick_shape32")]


class _Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("newton_iters", ctypes.c_int),
                ("rejected", ctypes.c_int), ("cg_iters", ctypes.c_int),
                ("restarts", ctypes.c_int), ("boundary_exits", ctypes.c_int),
                ("negcurv_exits", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("stall_exits", ctypes.c_int),
                ("r_eq", ctypes.c_double), ("r_nr", ctypes.c_double),
                ("R", ctypes.c_double), ("rho_last", ctypes.c_double),
                ("time_ms", ctypes.c_double)]


class _LbfgsParams(ctypes.Structure):
    _fields_ = [("eta_eq", ctypes.c_double), ("eta_nr", ctypes.c_double),
                ("max_iters", ctypes.c_int), ("m", ctypes.c_int), ("c1", ctypes.c_double),
                ("max_backtracks", ctypes.c_int)]


class _LbfgsReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("trials", ctypes.c_int),
                ("pairs_skipped", ctypes.c_int), ("resets", ctypes.c_int),
                ("r_eq", ctypes.c_double), ("r_nr", ctypes.c_double), ("time_ms", ctypes.c_double)]


LBFGS_DEFAULTS = {"eta_eq": 1e-8, "eta_nr": 1e-8, "max_iters": 500, "m": 5, "c1": 1e-4,
                  "max_backtracks": 30}


class _Record(ctypes.Structure):
    _fields_ = [("flag", ctypes.c_int), ("cg_iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("accepted", ctypes.c_int), ("dm", ctypes.c_double), ("dW", ctypes.c_double),
                ("rho", ctypes.c_double), ("R_before", ctypes.c_double),
                ("p_norm", ctypes.c_double)]


EXPORTS = {
    "hfe_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(_Grid)]),
    "hfe_create": (ctypes.c_int, [ctypes.POINTER(_Grid), ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "hfe_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "hfe_set_microstructure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "hfe_set_material": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_Material)]),
    "hfe_apply_load_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_solve_increment": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Params),
                                           ctypes.POINTER(_Report)]),
    "hfe_homogenized_stress": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "hfe_get_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]),
    "hfe_get_newton_log": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Record), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]),
    "hfe_set_displacement": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_get_cg_trace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "hfe_apply_projected_hessian": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_apply_projected_hessian_f32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_apply_stiffness": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Tuning)]),
    "hfe_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Tuning)]),
    "hfe_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Tuning)]),
    "hfe_set_eigenstrain": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "hfe_set_mean_stress_control": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    # learned warm start (paper_2207_10657_amd.warmstart)
    "hfe_nn_conv3d": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "hfe_nn_conv3d_backward_data": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                                                   ctypes.c_void_p]),
    "hfe_nn_conv3d_backward_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                                      ctypes.c_void_p, ctypes.c_void_p,
                                                      ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                      ctypes.c_void_p, ctypes.c_void_p,
                                                      ctypes.c_void_p]),
    "hfe_nn_mse_partials": (ctypes.c_size_t, [ctypes.c_longlong]),
    "hfe_nn_mse_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_nn_mse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "hfe_nn_adam": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_longlong, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_nn_to_bf16": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "hfe_solve_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_Params),
                                       ctypes.c_void_p]),
    "hfe_effective_stiffness": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double,
                                               ctypes.POINTER(_Params), ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "hfe_apply_green": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_fft_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_fft_inverse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hfe_kernel_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_char_p),
                                        ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "hfe_soft_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
    "hfe_nn_pool2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_nn_pool2_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "hfe_nn_upsample2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hfe_nn_upsample2_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                                                 ctypes.c_void_p]),
    "hfe_lbfgs_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(_Grid), ctypes.c_int]),
    "hfe_solve_increment_lbfgs": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_LbfgsParams),
                                                 ctypes.c_void_p, ctypes.c_size_t,
                                                 ctypes.POINTER(_LbfgsReport)]),
    "hfe_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libhfe.so and declare its exports. Raises ImportError if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhfe.so not built (%s); run paper_2207_10657_amd.build.build()" % path)
    # torch first: libhfe.so must bind to the HIP runtime torch has loaded.
    # Loaded before torch, it would bind the system's runtime, torch would
    # then load its own, and device memory from one would be unknown to the
    # other (hfe_create fails on the workspace torch allocated).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HfeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


def _grid(shape, element):
    shape = tuple(int(s) for s in shape)
    g = _Grid()
    if len(shape) == 2:
        g.dim = 2
        g.n[0], g.n[1], g.n[2] = shape[1], shape[0], 1
    else:
        g.dim = 3
        g.n[0], g.n[1], g.n[2] = shape[2], shape[1], shape[0]
    g.element = {"q1": HFE_Q1, "p1pair": HFE_P1_PAIR}[element]
    return g


def workspace_bytes(shape, element):
    lib = load_library()
    return int(lib.hfe_workspace_bytes(ctypes.byref(_grid(shape, element))))


# CG arithmetic (hfe_solver_params.precision)
PRECISIONS = {"fp64": 0, "mixed": 1}
DEFAULT_PARAMS = {"eta_eq": 1e-8, "eta_nr": 1e-8, "eta_cg": 1e-6, "eta_up": 0.15,
                  "R0": 0.0, "Rmax": 0.0, "i_nr_max": 50, "j_cg_max": 2000, "precision": 0,
                  "restart": 0.2, "cg_stall": 0}


def _params(params):
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update({k: v for k, v in params.items() if v is not None and k in p})
    if isinstance(p["precision"], str):
        p["precision"] = PRECISIONS[p["precision"]]
    return _Params(**{k: p[k] for k in DEFAULT_PARAMS})


def _report(rep):
    out = {name: getattr(rep, name) for name, _ in _Report._fields_}
    out["converged"] = rep.status == 0
    return out


def solve_batch(solvers, params=None):
    """One load increment on each of several solvers at once
    (hfe_solve_batch): their work overlaps on the device when each runs on its
    own stream (``Solver(..., own_stream=True)``). Returns the reports."""
    lib = load_library()
    n = len(solvers)
    arr = (ctypes.c_void_p * n)(*[s.ctx.value for s in solvers])
    cp = _params(params)
    reps = (_Report * n)()
    st = lib.hfe_solve_batch(arr, n, ctypes.byref(cp), reps)
    if st != 0:
        msgs = "; ".join(lib.hfe_last_error(s.ctx).decode() for s in solvers)
        raise HfeError(st, msgs)
    return [_report(reps[i]) for i in range(n)]


def effective_stiffness(solvers, strain=1e-4, params=None):
    """The 6x6 effective stiffness (Voigt xx, yy, zz, yz, xz, xy, engineering
    shears) about the current states of six solvers of one cell
    (hfe_effective_stiffness); returns (C, reports)."""
    lib = load_library()
    if len(solvers) != 6:
        raise ValueError("six solvers, one per unit load case")
    arr = (ctypes.c_void_p * 6)(*[s.ctx.value for s in solvers])
    cp = _params(params)
    C = np.zeros(36)
    reps = (_Report * 6)()
    st = lib.hfe_effective_stiffness(arr, float(strain), ctypes.byref(cp),
                                     C.ctypes.data_as(ctypes.c_void_p), reps)
    if st != 0:
        msgs = "; ".join(lib.hfe_last_error(s.ctx).decode() for s in solvers)
        raise HfeError(st, msgs)
    return C.reshape(6, 6), [_report(reps[i]) for i in range(6)]


class Solver:
    """One periodic cell on one GPU.

    ``shape`` is (ny, nx) for 2D (element ``p1pair``) or (nz, ny, nx) for 3D
    (element ``q1``). Nodal fields are numpy arrays (dim, *shape); point fields
    (*shape, nq, dim, dim) or (*shape, nq).
    """

    def __init__(self, shape, element, device="cuda:0", own_stream=False):
        """``own_stream``: run on a new stream of this solver (default
        priority) instead of torch's current stream, so that the solves of
        several solvers in ``solve_batch`` overlap on the device."""
        import torch
        self.torch = torch
        self.lib = load_library()
        self.shape = tuple(int(s) for s in shape)
        self.element = element
        self.dim = len(self.shape)
        self.nq = 8 if element == "q1" else 2
        self.N = int(np.prod(self.shape))
        self.device = torch.device(device)
        g = _grid(self.shape, element)
        nbytes = int(self.lib.hfe_workspace_bytes(ctypes.byref(g)))
        if nbytes == 0:
            raise HfeError(-1, "unsupported grid %s / %s" % (self.shape, element))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.own_stream = bool(own_stream)
        if self.own_stream:
            self.stream = torch.cuda.Stream(self.device)
            self.workspace.record_stream(self.stream)
        else:
            self.stream = torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        st = self.lib.hfe_create(ctypes.byref(g), ctypes.c_void_p(self.workspace.data_ptr()),
                                 nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(ctx))
        if st != 0:
            raise HfeError(st, "hfe_create failed")
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hfe_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise HfeError(st, self.lib.hfe_last_error(self.ctx).decode())

    # -- problem definition ---------------------------------------------
    def set_microstructure(self, phase, n_phases):
        ph = np.ascontiguousarray(phase, dtype=np.uint8)
        if ph.shape != self.shape:
            raise ValueError("phase map shape %s != grid %s" % (ph.shape, self.shape))
        self._check(self.lib.hfe_set_microstructure(self.ctx, ph.ctypes.data_as(ctypes.c_void_p),
                                                    int(n_phases)))

    def set_material(self, phase, mat):
        m = _Material()
        kinds = {"elastic": HFE_ELASTIC, "damage": HFE_DAMAGE_ENERGY_NORM,
                 "tensile": HFE_DAMAGE_TENSILE}
        if mat["kind"] not in kinds:
            raise ValueError("unknown material kind %r" % (mat["kind"],))
        m.kind = kinds[mat["kind"]]
        m.E, m.nu = float(mat["E"]), float(mat["nu"])
        m.kappa0 = float(mat.get("kappa0", 0.0))
        m.kappaf = float(mat.get("kappaf", 0.0))
        self._check(self.lib.hfe_set_material(self.ctx, int(phase), ctypes.byref(m)))

    def setup(self, phase, materials):
        self.set_microstructure(phase, len(materials))
        for p, m in enumerate(materials):
            self.set_material(p, m)
            if m.get("eig") is not None:
                self.set_eigenstrain(p, m["eig"])

    def set_eigenstrain(self, phase, eig):
        """Eigenstrain of a phase (3x3), added to the strain before the law."""
        a = np.ascontiguousarray(np.asarray(eig, dtype=np.float64).reshape(3, 3))
        self._check(self.lib.hfe_set_eigenstrain(self.ctx, int(phase),
                                                 a.ctypes.data_as(ctypes.c_void_p)))

    def set_mean_stress_control(self, free):
        """Free macroscopic strain components with zero mean stress: a
        symmetric boolean 3x3 (or an int mask, Voigt bits xx yy zz yz xz xy)."""
        if isinstance(free, (int, np.integer)):
            mask = int(free)
        else:
            f = np.asarray(free, dtype=bool).reshape(3, 3)
            f = f | f.T
            mask = 0
            for v, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))):
                if f[i, j]:
                    mask |= 1 << v
        self._check(self.lib.hfe_set_mean_stress_control(self.ctx, mask))

    # -- Algorithm 2 -----------------------------------------------------
    def apply_load_step(self, dE):
        a = np.ascontiguousarray(np.asarray(dE, dtype=np.float64).reshape(3, 3))
        self._check(self.lib.hfe_apply_load_step(self.ctx, a.ctypes.data_as(ctypes.c_void_p)))

    def solve_increment(self, params=None):
        cp = _params(params)
        rep = _Report()
        self._check(self.lib.hfe_solve_increment(self.ctx, ctypes.byref(cp), ctypes.byref(rep)))
        return _report(rep)

    def solve_increment_lbfgs(self, params=None):
        """The increment by L-BFGS on the approximate energy increment
        (hfe_solve_increment_lbfgs); params: keys of LBFGS_DEFAULTS. The pair
        storage is a device buffer of this solver, kept between calls."""
        p = dict(LBFGS_DEFAULTS)
        if params:
            p.update({k: v for k, v in params.items() if v is not None})
        cp = _LbfgsParams(**p)
        g = _grid(self.shape, self.element)
        nbytes = int(self.lib.hfe_lbfgs_workspace_bytes(ctypes.byref(g), int(p["m"])))
        if nbytes == 0:
            raise HfeError(-1, "bad L-BFGS memory size m = %s" % p["m"])
        ws = getattr(self, "_lbfgs_ws", None)
        if ws is None or ws.numel() < nbytes:
            ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
            if self.own_stream:
                ws.record_stream(self.stream)
            self._lbfgs_ws = ws
        rep = _LbfgsReport()
        self._check(self.lib.hfe_solve_increment_lbfgs(
            self.ctx, ctypes.byref(cp), ctypes.c_void_p(ws.data_ptr()), nbytes, ctypes.byref(rep)))
        out = {name: getattr(rep, name) for name, _ in _LbfgsReport._fields_}
        out["converged"] = out["status"] == 0
        return out

    def newton_log(self, max_records=10000):
        recs = (_Record * max_records)()
        cnt = ctypes.c_int()
        self._check(self.lib.hfe_get_newton_log(self.ctx, recs, max_records, ctypes.byref(cnt)))
        return [{name: getattr(recs[i], name) for name, _ in _Record._fields_}
                for i in range(cnt.value)]

    def cg_trace(self, max_iters=1000000):
        out = np.zeros((max_iters, 2))
        cnt = ctypes.c_int()
        self._check(self.lib.hfe_get_cg_trace(self.ctx, out.ctypes.data_as(ctypes.c_void_p),
                                              max_iters, ctypes.byref(cnt)))
        return out[: cnt.value]

    def get_state(self):
        u = np.zeros((self.dim,) + self.shape)
        kh = np.zeros(self.shape + (self.nq,))
        E = np.zeros(9)
        R = np.zeros(2)
        self._check(self.lib.hfe_get_state(self.ctx, *(a.ctypes.data_as(ctypes.c_void_p)
                                                       for a in (u, kh, E, R))))
        return {"u": u, "kappa_hist": kh, "E": E.reshape(3, 3), "R": R[0], "Rmax": R[1]}

    def set_state(self, u, kappa_hist, E, R, Rmax):
        u = np.ascontiguousarray(u, dtype=np.float64)
        kh = np.ascontiguousarray(kappa_hist, dtype=np.float64)
        if u.shape != (self.dim,) + self.shape or kh.shape != self.shape + (self.nq,):
            raise ValueError("state shapes")
        Em = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(9))
        Rr = np.array([R, Rmax], dtype=np.float64)
        self._check(self.lib.hfe_set_state(self.ctx, *(a.ctypes.data_as(ctypes.c_void_p)
                                                       for a in (u, kh, Em, Rr))))

    def residual(self):
        """r_eq of the last evaluated state (hfe_residual)."""
        out = ctypes.c_double(0.0)
        self._check(self.lib.hfe_residual(self.ctx, ctypes.byref(out)))
        return out.value

    def homogenized_stress(self):
        out = np.zeros(9)
        self._check(self.lib.hfe_homogenized_stress(self.ctx, out.ctypes.data_as(ctypes.c_void_p)))
        return out.reshape(3, 3)

    def field(self, which):
        d, nq = self.dim, self.nq
        shapes = {FIELD_U: (d,) + self.shape,
                  FIELD_GRAD: self.shape + (nq, d, d),
                  FIELD_STRESS: self.shape + (nq, d, d),
                  FIELD_DAMAGE: self.shape + (nq,),
                  FIELD_KAPPA: self.shape + (nq,),
                  FIELD_SOFTENING: self.shape + (nq,)}
        out = np.zeros(shapes[which])
        self._check(self.lib.hfe_get_field(self.ctx, which, out.ctypes.data_as(ctypes.c_void_p),
                                           out.size))
        return out

    def displacement(self):
        return self.field(FIELD_U)

    def gradient(self):
        return self.field(FIELD_GRAD)

    def damage(self):
        return self.field(FIELD_DAMAGE)

    def set_displacement(self, u):
        a = np.ascontiguousarray(u, dtype=np.float64)
        if a.shape != (self.dim,) + self.shape:
            raise ValueError("displacement shape")
        self._check(self.lib.hfe_set_displacement(self.ctx, a.ctypes.data_as(ctypes.c_void_p)))

    # -- operators on device tensors ([dim][N] float64, contiguous) -------
    def _sync_in(self):
        """Device-tensor operators: the solver's stream waits for torch's."""
        if self.own_stream:
            self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _sync_out(self):
        if self.own_stream:
            self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _dev(self, t, dtype=None):
        torch = self.torch
        dtype = torch.float64 if dtype is None else dtype
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
            raise ValueError("expected a contiguous %s device tensor" % dtype)
        return ctypes.c_void_p(t.data_ptr())

    def new_nodal(self):
        return self.torch.zeros((self.dim,) + self.shape, dtype=self.torch.float64,
                                device=self.device)

    def apply_projected_hessian(self, d, out=None):
        out = self.new_nodal() if out is None else out
        dots = np.zeros(2)
        self._sync_in()
        self._check(self.lib.hfe_apply_projected_hessian(self.ctx, self._dev(d), self._dev(out),
                                                         dots.ctypes.data_as(ctypes.c_void_p)))
        self._sync_out()
        return out, dots

    def apply_projected_hessian_f32(self, d, out=None):
        """The projected Hessian in the FP32 arithmetic of the mixed-precision
        CG (3D): float32 device tensors [dim][N], dots {d.Kd, |Dd|^2} in FP64."""
        torch = self.torch
        out = torch.zeros((self.dim,) + self.shape, dtype=torch.float32,
                          device=self.device) if out is None else out
        dots = np.zeros(2)
        self._sync_in()
        self._check(self.lib.hfe_apply_projected_hessian_f32(
            self.ctx, self._dev(d, torch.float32), self._dev(out, torch.float32),
            dots.ctypes.data_as(ctypes.c_void_p)))
        self._sync_out()
        return out, dots

    def tuning(self):
        t = _Tuning()
        self._check(self.lib.hfe_get_tuning(self.ctx, ctypes.byref(t)))
        return {name: getattr(t, name) for name, _ in _Tuning._fields_}

    def set_tuning(self, **kw):
        cur = self.tuning()
        cur.update(kw)
        t = _Tuning(**cur)
        self._check(self.lib.hfe_set_tuning(self.ctx, ctypes.byref(t)))

    def autotune(self):
        """Time the launch shapes on this grid (and, after a load step, the
        Hessian brick shapes at the current state); keep the fastest."""
        t = _Tuning()
        self._check(self.lib.hfe_autotune(self.ctx, ctypes.byref(t)))
        return {name: getattr(t, name) for name, _ in _Tuning._fields_}

    def apply_stiffness(self, d, out=None):
        out = self.new_nodal() if out is None else out
        self._sync_in()
        self._check(self.lib.hfe_apply_stiffness(self.ctx, self._dev(d), self._dev(out)))
        self._sync_out()
        return out

    def apply_green(self, f, out=None):
        out = self.new_nodal() if out is None else out
        self._sync_in()
        self._check(self.lib.hfe_apply_green(self.ctx, self._dev(f), self._dev(out)))
        self._sync_out()
        return out

    def _spec_shape(self):
        if self.dim == 2:
            ny, nx = self.shape
            return (2, 1, ny, nx // 2 + 1, 2)
        nz, ny, nx = self.shape
        return (3, nz, ny, nx // 2 + 1, 2)

    def fft_forward(self, f):
        out = self.torch.zeros(self._spec_shape(), dtype=self.torch.float64, device=self.device)
        self._sync_in()
        self._check(self.lib.hfe_fft_forward(self.ctx, self._dev(f), self._dev(out)))
        self._sync_out()
        return out

    def fft_inverse(self, spec):
        out = self.new_nodal()
        self._sync_in()
        self._check(self.lib.hfe_fft_inverse(self.ctx, self._dev(spec), self._dev(out)))
        self._sync_out()
        return out

    # -- profiling -------------------------------------------------------
    def set_profiling(self, on):
        self._check(self.lib.hfe_set_profiling(self.ctx, 1 if on else 0))

    def kernel_stats(self, max_kernels=32):
        names = (ctypes.c_char_p * max_kernels)()
        counts = (ctypes.c_int * max_kernels)()
        ms = (ctypes.c_double * max_kernels)()
        n = ctypes.c_int()
        self._check(self.lib.hfe_kernel_stats(self.ctx, names, counts, ms, max_kernels,
                                              ctypes.byref(n)))
        return {names[i].decode(): (counts[i], ms[i]) for i in range(n.value)}

    def soft_points(self):
        """(softening points of the evaluated state, their mean over the Hessian
        launches timed since the last set_profiling)."""
        cur, mean = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.hfe_soft_points(self.ctx, ctypes.byref(cur), ctypes.byref(mean)))
        return cur.value, mean.value
