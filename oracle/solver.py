"""Steihaug-CG with restart and the FAIEF trust-region Newton solver (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Both follow the paper's Algorithms 1 and 2 in strain space, under these
readings of its text (the printed listings reuse symbols and are partly
garbled):

Steihaug (Algorithm 1; Sec. 2.2, truncated CG of Steihaug with the reset of
Powell and Dai, eq. 1): z is the iterate, r = A z + g the model gradient
(g = G sigma, so the printed right-hand side is b = -g), d_0 = -r_0.
  * negative curvature (d.Ad <= 0): return z + tau d on ||.|| = R, choosing
    of the two roots the one with the smaller model value (ties: tau > 0);
  * boundary (||z + alpha d|| >= R): return z + tau d with the root tau >= 0;
  * convergence: ||r_{j+1}|| <= eta_cg ||r_0||;
  * reset: if |r_{j+1}.r_j| > c r_{j+1}.r_{j+1} (Powell's constant c = 0.2
    in the paper, a knob here), recompute the residual r_{j+1} = A z_{j+1} + g
    and take beta = 0 (a steepest-descent restart). Any c < 0 restarts after
    every step, which turns the method into steepest descent with exact line
    search; c = inf never restarts (plain CG);
  * after j_max steps the last iterate is returned (an interior step);
  * optional stall exit (not in the paper; ``stall`` > 0 iterations): the
    residual norm is followed against a reference that starts at ||r_0||
    and is replaced by every residual at or below half of it; once ``stall``
    iterations pass without such a replacement the current iterate is
    returned as an interior step (flag STALL). Tested after convergence and
    before the reset.

Trust region (Algorithm 2; eq. modeling_trust, eq. incr_energy_func, eq.
rho_bar): Delta m = sigma:p + p:B:p/2 and DeltaW = (sigma + sigma_trial):p/2
are both "new minus old", so rho = DeltaW / Delta m. R <- R/4 if rho < 1/4,
R <- min(2R, R_max) if rho > 3/4 and the step lies on the boundary; the step is
accepted iff rho > eta_up. A non-finite rho, or Delta m >= 0, counts as a
rejection. Equilibrium is measured relative to the stress,
r_eq = ||G sigma|| / ||sigma||; r_NR = ||p|| / ||H|| as printed. Convergence
needs an interior step and (r_eq <= eta_eq or r_NR <= eta_NR). The history
(kappa_hist) is committed only when a load step converges.

Mean-stress control (Sec. 3.3 imposes a zero mean stress with a modified
projector from cited work; this is the reading used here): chosen components
of the macroscopic strain are unknowns whose mean stress must vanish. The
projector becomes G_M = G + M, where M maps a field to its mean in the free
components (for a free shear pair (i, j) the mean of (X_ij + X_ji)/2 in both
entries), an orthogonal projector onto uniform fields that G annihilates, so
G_M is again an orthogonal projector. The model gradient is G_M sigma, the
projected Hessian G_M B, and the steps p = D du + uniform free part; an
accepted step moves E by the mean of p. At convergence G sigma = 0 and the
mean stress vanishes in the free components.

Eigenstrain (Algorithm 2, the eps_eval lines): a phase's eigenstrain is added
to the strain before every evaluation of the law, the trial evaluation
included; r_NR keeps the strain without it. A load by eigenstrain alone (zero
first macroscopic increment) takes the radius scale from the largest phase
eigenstrain.

Pinned by (``tests/test_oracle_solver.py``, ``tests/test_oracle_cell.py``):
dense SPD solves and exact boundary exits (Steihaug); the 1D damage-spring
system of Sec. 3.1 against a brute-force energy scan; the homogeneous and
laminate closed forms; a dense FE solve of heterogeneous elasticity; the
exactness of the FAIEF ratio for quadratic energies and its third-order
error for the damage law.
"""
import math
import numpy as np

from . import fe, material
from .projection import Projector

INTERIOR, BOUNDARY, NEGCURV, MAXITER, STALL = 1, 2, 3, 4, 5
FLAG_NAMES = {INTERIOR: "interior", BOUNDARY: "boundary", NEGCURV: "negcurv",
              MAXITER: "maxiter", STALL: "stall"}


def inner(X, Y):
    """Plain (unweighted) sum over all points and components."""
    return float(np.sum(X * Y))


def _roots(zz, zd, dd, R):
    """Both roots of zz + 2 tau zd + tau^2 dd = R^2 (zz < R^2), cancellation free."""
    b = 2.0 * zd
    c = zz - R * R
    disc = math.sqrt(max(b * b - 4.0 * dd * c, 0.0))
    qq = -0.5 * (b + math.copysign(disc, b))
    t1 = qq / dd
    t2 = c / qq if qq != 0.0 else -t1
    return min(t1, t2), max(t1, t2)


def steihaug(apply_A, g, R, eta_cg, j_max, dot=inner, log=None, restart=0.2, stall=0):
    """Truncated CG on min g.p + p.Ap/2, ||p|| <= R. Returns (p, flag, info).

    ``restart`` is the constant of Powell's reset test (eq. 1); ``stall`` the
    window of the optional stall exit (0: off)."""
    info = {"iters": 0, "restarts": 0, "matvecs": 0}
    z = np.zeros_like(g)
    r = g.copy()
    rr = dot(r, r)
    rr0 = rr
    if rr0 == 0.0:
        return z, INTERIOR, info
    d = -r
    rr_ref, j_ref = rr0, 0
    for j in range(j_max):
        Ad = apply_A(d)
        info["matvecs"] += 1
        kappa = dot(d, Ad)
        info["iters"] = j + 1
        zz, zd, dd = dot(z, z), dot(z, d), dot(d, d)
        if kappa <= 0.0:
            if log is not None:
                log.append(("cg", j, kappa, math.nan))
            tm, tp = _roots(zz, zd, dd, R)
            rd = dot(r, d)
            m_m = tm * rd + 0.5 * tm * tm * kappa
            m_p = tp * rd + 0.5 * tp * tp * kappa
            tau = tm if m_m < m_p else tp
            return z + tau * d, NEGCURV, info
        alpha = rr / kappa
        z_new = z + alpha * d
        if math.sqrt(dot(z_new, z_new)) >= R:
            if log is not None:
                log.append(("cg", j, kappa, math.nan))
            _, tp = _roots(zz, zd, dd, R)
            return z + tp * d, BOUNDARY, info
        r_new = r + alpha * Ad
        rr_new = dot(r_new, r_new)
        if log is not None:
            # curvature and ||r_{j+1}|| / ||r_0|| (the CG stopping measure)
            log.append(("cg", j, kappa, math.sqrt(rr_new / rr0)))
        if math.sqrt(rr_new) <= eta_cg * math.sqrt(rr0):
            return z_new, INTERIOR, info
        if rr_new <= 0.25 * rr_ref:
            rr_ref, j_ref = rr_new, j + 1
        elif stall > 0 and j + 1 - j_ref >= stall:
            return z_new, STALL, info
        if abs(dot(r_new, r)) > restart * rr_new:
            r_new = apply_A(z_new) + g
            info["matvecs"] += 1
            rr_new = dot(r_new, r_new)
            beta = 0.0
            info["restarts"] += 1
        else:
            beta = rr_new / rr
        d = -r_new + beta * d
        z, r, rr = z_new, r_new, rr_new
    return z, MAXITER, info


DEFAULTS = {"eta_eq": 1e-8, "eta_nr": 1e-8, "eta_cg": 1e-6, "eta_up": 0.15,
            "i_nr_max": 50, "j_cg_max": 2000, "restart": 0.2, "cg_stall": 0}


def default_radii(n_qp, dE):
    """R0 = 10 sqrt(N_qp) ||dE||_F, Rmax = 1000 sqrt(N_qp) ||dE||_F (strain space).

    The paper gives no values; the sqrt(N_qp) factor follows its remark that
    the radius has to grow with the resolution (Sec. 3.2).
    """
    s = math.sqrt(n_qp) * float(np.linalg.norm(dE))
    return 10.0 * s, 1000.0 * s


def tr_update(rho, R, Rmax, on_boundary):
    """Radius update of Algorithm 2: shrink by 4 or expand by 2 (capped)."""
    if rho < 0.25:
        return 0.25 * R
    if rho > 0.75 and on_boundary:
        return min(2.0 * R, Rmax)
    return R


def faief_ratio(sigma_p, p_B_p, sigma_t_p):
    """(Delta m, Delta W_bar, rho_bar) from the three inner products.

    Delta m = sigma:p + p:B:p/2 (eq. modeling_trust, model change new - old),
    Delta W_bar = (sigma + sigma_trial):p / 2 (eq. incr_energy_func),
    rho_bar = Delta W_bar / Delta m (eq. rho_bar). A non-negative or
    non-finite Delta m gives rho = -inf (rejection).
    """
    dm = sigma_p + 0.5 * p_B_p
    dW = 0.5 * (sigma_p + sigma_t_p)
    if dm < 0.0 and math.isfinite(dm) and math.isfinite(dW):
        rho = dW / dm
    else:
        rho = -math.inf
    if not math.isfinite(rho):
        rho = -math.inf
    return dm, dW, rho


class CellSolver:
    """Periodic cell under macroscopic strain control, solved in strain space.

    ``R0``/``Rmax`` fix the trust radius; by default they come from the first
    load increment via ``default_radii``. The radius is state: it carries over
    from one load step to the next (Algorithm 2 initialises it once).
    """

    def __init__(self, phase, materials, element, R0=None, Rmax=None):
        self.element = element
        self.dim = fe.element_dim(element)
        self.grid = tuple(np.asarray(phase).shape)
        if len(self.grid) != self.dim:
            raise ValueError("phase map dimension does not match the element")
        self.nq = fe.shape_gradients(element).shape[0]
        self.mat = material.MaterialField(phase, materials, self.nq)
        self.G = Projector(self.grid, element)
        self.H = np.zeros(self.grid + (self.nq, self.dim, self.dim))
        self.E = np.zeros((3, 3))
        self.kappa_hist = self.mat.initial_history()
        self.R = R0
        self.Rmax = Rmax
        self.state = None
        self.sigma = None
        self.g = None
        self.r_eq = None
        self.n_qp = int(np.prod(self.grid)) * self.nq
        self.free = np.zeros((self.dim, self.dim), dtype=bool)

    def set_mean_stress_control(self, free):
        """Free macroscopic strain components (a symmetric boolean 3x3, the
        d x d block used) whose mean stress is held at zero from the next load
        step on; all False restores full strain control."""
        f = np.asarray(free, dtype=bool).reshape(3, 3)[: self.dim, : self.dim]
        self.free = f | f.T

    def _mean_free(self, X):
        """M X: the uniform field of X's mean in the free components (a free
        shear pair gets the mean of (X_ij + X_ji) / 2 in both entries)."""
        m = X.mean(axis=tuple(range(self.dim + 1)))
        m = 0.5 * (m + m.T)
        out = np.zeros_like(X)
        out[...] = np.where(self.free, m, 0.0)
        return out

    def project(self, X):
        """G_M X = G X + M X (G alone without stress control)."""
        if not self.free.any():
            return self.G(X)
        return self.G(X) + self._mean_free(X)

    def set_eigenstrain(self, phase, eig):
        """Eigenstrain of a phase from now on (Algorithm 2 adds it to the
        strain before every evaluation); the next apply_load_step evaluates
        the state with it."""
        self.mat.set_eigenstrain(phase, eig)

    # -- state evaluation -------------------------------------------------
    def _evaluate(self, H):
        return material.evaluate(self.mat, H, self.kappa_hist)

    def _set_state(self, st):
        self.state = st
        self.sigma = st["sigma"]
        self.g = self.project(self.sigma)
        ns = math.sqrt(inner(self.sigma, self.sigma))
        self.r_eq = math.sqrt(inner(self.g, self.g)) / ns if ns > 0.0 else 0.0

    def apply_hessian(self, X):
        """Projected Hessian G : B : X (eq. project_stress_linear); G_M : B : X
        under mean-stress control."""
        return self.project(material.apply_tangent(self.mat, self.state, X))

    # -- Algorithm 2 --------------------------------------------------------
    def apply_load_step(self, dE):
        """H <- H + dE (previous fluctuation kept); evaluate sigma, B, G sigma."""
        dE = np.asarray(dE, dtype=np.float64)
        self.E = self.E + dE
        d = self.dim
        self.H = self.H + dE[:d, :d]
        if self.R is None or self.Rmax is None:
            # the load that sets the radius scale: the first macroscopic
            # increment, or, for a load by eigenstrain alone, the largest
            # phase eigenstrain
            load = dE[:d, :d]
            if not np.any(load):
                norms = [np.linalg.norm(e) for e in self.mat.eig_table]
                load = self.mat.eig_table[int(np.argmax(norms))]
            R0, Rmax = default_radii(self.n_qp, load)
            self.R = R0 if self.R is None else self.R
            self.Rmax = Rmax if self.Rmax is None else self.Rmax
        self._set_state(self._evaluate(self.H))
        return self.r_eq

    def solve_increment(self, params=None, log=None):
        p = dict(DEFAULTS)
        if params:
            p.update({k: v for k, v in params.items() if v is not None})
        rep = {"newton_iters": 0, "rejected": 0, "cg_iters": 0, "restarts": 0,
               "boundary_exits": 0, "negcurv_exits": 0, "matvecs": 0, "stall_exits": 0,
               "converged": False, "rho": [], "flags": [], "cg_per_newton": [],
               "restarts_per_newton": [],
               "r_nr": None}
        if self.r_eq <= p["eta_eq"]:
            rep["converged"] = True
            self._commit()
            rep.update(self._report_tail())
            return rep
        for it in range(p["i_nr_max"]):
            rep["newton_iters"] = it + 1
            step, flag, info = steihaug(self.apply_hessian, self.g, self.R,
                                        p["eta_cg"], p["j_cg_max"], log=log,
                                        restart=p["restart"], stall=p["cg_stall"])
            rep["cg_iters"] += info["iters"]
            rep["restarts"] += info["restarts"]
            rep["matvecs"] += info["matvecs"]
            rep["cg_per_newton"].append(info["iters"])
            rep["restarts_per_newton"].append(info["restarts"])
            rep["flags"].append(flag)
            if flag == BOUNDARY:
                rep["boundary_exits"] += 1
            elif flag == NEGCURV:
                rep["negcurv_exits"] += 1
            elif flag == STALL:
                rep["stall_exits"] += 1
            sp = inner(self.sigma, step)
            pBp = inner(step, material.apply_tangent(self.mat, self.state, step))
            st_t = self._evaluate(self.H + step)
            stp = inner(st_t["sigma"], step)
            dm, dW, rho = faief_ratio(sp, pBp, stp)
            rep["rho"].append(rho)
            if log is not None:
                log.append(("newton", it, flag, info["iters"], dm, dW, rho, self.R))
            on_boundary = flag in (BOUNDARY, NEGCURV)
            self.R = tr_update(rho, self.R, self.Rmax, on_boundary)
            if rho > p["eta_up"]:
                self.H = self.H + step
                if self.free.any():
                    # the uniform part of the step moves the free macroscopic strain
                    dEf = self._mean_free(step).reshape(-1, self.dim, self.dim)[0]
                    self.E[: self.dim, : self.dim] += dEf
                r_nr = math.sqrt(inner(step, step)) / math.sqrt(inner(self.H, self.H))
                self._set_state(st_t)
                rep["r_nr"] = r_nr
                if not on_boundary and (self.r_eq <= p["eta_eq"] or r_nr <= p["eta_nr"]):
                    rep["converged"] = True
                    self._commit()
                    rep.update(self._report_tail())
                    return rep
            else:
                rep["rejected"] += 1
        rep.update(self._report_tail())
        return rep

    def checkpoint(self):
        """State for a restart: nodal u, history, macroscopic strain, radii."""
        return {"u": self.displacement(), "kappa_hist": self.kappa_hist.copy(),
                "E": self.E.copy(), "R": self.R, "Rmax": self.Rmax}

    def restore(self, ck):
        """Resume from a checkpoint: H = E + D u, the history and the radii;
        the next apply_load_step evaluates the state."""
        E = np.asarray(ck["E"], dtype=np.float64).reshape(3, 3)
        self.E = E.copy()
        self.H = fe.gradient(np.asarray(ck["u"], dtype=np.float64), self.element) \
            + E[: self.dim, : self.dim]
        self.kappa_hist = np.asarray(ck["kappa_hist"], dtype=np.float64).copy()
        self.R, self.Rmax = float(ck["R"]), float(ck["Rmax"])

    def _commit(self):
        self.kappa_hist = material.committed_history(self.mat, self.state, self.kappa_hist)

    def _report_tail(self):
        return {"r_eq": self.r_eq, "R": self.R}

    # -- outputs ------------------------------------------------------------
    def homogenized_stress(self):
        """Plain mean of the stress over all quadrature points, as 3x3."""
        out = np.zeros((3, 3))
        d = self.dim
        out[:d, :d] = self.sigma.mean(axis=tuple(range(d + 1)))
        if d == 2:
            out[2, 2] = self.state["sigma_zz"].mean()
        return out

    def damage(self):
        """d(kappa_hist) per point (committed history)."""
        m = self.mat
        return np.where(m.damage, material.damage_of_kappa(
            np.where(m.damage, self.kappa_hist, 1.0), m.k0, m.kf), 0.0)

    def displacement(self):
        """Nodal fluctuation u (d, *grid), zero mean, with D u = H - E.

        Recovered with the FE Green's function of D^T D.
        """
        fluct = self.H - self.E[:self.dim, :self.dim]
        f = fe.divergence(fluct, self.element)
        fh = np.fft.fftn(f, axes=tuple(range(1, self.dim + 1)))
        uh = fh * self.G.invS[None, ...]
        return np.fft.ifftn(uh, axes=tuple(range(1, self.dim + 1))).real
