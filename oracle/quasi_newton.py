"""L-BFGS on the approximate incremental energy (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2 observes that quasi-Newton methods need the objective itself, and
that the first-order approximation of the energy increment (eq.
incr_energy_func) makes them usable where the stored energy is not at hand.
The paper evaluates no such method; this module writes one out, in strain
space like the rest of the oracle, under these readings:

* unknown: the compatible strain H = E + D u of the load step; gradient
  g = G sigma (eq. proj_operator), the residual of Algorithm 2;
* direction: p = -H_k g by the two-loop recursion of L-BFGS (Nocedal, 1980)
  over the last m pairs (s, y), s the accepted step and y the change of g;
  H_0 = gamma I with gamma = s.y / y.y of the newest pair, and before any pair
  gamma = 1 / max over phases of (lambda + 2 mu), the largest eigenvalue of an
  isotropic elastic phase on compatible fields;
* a direction with sigma:p >= 0 is replaced by -gamma g and the memory cleared;
* step length: backtracking from alpha = 1, halving at most 30 times, until
  the Armijo condition holds with the approximate energy increment,
  DeltaW_bar(alpha p) <= c1 alpha sigma:p with c1 = 1e-4, where
  DeltaW_bar(v) = (sigma(H) + sigma(H + v)) : v / 2 (eq. incr_energy_func,
  history frozen); no step found ends the increment unconverged;
* a pair is kept only if s.y > 1e-12 |s| |y| (the damage energy is not convex,
  so the curvature condition can fail);
* convergence as Algorithm 2: r_eq = |G sigma| / |sigma| <= eta_eq, or
  r_NR = |s| / |H| <= eta_NR after an accepted step; the history is committed
  when the increment converges.

Pinned by ``tests/test_oracle_quasi_newton.py``: the two-loop recursion
against the explicit BFGS update of a dense inverse-Hessian matrix, the
energy increment against the exact stored energy on a quadratic (elastic)
problem, the laminate closed form, and the elastic equilibrium of the
trust-region Newton solver.
"""
import math

import numpy as np

from . import material
from .solver import inner

QN_DEFAULTS = {"eta_eq": 1e-8, "eta_nr": 1e-8, "i_qn_max": 500, "m": 5, "c1": 1e-4,
               "max_backtracks": 30}


def two_loop(q, pairs, gamma, dot):
    """-(inverse-Hessian approximation) applied to q: the L-BFGS two-loop
    recursion over pairs (s, y, rho = 1 / s.y), oldest first; returns H q."""
    q = q.copy()
    alphas = []
    for s, y, rho in reversed(pairs):
        a = rho * dot(s, q)
        q -= a * y
        alphas.append(a)
    r = gamma * q
    for (s, y, rho), a in zip(pairs, reversed(alphas)):
        b = rho * dot(y, r)
        r += (a - b) * s
    return r


def initial_gamma(mat):
    """1 / max over the cell of (lambda + 2 mu)."""
    return 1.0 / float(np.max(mat.lam + 2.0 * mat.mu))


def energy_increment(sigma, sigma_t, v):
    """DeltaW_bar(v) = (sigma + sigma_t) : v / 2 (eq. incr_energy_func)."""
    return 0.5 * (inner(sigma, v) + inner(sigma_t, v))


def solve_increment_lbfgs(cs, params=None):
    """One load increment of the CellSolver `cs` (apply_load_step done) by
    L-BFGS on the approximate energy. Returns a report dict."""
    p = dict(QN_DEFAULTS)
    if params:
        p.update({k: v for k, v in params.items() if v is not None})
    rep = {"iters": 0, "trials": 0, "pairs_skipped": 0, "resets": 0, "converged": False,
           "r_nr": None}
    if cs.r_eq <= p["eta_eq"]:
        rep["converged"] = True
        cs._commit()
        rep.update(cs._report_tail())
        return rep
    gamma0 = initial_gamma(cs.mat)
    pairs = []
    for it in range(p["i_qn_max"]):
        rep["iters"] = it + 1
        g = cs.g
        if pairs:
            s_new, y_new, _ = pairs[-1]
            gamma = inner(s_new, y_new) / inner(y_new, y_new)
        else:
            gamma = gamma0
        d = -two_loop(g, pairs, gamma, inner)
        sp = inner(cs.sigma, d)
        if not sp < 0.0:
            pairs = []
            rep["resets"] += 1
            d = -gamma0 * g
            sp = inner(cs.sigma, d)
        alpha = 1.0
        accepted = None
        for _ in range(p["max_backtracks"] + 1):
            v = alpha * d
            st_t = cs._evaluate(cs.H + v)
            rep["trials"] += 1
            dW = energy_increment(cs.sigma, st_t["sigma"], v)
            if dW <= p["c1"] * alpha * sp:
                accepted = (v, st_t)
                break
            alpha *= 0.5
        if accepted is None:
            break
        v, st_t = accepted
        g_old = cs.g
        cs.H = cs.H + v
        cs._set_state(st_t)
        y = cs.g - g_old
        sy = inner(v, y)
        if sy > 1e-12 * math.sqrt(inner(v, v) * inner(y, y)):
            pairs.append((v, y, 1.0 / sy))
            if len(pairs) > p["m"]:
                pairs.pop(0)
        else:
            rep["pairs_skipped"] += 1
        r_nr = math.sqrt(inner(v, v)) / math.sqrt(inner(cs.H, cs.H))
        rep["r_nr"] = r_nr
        if cs.r_eq <= p["eta_eq"] or r_nr <= p["eta_nr"]:
            rep["converged"] = True
            cs._commit()
            break
    rep.update(cs._report_tail())
    return rep


def exact_energy(cs, H):
    """Stored energy at H with the history frozen (for the pins)."""
    return material.energy(cs.mat, H, cs.kappa_hist)
