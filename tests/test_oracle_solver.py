"""Pins of the oracle's Steihaug-CG (Algorithm 1) and of the FAIEF trust-region
driver (Algorithm 2) on small systems with known answers.

* SPD systems with an inactive trust region: the result is the solution of
  the linear system (numpy.linalg.solve), without restarts in FP64.
* Boundary and negative-curvature exits land on the sphere ||p|| = R and
  decrease the model.
* The 1D damage-spring ring of Sec. 3.1: its post-peak nodal stiffness has the
  printed eigenvalues (eq. K_mat), and the trust-region solver with the
  approximate ratio (eq. rho_bar) and with the exact one (eq. rho) reach the
  minimiser of the energy found by a brute-force scan.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import solver
from oracle.spring import SpringRing

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "spring_1d.json")


def _spd(n, rng, cond=50.0):
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.geomspace(1.0, cond, n)
    return Q @ np.diag(ev) @ Q.T


def test_steihaug_interior_is_linear_solve():
    rng = np.random.default_rng(0)
    A = _spd(30, rng)
    g = rng.normal(size=30)
    p, flag, info = solver.steihaug(lambda v: A @ v, g, 1e9, 1e-13, 500)
    assert flag == solver.INTERIOR
    np.testing.assert_allclose(p, np.linalg.solve(A, -g), rtol=1e-10, atol=1e-12)
    assert info["restarts"] == 0


def test_steihaug_boundary_exit():
    rng = np.random.default_rng(1)
    A = _spd(20, rng)
    g = rng.normal(size=20)
    full = np.linalg.norm(np.linalg.solve(A, -g))
    R = 0.3 * full
    p, flag, _ = solver.steihaug(lambda v: A @ v, g, R, 1e-12, 500)
    assert flag == solver.BOUNDARY
    assert abs(np.linalg.norm(p) - R) <= 1e-12 * R
    assert g @ p + 0.5 * p @ A @ p < 0.0


def test_steihaug_negative_curvature_exit():
    rng = np.random.default_rng(2)
    n = 12
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(np.linspace(-1.0, 3.0, n)) @ Q.T
    g = rng.normal(size=n)
    R = 2.0
    p, flag, _ = solver.steihaug(lambda v: A @ v, g, R, 1e-12, 500)
    assert flag in (solver.NEGCURV, solver.BOUNDARY)
    assert abs(np.linalg.norm(p) - R) <= 1e-12 * R
    assert g @ p + 0.5 * p @ A @ p < 0.0


def test_steihaug_restart_after_every_step_is_steepest_descent():
    """Powell's reset (eq. 1) with a negative constant fires after every step
    (the measure |r_{j+1}.r_j| / r_{j+1}.r_{j+1} is never negative): the
    residual is recomputed as A z + g and the direction restarts along it
    (beta = 0). The iterates are then those of steepest descent with exact
    line search, written out here from its textbook definition:
        r_j = A z_j + g,  z_{j+1} = z_j - (r_j.r_j / r_j.A r_j) r_j."""
    rng = np.random.default_rng(4)
    n, k = 24, 17
    A = _spd(n, rng, cond=30.0)
    g = rng.normal(size=n)
    p, flag, info = solver.steihaug(lambda v: A @ v, g, 1e9, 1e-14, k, restart=-1.0)
    z = np.zeros(n)
    for _ in range(k):
        r = A @ z + g
        z = z - (r @ r) / (r @ (A @ r)) * r
    assert flag == solver.MAXITER
    assert info["restarts"] == k and info["matvecs"] == 2 * k
    assert np.linalg.norm(p - z) <= 1e-12 * np.linalg.norm(z)
    # and it is not CG: plain CG (no reset) is much further along after k steps
    q, _, info_cg = solver.steihaug(lambda v: A @ v, g, 1e9, 1e-14, k, restart=np.inf)
    x = np.linalg.solve(A, -g)
    assert info_cg["restarts"] == 0
    assert np.linalg.norm(q - x) < 1e-2 * np.linalg.norm(p - x)


def test_steihaug_restart_keeps_the_model_decreasing_and_stops_on_the_sphere():
    """With resets at every step the trust-region exits still land on
    ||p|| = R, and a reset iterate keeps Algorithm 1's residual equal to the
    true model gradient A z + g (checked through the returned interior step:
    its model gradient norm meets the stopping test)."""
    rng = np.random.default_rng(5)
    n = 16
    A = _spd(n, rng, cond=8.0)
    g = rng.normal(size=n)
    x = np.linalg.solve(A, -g)
    R = 0.97 * np.linalg.norm(x)
    p, flag, info = solver.steihaug(lambda v: A @ v, g, R, 1e-10, 400, restart=-1.0)
    assert flag == solver.BOUNDARY and info["restarts"] >= 1
    assert abs(np.linalg.norm(p) - R) <= 1e-12 * R
    assert g @ p + 0.5 * p @ A @ p < 0.0
    p, flag, info = solver.steihaug(lambda v: A @ v, g, 1e9, 1e-8, 4000, restart=-1.0)
    assert flag == solver.INTERIOR and info["restarts"] >= 1
    assert np.linalg.norm(A @ p + g) <= 1.0001e-8 * np.linalg.norm(g)


def test_steihaug_stall_exit():
    """The optional stall exit (not in the paper) on a singular SPD system
    whose right-hand side has a component in the null space: the model
    gradient A z + g cannot fall below that component, so the CG stalls. The
    exit returns the CG iterate of the iteration at which it fires (the same
    iterate plain CG reaches after as many iterations). On a well-conditioned
    system it never fires."""
    rng = np.random.default_rng(6)
    n = 20
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.geomspace(1.0, 40.0, n)
    ev[0] = 0.0
    A = Q @ np.diag(ev) @ Q.T
    g = Q @ np.concatenate([[1e-3], rng.normal(size=n - 1)])
    p, flag, info = solver.steihaug(lambda v: A @ v, g, np.inf, 1e-12, 500, stall=6)
    assert flag == solver.STALL
    assert 6 <= info["iters"] < 500
    q, flag_q, info_q = solver.steihaug(lambda v: A @ v, g, np.inf, 1e-12, info["iters"])
    assert flag_q == solver.MAXITER and info_q["iters"] == info["iters"]
    np.testing.assert_array_equal(p, q)
    # a well-conditioned SPD system halves its residual well within the window
    B = _spd(20, rng, cond=10.0)
    p, flag, info = solver.steihaug(lambda v: B @ v, g, 1e9, 1e-12, 500, stall=6)
    assert flag == solver.INTERIOR
    np.testing.assert_allclose(p, np.linalg.solve(B, -g), rtol=1e-9, atol=1e-12)


def test_steihaug_zero_gradient_returns_zero():
    p, flag, info = solver.steihaug(lambda v: v, np.zeros(5), 1.0, 1e-6, 10)
    assert flag == solver.INTERIOR and np.all(p == 0) and info["iters"] == 0


def test_faief_ratio_exact_for_quadratic_energy():
    # W(x) = x.Ax/2 + b.x: DeltaW_bar equals the true change, so rho = 1
    rng = np.random.default_rng(3)
    A = _spd(8, rng)
    b = rng.normal(size=8)
    x = rng.normal(size=8)
    p = rng.normal(size=8) * 0.1
    sig = A @ x + b
    sig_t = A @ (x + p) + b
    dm, dW, rho = solver.faief_ratio(sig @ p, p @ A @ p, sig_t @ p)
    W = lambda y: 0.5 * y @ A @ y + b @ y
    assert abs(dW - (W(x + p) - W(x))) <= 1e-13 * abs(dW)
    if dm < 0:
        assert abs(rho - dW / dm) < 1e-15


def test_radius_update_rules():
    # Algorithm 2: shrink by 4 below 1/4, double (capped) above 3/4 on the
    # boundary, otherwise keep
    assert solver.tr_update(0.1, 8.0, 100.0, True) == 2.0
    assert solver.tr_update(0.9, 8.0, 100.0, True) == 16.0
    assert solver.tr_update(0.9, 8.0, 10.0, True) == 10.0
    assert solver.tr_update(0.9, 8.0, 100.0, False) == 8.0
    assert solver.tr_update(0.5, 8.0, 100.0, True) == 8.0


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("alpha", [1.0, -0.5, -1.0])
def test_spring_stiffness_eigenvalues(alpha):
    gd = _golden()
    k = gd["k"]
    s = SpringRing(k=k, gamma0=gd["gamma0"], alpha=alpha, x_bar=gd["x_bar"])
    # a post-peak state of the damage spring (gamma0 < gamma < end of softening)
    gam = np.array([gd["x_bar"], gd["x_bar"], gd["gamma0"] + 0.02])
    ev = np.sort(np.linalg.eigvalsh(s.nodal_stiffness(gam)))
    ref = np.sort([0.0, 3.0 * k, (2.0 * alpha + 1.0) * k])
    np.testing.assert_allclose(ev, ref, atol=1e-14)


def _brute_force_min(s):
    # scan the two free degrees of freedom (zero-sum fluctuation of the
    # elongations), then refine around the best point
    best = None
    lo, hi = -0.2, 0.25
    for it in range(6):
        ts = np.linspace(lo, hi, 181)
        for t1 in ts:
            for t2 in ts:
                gam = np.array([s.x_bar + t1, s.x_bar + t2, s.x_bar - t1 - t2])
                w = s.energy(gam)
                if best is None or w < best[0]:
                    best = (w, t1, t2)
        span = (hi - lo) / 20
        c = 0.5 * (best[1] + best[2])
        lo, hi = min(best[1], best[2]) - span, max(best[1], best[2]) + span
    w, t1, t2 = best
    return np.array([s.x_bar + t1, s.x_bar + t2, s.x_bar - t1 - t2]), w


@pytest.mark.parametrize("alpha", [1.0, -0.5, -1.0])
def test_spring_trust_region_finds_energy_minimiser(alpha):
    gd = _golden()
    s = SpringRing(k=gd["k"], gamma0=gd["gamma0"], alpha=alpha, x_bar=gd["x_bar"])
    gam_bf, w_bf = _brute_force_min(s)
    for standard in (False, True):
        gam, info = s.solve(standard=standard)
        # the compatible constraint: mean elongation stays the imposed stretch
        assert abs(gam.mean() - gd["x_bar"]) < 1e-14
        assert s.energy(gam) <= w_bf + 1e-9
        np.testing.assert_allclose(gam, gam_bf, atol=2e-3)
    if alpha < -0.5 + 1e-12:
        # non-convex cases: the damage spring ends up past the transition
        # point (the plain Newton-CG of the paper stops at the concave point)
        assert gam[2] > gd["transition_point_x0"]
