"""Pins of the L-BFGS oracle (the quasi-Newton use of the approximate energy
increment that Sec. 2.2 proposes).

* The two-loop recursion equals the explicit BFGS update of a dense
  inverse-Hessian matrix built from the same pairs.
* On an elastic (quadratic) cell the approximate increment (eq.
  incr_energy_func) equals the exact change of the stored energy, so the
  Armijo test sees the true energy.
* Laminates: the classical harmonic / arithmetic means (as for Newton).
* Heterogeneous elasticity: the same equilibrium as the trust-region Newton
  solver (the elastic equilibrium is unique).
* A damage cell: every increment converges to an equilibrium, with the mean
  strain equal to E and 0 <= d <= 1.
"""
import numpy as np
import pytest

from oracle import quasi_newton as qn
from oracle.solver import CellSolver, inner
from synthetic import laminate_microstructure, inclusion_microstructure, MATRIX_DAMAGE, INCLUSION_ELASTIC
from tests.test_oracle_cell import EL1, EL2, _laminate_means, TIGHT

QN_TIGHT = {"eta_eq": 1e-12, "eta_nr": 1e-15, "i_qn_max": 2000}


def test_two_loop_matches_dense_bfgs_update():
    rng = np.random.default_rng(0)
    n, m = 9, 5
    B = rng.normal(size=(n, n))
    A = B @ B.T + n * np.eye(n)
    pairs = []
    for _ in range(m):
        s = rng.normal(size=n)
        y = A @ s
        pairs.append((s, y, 1.0 / float(s @ y)))
    gamma = 0.37
    H = gamma * np.eye(n)
    I = np.eye(n)
    for s, y, rho in pairs:
        H = (I - rho * np.outer(s, y)) @ H @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
    q = rng.normal(size=n)
    r = qn.two_loop(q, pairs, gamma, lambda a, b: float(a @ b))
    np.testing.assert_allclose(r, H @ q, rtol=1e-12, atol=1e-14)
    # the secant equation of the newest pair
    s, y, _ = pairs[-1]
    np.testing.assert_allclose(qn.two_loop(y, pairs, gamma, lambda a, b: float(a @ b)), s,
                               rtol=1e-10)


@pytest.mark.parametrize("element,grid", [("q1", (4, 3, 5)), ("p1pair", (6, 5))])
def test_energy_increment_is_exact_for_elasticity(element, grid):
    rng = np.random.default_rng(1)
    phase = (rng.random(grid) < 0.4).astype(np.uint8)
    cs = CellSolver(phase, [EL1, EL2], element)
    dE = np.zeros((3, 3))
    dE[0, 0] = 1e-3
    cs.apply_load_step(dE)
    H = cs.H + 1e-4 * rng.normal(size=cs.H.shape)
    v = 1e-4 * rng.normal(size=cs.H.shape)
    st0 = cs._evaluate(H)
    st1 = cs._evaluate(H + v)
    dW = qn.energy_increment(st0["sigma"], st1["sigma"], v)
    exact = qn.exact_energy(cs, H + v) - qn.exact_energy(cs, H)
    assert abs(dW - exact) < 1e-11 * abs(exact)


@pytest.mark.parametrize("element,grid", [("q1", (3, 2, 8)), ("p1pair", (3, 8))])
def test_lbfgs_laminate_closed_form(element, grid):
    layers = np.array([0, 0, 1, 1, 1, 0, 1, 0], dtype=np.uint8)
    phase = laminate_microstructure(grid, layers)
    mats = [EL1, EL2]
    frac = np.array([np.mean(layers == 0), np.mean(layers == 1)])
    Cxxxx, Cyyxx, mu_xy = _laminate_means(mats, frac)
    for comp in ("xx", "xy"):
        s = CellSolver(phase, mats, element)
        dE = np.zeros((3, 3))
        if comp == "xx":
            dE[0, 0] = 1e-3
        else:
            dE[0, 1] = dE[1, 0] = 1e-3
        s.apply_load_step(dE)
        rep = qn.solve_increment_lbfgs(s, QN_TIGHT)
        assert rep["converged"], rep
        Sig = s.homogenized_stress()
        if comp == "xx":
            np.testing.assert_allclose(Sig[0, 0], Cxxxx * 1e-3, rtol=1e-10)
            np.testing.assert_allclose(Sig[1, 1], Cyyxx * 1e-3, rtol=1e-10)
        else:
            np.testing.assert_allclose(Sig[0, 1], 2 * mu_xy * 1e-3, rtol=1e-10)


@pytest.mark.parametrize("element,grid", [("q1", (6, 5, 4)), ("p1pair", (12, 10))])
def test_lbfgs_matches_newton_on_heterogeneous_elasticity(element, grid):
    rng = np.random.default_rng(2)
    phase = (rng.random(grid) < 0.35).astype(np.uint8)
    dE = np.zeros((3, 3))
    dE[0, 0] = 1e-3
    dE[0, 1] = dE[1, 0] = 4e-4
    a = CellSolver(phase, [EL1, EL2], element)
    a.apply_load_step(dE)
    assert a.solve_increment(TIGHT)["converged"]
    b = CellSolver(phase, [EL1, EL2], element)
    b.apply_load_step(dE)
    rep = qn.solve_increment_lbfgs(b, QN_TIGHT)
    assert rep["converged"], rep
    assert rep["iters"] > 1
    np.testing.assert_allclose(b.homogenized_stress(), a.homogenized_stress(), rtol=1e-9,
                               atol=1e-15)
    np.testing.assert_allclose(b.H, a.H, rtol=0, atol=1e-9 * np.abs(a.H).max())


def test_lbfgs_damage_cell_reaches_equilibria():
    phase, _ = inclusion_microstructure((8, 8, 8), 1.0, 2.0, 0.25, 3)
    mats = [dict(MATRIX_DAMAGE), dict(INCLUSION_ELASTIC)]
    s = CellSolver(phase, mats, "q1")
    dE = np.zeros((3, 3))
    dE[0, 0] = 4e-4
    for k in range(5):
        s.apply_load_step(dE)
        rep = qn.solve_increment_lbfgs(s, {"eta_eq": 1e-8, "eta_nr": 1e-12})
        assert rep["converged"], (k, rep)
        assert s.r_eq <= 1e-8 or rep["r_nr"] <= 1e-12
        d = s.damage()
        assert d.min() >= 0.0 and d.max() <= 1.0
        # the fluctuation has zero mean: the mean strain is E
        np.testing.assert_allclose(s.H.mean(axis=(0, 1, 2, 3)), s.E, atol=1e-12)
    assert s.damage().max() > 0.0        # the path reaches the damage regime
