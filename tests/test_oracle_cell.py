"""Pins of the oracle's cell solver (Algorithm 2 around Algorithm 1 with the
projector of eq. proj_operator and the FAIEF ratio of eq. rho_bar).

* Homogeneous elastic cell: the fluctuation stays zero, the step converges
  without Newton iterations, Sigma = C : E.
* Homogeneous damage cell: Sigma = (1 - d(kappa(E))) C : E on the linear
  softening line.
* Laminates normal to x (grid-aligned interfaces, so the FE solution is exact):
  the classical harmonic/arithmetic means.
* Heterogeneous elasticity: the dense FE solution of
  min 1/2 <D u + E, C (D u + E)> (the projection scheme solves the same FE
  problem, Sec. 1 and 2.1).
* FAIEF: rho_bar = 1 to rounding on linear problems; third-order error against
  the exact stored energy for damage (eq. energy_estim, eq. incr_energy_func).
* The projected Hessian is the derivative of the projected residual.
* Invariants of a damage trajectory: mean strain = E, monotone history,
  0 <= d <= 1, invariance of Sigma under periodic shifts of the cell.
"""
import math

import numpy as np
import pytest

from oracle import fe, material
from oracle.solver import CellSolver, inner, INTERIOR
from synthetic import laminate_microstructure, MATRIX_DAMAGE, INCLUSION_ELASTIC
from tests.test_oracle_fe import _dense_gradient_matrix

TIGHT = {"eta_eq": 1e-13, "eta_nr": 1e-15, "eta_cg": 1e-13, "j_cg_max": 5000}
EL1 = {"kind": "elastic", "E": 1.0, "nu": 0.3, "kappa0": 0.0, "kappaf": 0.0}
EL2 = {"kind": "elastic", "E": 7.0, "nu": 0.2, "kappa0": 0.0, "kappaf": 0.0}


def _lame(m):
    E, nu = m["E"], m["nu"]
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def _C_E(m, Emac):
    lam, mu = _lame(m)
    return lam * np.trace(Emac) * np.eye(3) + 2 * mu * Emac


@pytest.mark.parametrize("element,grid", [("q1", (3, 4, 5)), ("p1pair", (6, 5))])
def test_homogeneous_elastic(element, grid):
    phase = np.zeros(grid, dtype=np.uint8)
    s = CellSolver(phase, [EL2], element)
    dE = np.array([[1e-3, 2e-4, 0], [2e-4, -3e-4, 1e-4], [0, 1e-4, 5e-4]])
    if len(grid) == 2:
        dE[2, :] = dE[:, 2] = 0.0
    r = s.apply_load_step(dE)
    assert r < 1e-14
    rep = s.solve_increment(TIGHT)
    assert rep["converged"] and rep["newton_iters"] == 0
    np.testing.assert_allclose(s.homogenized_stress(), _C_E(EL2, dE), rtol=1e-13, atol=1e-18)


def test_homogeneous_damage_on_softening_line():
    phase = np.zeros((4, 4), dtype=np.uint8)
    s = CellSolver(phase, [MATRIX_DAMAGE], "p1pair")
    e = 2.5e-3
    dE = np.zeros((3, 3))
    dE[0, 0] = e
    s.apply_load_step(dE)
    rep = s.solve_increment(TIGHT)
    assert rep["converged"]
    lam, mu = _lame(MATRIX_DAMAGE)
    kap = math.sqrt((lam + 2 * mu) * e * e / MATRIX_DAMAGE["E"])
    k0, kf = MATRIX_DAMAGE["kappa0"], MATRIX_DAMAGE["kappaf"]
    # equivalent stress on the straight softening line through (k0, E k0), (kf, 0)
    seq = MATRIX_DAMAGE["E"] * k0 * (kf - kap) / (kf - k0)
    one_minus_d = seq / (MATRIX_DAMAGE["E"] * kap)
    Sig = s.homogenized_stress()
    np.testing.assert_allclose(Sig[0, 0], one_minus_d * (lam + 2 * mu) * e, rtol=1e-12)
    np.testing.assert_allclose(Sig[2, 2], one_minus_d * lam * e, rtol=1e-12)
    np.testing.assert_allclose(s.damage(), 1.0 - one_minus_d, rtol=1e-12)


def _laminate_means(mats, frac):
    lam = np.array([_lame(m)[0] for m in mats])
    mu = np.array([_lame(m)[1] for m in mats])
    M = lam + 2 * mu
    avg = lambda v: float(np.sum(frac * v))
    Cxxxx = 1.0 / avg(1.0 / M)
    Cyyxx = avg(lam / M) / avg(1.0 / M)
    mu_xy = 1.0 / avg(1.0 / mu)
    return Cxxxx, Cyyxx, mu_xy


@pytest.mark.parametrize("element,grid", [("q1", (3, 2, 8)), ("p1pair", (3, 8))])
def test_laminate_closed_form(element, grid):
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
        rep = s.solve_increment(TIGHT)
        assert rep["converged"]
        Sig = s.homogenized_stress()
        if comp == "xx":
            np.testing.assert_allclose(Sig[0, 0], Cxxxx * 1e-3, rtol=1e-11)
            np.testing.assert_allclose(Sig[1, 1], Cyyxx * 1e-3, rtol=1e-11)
        else:
            np.testing.assert_allclose(Sig[0, 1], 2 * mu_xy * 1e-3, rtol=1e-11)


def _dense_fe_solution(phase, mats, element, dE):
    grid = phase.shape
    dim = fe.element_dim(element)
    nq = fe.shape_gradients(element).shape[0]
    D = _dense_gradient_matrix(grid, element)
    n_pts = int(np.prod(grid)) * nq
    # per-point elasticity acting on the full gradient (minor symmetries)
    C = np.zeros((n_pts * dim * dim, n_pts * dim * dim))
    flat_phase = np.repeat(phase.reshape(-1), nq)
    for p in range(n_pts):
        lam, mu = _lame(mats[flat_phase[p]])
        for i in range(dim):
            for j in range(dim):
                for k in range(dim):
                    for l in range(dim):
                        v = lam * (i == j) * (k == l) + mu * ((i == k) * (j == l) + (i == l) * (j == k))
                        C[p * dim * dim + i * dim + j, p * dim * dim + k * dim + l] = v
    Ef = np.tile(dE[:dim, :dim].reshape(-1), n_pts)
    K = D.T @ C @ D
    f = -D.T @ C @ Ef
    u, *_ = np.linalg.lstsq(K, f, rcond=None)
    return (D @ u + Ef).reshape(grid + (nq, dim, dim))


@pytest.mark.parametrize("element,grid", [("q1", (3, 2, 3)), ("p1pair", (5, 6))])
def test_heterogeneous_elastic_matches_dense_fe(element, grid):
    rng = np.random.default_rng(7)
    phase = (rng.random(grid) < 0.4).astype(np.uint8)
    mats = [EL1, EL2]
    dE = np.zeros((3, 3))
    dE[0, 0], dE[0, 1], dE[1, 0], dE[1, 1] = 1e-3, 3e-4, 3e-4, -2e-4
    s = CellSolver(phase, mats, element)
    s.apply_load_step(dE)
    rep = s.solve_increment(TIGHT)
    assert rep["converged"]
    H_ref = _dense_fe_solution(phase, mats, element, dE)
    np.testing.assert_allclose(s.H, H_ref, rtol=0, atol=1e-12 * np.abs(H_ref).max())
    # FAIEF is exact on a quadratic energy: every accepted step has rho = 1
    assert all(abs(r - 1.0) < 1e-9 for r in rep["rho"])


def test_faief_third_order_for_damage():
    rng = np.random.default_rng(8)
    grid = (4, 4)
    phase = np.zeros(grid, dtype=np.uint8)
    mf = material.MaterialField(phase, [MATRIX_DAMAGE], 2)
    H = 2.5e-3 * np.ones(grid + (2, 2, 2)) * np.array([[1.0, 0.2], [0.1, -0.3]])
    kh = mf.initial_history()
    P = rng.normal(size=H.shape) * 2e-4
    errs = []
    for t in (1.0, 0.5, 0.25):
        p = t * P
        st0 = material.evaluate(mf, H, kh)
        st1 = material.evaluate(mf, H + p, kh)
        dW_bar = 0.5 * (inner(st0["sigma"], p) + inner(st1["sigma"], p))
        dW = material.energy(mf, H + p, kh) - material.energy(mf, H, kh)
        errs.append(abs(dW_bar - dW))
    # halving the step divides the error by ~8
    assert errs[0] / errs[1] > 6.0 and errs[1] / errs[2] > 6.0


def test_projected_hessian_is_derivative_of_projected_residual():
    rng = np.random.default_rng(9)
    grid = (6, 5)
    phase = (rng.random(grid) < 0.3).astype(np.uint8)
    s = CellSolver(phase, [MATRIX_DAMAGE, INCLUSION_ELASTIC], "p1pair")
    dE = np.zeros((3, 3))
    dE[0, 0] = 2e-3
    s.apply_load_step(dE)
    u = rng.normal(size=(2,) + grid) * 1e-4
    s.H = s.H + fe.gradient(u, "p1pair")
    s._set_state(s._evaluate(s.H))
    v = rng.normal(size=(2,) + grid) * 1e-4
    X = fe.gradient(v, "p1pair")
    h = 1e-4
    gp = s.G(material.evaluate(s.mat, s.H + h * X, s.kappa_hist)["sigma"])
    gm = s.G(material.evaluate(s.mat, s.H - h * X, s.kappa_hist)["sigma"])
    fd = (gp - gm) / (2 * h)
    an = s.apply_hessian(X)
    assert np.max(np.abs(fd - an)) <= 1e-5 * np.max(np.abs(an))
    # symmetric on compatible fields
    Y = fe.gradient(rng.normal(size=(2,) + grid), "p1pair")
    assert abs(inner(Y, s.apply_hessian(X)) - inner(X, s.apply_hessian(Y))) < 1e-10 * abs(inner(Y, s.apply_hessian(X)))


def test_large_radius_gives_newton_cg():
    # convex problem, inactive trust region: every Steihaug exit is interior
    # and the first Newton step already solves the linear problem
    rng = np.random.default_rng(11)
    phase = (rng.random((4, 3, 4)) < 0.4).astype(np.uint8)
    s = CellSolver(phase, [EL1, EL2], "q1", R0=1e6, Rmax=1e7)
    dE = np.zeros((3, 3))
    dE[1, 1] = 1e-3
    s.apply_load_step(dE)
    rep = s.solve_increment(TIGHT)
    assert rep["converged"] and rep["newton_iters"] == 1
    assert rep["flags"] == [INTERIOR]


def _damage_run(phase, steps, element="p1pair"):
    s = CellSolver(phase, [MATRIX_DAMAGE, INCLUSION_ELASTIC], element)
    hist = []
    dE = np.zeros((3, 3))
    dE[0, 0] = 3e-4
    for _ in range(steps):
        s.apply_load_step(dE)
        s.solve_increment({"i_nr_max": 30, "j_cg_max": 400})
        hist.append((s.kappa_hist.copy(), s.homogenized_stress(), s.damage()))
    return s, hist


def test_damage_trajectory_invariants():
    rng = np.random.default_rng(12)
    phase = (rng.random((8, 8)) < 0.25).astype(np.uint8)
    s, hist = _damage_run(phase, 3)
    for a, b in zip(hist[:-1], hist[1:]):
        assert np.all(b[0] >= a[0])
    for _, _, d in hist:
        assert np.all(d >= 0.0) and np.all(d <= 1.0)
    # mean of the full gradient is the macroscopic strain
    np.testing.assert_allclose(s.H.mean(axis=(0, 1, 2)), s.E[:2, :2], atol=1e-15)
    # a periodic shift of the microstructure shifts the fields, not Sigma
    s2, hist2 = _damage_run(np.roll(phase, (3, 5), axis=(0, 1)), 3)
    assert hist[-1][2].max() > 0.5          # damage has localised somewhere
    for (_, S1, _), (_, S2, _) in zip(hist, hist2):
        np.testing.assert_allclose(S2, S1, rtol=1e-7, atol=1e-9 * np.abs(S1).max())


@pytest.mark.slow
def test_rounding_sensitivity_of_the_method():
    """The oracle against itself with only the summation order of its inner
    products changed: on the 3D inclusion cell the CG traces separate by more
    than 1e-2 (relative) within four load steps. This is the rounding noise
    against which a GPU/oracle difference in a stopping decision is judged."""
    import oracle.solver as S
    from synthetic import workload
    w = workload("c1_3d16", steps=4)
    orig = S.steihaug

    def run(dot):
        def st(apply_A, g, R, eta, jmax, dot_=None, log=None, **kw):
            return orig(apply_A, g, R, eta, jmax, dot=dot, log=log, **kw)
        S.steihaug = st
        try:
            o = CellSolver(w.phase, w.materials, w.element)
            traces = []
            for dE in w.load_path:
                o.apply_load_step(dE)
                log = []
                o.solve_increment(log=log)
                traces.append(np.array([e[3] for e in log if e[0] == "cg"]))
            return traces
        finally:
            S.steihaug = orig

    a = run(lambda X, Y: float(np.sum(X * Y)))
    b = run(lambda X, Y: float(np.sum((X * Y).ravel()[::-1])))
    drift = 0.0
    for ta, tb in zip(a, b):
        m = min(len(ta), len(tb))
        ok = np.isfinite(ta[:m]) & np.isfinite(tb[:m])
        if ok.any():
            drift = max(drift, float(np.max(np.abs(ta[:m][ok] - tb[:m][ok]) / np.abs(ta[:m][ok]))))
    assert drift > 1e-2, drift


def _oracle_effective_stiffness(phase, materials, strain, params):
    """Six unit load cases (Voigt xx, yy, zz, yz, xz, xy; engineering shears)."""
    voigt = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
    C = np.zeros((6, 6))
    for J, (i, j) in enumerate(voigt):
        dE = np.zeros((3, 3))
        dE[i, j] = dE[j, i] = strain if i == j else 0.5 * strain
        o = CellSolver(phase, materials, "q1")
        o.apply_load_step(dE)
        assert o.solve_increment(params)["converged"]
        S = o.homogenized_stress()
        C[:, J] = [S[a, b] for a, b in voigt] 
    return C / strain


def test_oracle_effective_stiffness_laminate_backus_and_symmetry():
    """The effective stiffness of a voxel laminate (normal x) equals the Backus
    averages in all 36 entries; that of a random two-phase elastic cell is
    symmetric positive definite and lies between the Reuss and Voigt bounds."""
    from synthetic import laminate_microstructure
    m1 = {"kind": "elastic", "E": 1.0, "nu": 0.3, "kappa0": 0.0, "kappaf": 0.0}
    m2 = {"kind": "elastic", "E": 7.0, "nu": 0.2, "kappa0": 0.0, "kappaf": 0.0}
    tight = {"eta_eq": 1e-12, "eta_nr": 1e-14, "eta_cg": 1e-10}
    layers = np.array([0, 0, 1, 1, 1, 0, 1, 0], dtype=np.uint8)
    shape = (4, 4, 8)
    C = _oracle_effective_stiffness(laminate_microstructure(shape, layers), [m1, m2], 1e-4, tight)
    f = np.array([np.mean(layers == 0), np.mean(layers == 1)])
    lam = np.array([m["E"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"])) for m in (m1, m2)])
    mu = np.array([m["E"] / (2 * (1 + m["nu"])) for m in (m1, m2)])
    M = lam + 2 * mu
    avg = lambda x: float(np.sum(f * x))
    Cnn = 1.0 / avg(1.0 / M)
    ref = np.zeros((6, 6))
    ref[0, 0] = Cnn
    ref[0, 1] = ref[1, 0] = ref[0, 2] = ref[2, 0] = avg(lam / M) * Cnn
    ref[1, 1] = ref[2, 2] = avg(M - lam ** 2 / M) + avg(lam / M) ** 2 * Cnn
    ref[1, 2] = ref[2, 1] = avg(lam - lam ** 2 / M) + avg(lam / M) ** 2 * Cnn
    ref[3, 3] = avg(mu)
    ref[4, 4] = ref[5, 5] = 1.0 / avg(1.0 / mu)
    assert np.abs(C - ref).max() < 1e-9 * np.abs(ref).max()
    # random two-phase cell
    rng = np.random.default_rng(5)
    phase = (rng.random((4, 4, 4)) < 0.4).astype(np.uint8)
    C = _oracle_effective_stiffness(phase, [m1, m2], 1e-4, tight)
    assert np.abs(C - C.T).max() < 1e-10 * np.abs(C).max()
    ev = np.linalg.eigvalsh(0.5 * (C + C.T))
    assert ev.min() > 0
    # Voigt / Reuss bounds on the bulk-like combination e.C.e for e = (1,1,1,0,0,0)
    def iso(m):
        l = m["E"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"]))
        u = m["E"] / (2 * (1 + m["nu"]))
        return np.array([[l + 2 * u, l, l, 0, 0, 0], [l, l + 2 * u, l, 0, 0, 0],
                         [l, l, l + 2 * u, 0, 0, 0], [0, 0, 0, u, 0, 0], [0, 0, 0, 0, u, 0],
                         [0, 0, 0, 0, 0, u]])
    fv = np.array([np.mean(phase == 0), np.mean(phase == 1)])
    Cv = fv[0] * iso(m1) + fv[1] * iso(m2)
    Cr = np.linalg.inv(fv[0] * np.linalg.inv(iso(m1)) + fv[1] * np.linalg.inv(iso(m2)))
    e = np.array([1.0, 1, 1, 0, 0, 0])
    assert e @ Cr @ e - 1e-12 <= e @ C @ e <= e @ Cv @ e + 1e-12


# ---- eigenstrain (Algorithm 2: eps_eval = eps + eps_eig) -----------------------

def test_oracle_eigenstrain_homogeneous_cell():
    """Every point carries eps_eig and E = 0: no fluctuation, Sigma = C : eps_eig."""
    m = {"kind": "elastic", "E": 3.0, "nu": 0.25, "kappa0": 0.0, "kappaf": 0.0}
    eig = np.array([[1e-3, 2e-4, 0.0], [2e-4, -5e-4, 1e-4], [0.0, 1e-4, 3e-4]])
    o = CellSolver(np.zeros((4, 4, 4), np.uint8), [m], "q1")
    o.set_eigenstrain(0, eig)
    r = o.apply_load_step(np.zeros((3, 3)))
    assert r < 1e-14
    lam, mu = 3.0 * 0.25 / (1.25 * 0.5), 3.0 / 2.5
    ref = lam * np.trace(eig) * np.eye(3) + 2 * mu * eig
    assert np.abs(o.homogenized_stress() - ref).max() < 1e-15


def test_oracle_eigenstrain_laminate_closed_form():
    """A laminate (normal x) whose phase 1 expands by theta I at E = 0: the
    in-plane strains vanish in every layer, the normal strains average to
    zero and carry one normal stress, sigma_xx = <b/M>/<1/M> with
    b = (3 lam + 2 mu) theta, M = lam + 2 mu; sigma_yy = sigma_zz =
    <lam eps_xx + b>."""
    from synthetic import laminate_microstructure
    m0 = {"kind": "elastic", "E": 1.0, "nu": 0.3, "kappa0": 0.0, "kappaf": 0.0}
    m1 = {"kind": "elastic", "E": 7.0, "nu": 0.2, "kappa0": 0.0, "kappaf": 0.0}
    theta = 2e-3
    layers = np.array([0, 0, 1, 1, 1, 0, 1, 0], dtype=np.uint8)
    phase = laminate_microstructure((4, 4, 8), layers)
    o = CellSolver(phase, [m0, m1], "q1")
    o.set_eigenstrain(1, theta * np.eye(3))
    o.apply_load_step(np.zeros((3, 3)))
    res = o.solve_increment({"eta_eq": 1e-12, "eta_nr": 1e-14, "eta_cg": 1e-10})
    assert res["converged"]
    assert all(abs(r - 1.0) < 1e-8 for r in res["rho"])        # a linear problem
    f = np.array([np.mean(layers == 0), np.mean(layers == 1)])
    lam = np.array([m["E"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"])) for m in (m0, m1)])
    mu = np.array([m["E"] / (2 * (1 + m["nu"])) for m in (m0, m1)])
    M = lam + 2 * mu
    b = (3 * lam + 2 * mu) * np.array([0.0, theta])
    sxx = np.sum(f * b / M) / np.sum(f / M)
    exx = (sxx - b) / M
    syy = np.sum(f * (lam * exx + b))
    S = o.homogenized_stress()
    scale = abs(syy)
    assert abs(S[0, 0] - sxx) < 1e-10 * scale
    assert abs(S[1, 1] - syy) < 1e-10 * scale and abs(S[2, 2] - syy) < 1e-10 * scale
    assert np.abs(S - np.diag(np.diag(S))).max() < 1e-10 * scale


def test_oracle_restore_continues_the_path():
    """checkpoint() / restore() resume a load path: the steps after a restore
    reach the results of the uninterrupted run (the displacement is recovered
    through the Green's function, so to rounding)."""
    from synthetic import workload
    w = workload("c1_3d8", steps=3)
    a = CellSolver(w.phase, w.materials, "q1")
    for dE in w.load_path[:2]:
        a.apply_load_step(dE)
        a.solve_increment()
    ck = a.checkpoint()
    b = CellSolver(w.phase, w.materials, "q1")
    b.restore(ck)
    for s in (a, b):
        s.apply_load_step(w.load_path[2])
        assert s.solve_increment()["converged"]
    Sa, Sb = a.homogenized_stress(), b.homogenized_stress()
    assert np.linalg.norm(Sa - Sb) <= 1e-10 * np.linalg.norm(Sa)
    assert np.max(np.abs(a.damage() - b.damage())) <= 1e-10
