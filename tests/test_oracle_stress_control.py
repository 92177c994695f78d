"""Pins of the oracle's mean-stress control (Sec. 3.3 holds the mean stress
of its cell at zero; the modified projector G_M = G + M of oracle/solver.py).

* G_M is an orthogonal projector: idempotent and self-adjoint in the plain
  point sum, with free normal and shear components.
* A homogeneous elastic cell under uniaxial stress (E_xx prescribed, the
  other normal components free): the textbook uniaxial-stress response,
  sigma_xx = E e, E_yy = E_zz = -nu e, in 3D; in 2D plane strain (E_yy free)
  sigma_xx = E e / (1 - nu^2), E_yy = -nu e / (1 - nu).
* A laminate (layers normal to x) of two phases with isotropic eigenstrains
  under free expansion (all normal components free, shears held at zero):
  zero mean stress, E_yy = E_zz = eta and E_xx = <eps_xx> from the closed
  form of the layered solution (sigma_xx = 0 in every layer, in-plane strain
  eta shared, <sigma_yy> = 0). Algorithm 2 adds the eigenstrain to the strain
  the law sees, so a positive one makes a free phase contract.
* A damaging cell under free expansion converges with zero mean stress in
  every free component.
"""
import numpy as np
import pytest

from oracle import material
from oracle.solver import CellSolver
from synthetic import laminate_microstructure, workload

EL1 = {"kind": "elastic", "E": 1.0, "nu": 0.3, "kappa0": 0.0, "kappaf": 0.0}
EL2 = {"kind": "elastic", "E": 7.0, "nu": 0.2, "kappa0": 0.0, "kappaf": 0.0}
TIGHT = {"eta_eq": 1e-12, "eta_nr": 1e-14, "eta_cg": 1e-12}


def test_modified_projector_is_an_orthogonal_projector():
    rng = np.random.default_rng(0)
    phase = (rng.random((4, 6, 5)) < 0.4).astype(np.uint8)
    o = CellSolver(phase, [EL1, EL2], "q1")
    free = np.zeros((3, 3), dtype=bool)
    free[1, 1] = free[2, 2] = free[0, 2] = free[2, 0] = True
    o.set_mean_stress_control(free)
    X = rng.normal(size=o.H.shape)
    Y = rng.normal(size=o.H.shape)
    PX = o.project(X)
    assert np.max(np.abs(o.project(PX) - PX)) < 1e-12 * np.max(np.abs(PX))
    assert abs(np.sum(PX * Y) - np.sum(X * o.project(Y))) < 1e-11 * np.sqrt(np.sum(X * X) * np.sum(Y * Y))
    # the uniform part lives exactly in the free components, symmetric
    m = PX.mean(axis=(0, 1, 2, 3))
    assert abs(m[0, 0]) < 1e-13 and abs(m[0, 1]) < 1e-13 and abs(m[1, 2]) < 1e-13
    assert abs(m[0, 2] - m[2, 0]) < 1e-13 and abs(m[1, 1] - X.mean(axis=(0, 1, 2, 3))[1, 1]) < 1e-12


@pytest.mark.parametrize("grid,el", [((4, 4, 4), "q1"), ((6, 6), "p1pair")])
def test_homogeneous_uniaxial_stress(grid, el):
    o = CellSolver(np.zeros(grid, np.uint8), [EL2], el)
    free = np.zeros((3, 3), dtype=bool)
    free[1, 1] = True
    if len(grid) == 3:
        free[2, 2] = True
    o.set_mean_stress_control(free)
    e = 1e-3
    dE = np.zeros((3, 3))
    dE[0, 0] = e
    o.apply_load_step(dE)
    rep = o.solve_increment(TIGHT)
    assert rep["converged"]
    S = o.homogenized_stress()
    Em, nu = EL2["E"], EL2["nu"]
    if len(grid) == 3:
        assert abs(S[0, 0] - Em * e) < 1e-10 * Em * e
        assert abs(o.E[1, 1] + nu * e) < 1e-10 * e and abs(o.E[2, 2] + nu * e) < 1e-10 * e
        assert abs(S[1, 1]) < 1e-10 * Em * e and abs(S[2, 2]) < 1e-10 * Em * e
    else:
        assert abs(S[0, 0] - Em * e / (1 - nu ** 2)) < 1e-10 * Em * e
        assert abs(o.E[1, 1] + nu * e / (1 - nu)) < 1e-10 * e
        assert abs(S[1, 1]) < 1e-10 * Em * e


def test_free_expansion_laminate_closed_form():
    layers = np.array([0, 0, 1, 1, 1, 0, 1, 0], dtype=np.uint8)
    shape = (4, 4, 8)
    phase = laminate_microstructure(shape, layers)
    th = np.array([0.0, 2e-3])
    mats = [EL1, dict(EL2, eig=th[1] * np.eye(3))]
    o = CellSolver(phase, mats, "q1")
    free = np.eye(3, dtype=bool)
    o.set_mean_stress_control(free)
    o.apply_load_step(np.zeros((3, 3)))
    rep = o.solve_increment(TIGHT)
    assert rep["converged"]
    f = np.array([np.mean(layers == 0), np.mean(layers == 1)])
    lam, mu = material.lame(np.array([EL1["E"], EL2["E"]]), np.array([EL1["nu"], EL2["nu"]]))
    M = lam + 2 * mu
    b = (3 * lam + 2 * mu) * th
    # the law sees eps + eps_eig (Algorithm 2), so sigma = C : eps + b I:
    # sigma_xx = M eps_xx + 2 lam eta + b = 0 in every layer, <sigma_yy> = 0
    eta = -np.sum(f * b * (1 - lam / M)) / np.sum(f * (2 * lam + 2 * mu - 2 * lam ** 2 / M))
    exx = -np.sum(f * (b + 2 * lam * eta) / M)
    S = o.homogenized_stress()
    scale = np.max(b)
    assert np.max(np.abs(S)) < 1e-10 * scale
    assert abs(o.E[1, 1] - eta) < 1e-10 * abs(eta) and abs(o.E[2, 2] - eta) < 1e-10 * abs(eta)
    assert abs(o.E[0, 0] - exx) < 1e-10 * abs(exx)
    assert abs(o.E[0, 1]) < 1e-15 and abs(o.E[1, 2]) < 1e-15


def test_free_expansion_of_a_damaging_cell():
    w = workload("gel_3d8", steps=4)
    o = CellSolver(w.phase, w.materials, "q1")
    o.set_mean_stress_control(np.eye(3, dtype=bool))
    for n, dE in enumerate(w.load_path):
        o.set_eigenstrain(w.eig_phase, w.eig_path[n])
        o.apply_load_step(dE)
        rep = o.solve_increment({"i_nr_max": 200})
        assert rep["converged"], n
        S = o.homogenized_stress()
        ns = np.sqrt(np.mean(np.sum(o.sigma * o.sigma, axis=(-2, -1))))
        assert np.max(np.abs(np.diag(S))) <= 1e-7 * ns, (n, S)
    # the eigenstrain is added to the strain the law sees: the free cell contracts
    assert o.E[0, 0] < 0 and o.E[1, 1] < 0 and o.E[2, 2] < 0
