"""Pins of the displacement-space oracle (oracle/uspace.py) against the
strain-space oracle and the closed forms it is built on.

* Its closed-form FE-Laplacian symbol equals sum |Dhat|^2 computed from the
  element's shape functions (projection.py's denominator of eq.
  proj_operator).
* D (L^+ K d) equals the strain-space projected Hessian G : B : (D d) (eq.
  project_stress_linear) at a softening state, in 3D and 2D, to 1e-12.
* The slab split is invisible: one slab and several give the same result to
  rounding, and K d is the adjoint pairing of the tangent, d.Kd = (Dd):B:(Dd).
"""
import numpy as np
import pytest

from oracle import fe, material
from oracle.projection import Projector
from oracle.uspace import UOperator, laplacian_symbol
from synthetic import MATRIX_DAMAGE, INCLUSION_ELASTIC, MATRIX_TENSILE


@pytest.mark.parametrize("grid,el", [((4, 6, 8), "q1"), ((6, 10), "p1pair"), ((5, 3, 4), "q1")])
def test_laplacian_symbol_is_sum_of_derivative_symbols(grid, el):
    S = laplacian_symbol(grid, el)
    ref = Projector(grid, el).S
    assert np.max(np.abs(S - ref)) < 1e-12 * np.max(ref)


def _state(grid, seed, mats):
    rng = np.random.default_rng(seed)
    phase = (rng.random(grid) < 0.3).astype(np.uint8)
    dim = len(grid)
    E = np.zeros((3, 3))
    E[0, 0] = 1.5e-3
    E[1, 1] = -2e-4
    E[0, 1] = E[1, 0] = 3e-4
    u = 4e-4 * rng.normal(size=(dim,) + grid)
    return phase, E, u, rng


@pytest.mark.parametrize("grid,el,mats", [
    ((8, 6, 10), "q1", [MATRIX_DAMAGE, INCLUSION_ELASTIC]),
    ((6, 8, 4), "q1", [MATRIX_TENSILE, INCLUSION_ELASTIC]),
    ((12, 8), "p1pair", [MATRIX_DAMAGE, INCLUSION_ELASTIC])])
def test_projected_hessian_equals_strain_space_oracle(grid, el, mats):
    phase, E, u, rng = _state(grid, 1, mats)
    nq = 8 if el == "q1" else 2
    mf = material.MaterialField(phase, mats, nq)
    kh = mf.initial_history()
    H = fe.gradient(u, el) + E[:len(grid), :len(grid)]
    st = material.evaluate(mf, H, kh)
    assert np.mean(st["cprime"] > 0) > 0.05
    d = rng.normal(size=(len(grid),) + grid)
    ref = Projector(grid, el)(material.apply_tangent(mf, st, fe.gradient(d, el)))
    op = UOperator(phase, mats, el, E, u, kh, workers=4, slabs=3)
    got = fe.gradient(op.apply(d), el)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_slabs_and_threads_do_not_change_the_result():
    grid = (9, 8, 6)
    mats = [MATRIX_DAMAGE, INCLUSION_ELASTIC]
    phase, E, u, rng = _state(grid, 2, mats)
    kh = material.MaterialField(phase, mats, 8).initial_history()
    d = rng.normal(size=(3,) + grid)
    a = UOperator(phase, mats, "q1", E, u, kh, workers=1, slabs=1)
    b = UOperator(phase, mats, "q1", E, u, kh, workers=4, slabs=5)
    Ka, Kb = a.stiffness(d), b.stiffness(d)
    assert np.max(np.abs(Ka - Kb)) <= 1e-14 * np.max(np.abs(Ka))
    mf = material.MaterialField(phase, mats, 8)
    st = material.evaluate(mf, fe.gradient(u, "q1") + E, kh)
    Dd = fe.gradient(d, "q1")
    dKd = np.sum(Dd * material.apply_tangent(mf, st, Dd))
    assert abs(np.sum(d * Kb) - dKd) <= 1e-12 * abs(dKd)
