"""GPU parity of whole load steps (Algorithm 2 around Algorithm 1) against the
strain-space oracle, in lockstep: the same Newton decisions (exit flags, CG
iteration counts, accept/reject) and, per step, the homogenized stress and the
gradient, stress and damage fields to a relative 1e-10 in FP64.

Closed forms first (homogeneous cell, laminate), then trajectories of the two
benchmark workloads: the 2D 32x32 plane-strain cell with 20 load steps (full
path) and the 3D inclusion cell at 16^3 (same recipe as the 64^3 workload).
"""
import numpy as np
import pytest

from oracle.solver import CellSolver
from synthetic import workload, laminate_microstructure
from tests.gpu_util import require_gpu, announce, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-10
EL1 = {"kind": "elastic", "E": 1.0, "nu": 0.3}
EL2 = {"kind": "elastic", "E": 7.0, "nu": 0.2}


def _pair(shape, phase, mats, R0=None, Rmax=None):
    from paper_2207_10657_amd import Solver
    el = "q1" if len(shape) == 3 else "p1pair"
    g = Solver(shape, el)
    g.setup(phase, mats)
    o = CellSolver(phase, [dict(m, kappa0=m.get("kappa0", 0.0), kappaf=m.get("kappaf", 0.0))
                           for m in mats], el, R0=R0, Rmax=Rmax)
    return g, o


@pytest.mark.parametrize("shape", [(6, 8, 4), (16, 16)])
def test_laminate_closed_form_on_gpu(shape):
    require_gpu()
    announce("laminate", shape)
    base = [0, 0, 1, 1, 1, 0, 1, 0]
    layers = np.array((base * 4)[: shape[-1]], dtype=np.uint8)
    phase = laminate_microstructure(shape, layers)
    g, _ = _pair(shape, phase, [EL1, EL2])
    dE = np.zeros((3, 3))
    dE[0, 0] = 1e-3
    g.apply_load_step(dE)
    rep = g.solve_increment({"eta_eq": 1e-12, "eta_nr": 1e-14, "eta_cg": 1e-12})
    assert rep["converged"]
    lam = np.array([m["E"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"])) for m in (EL1, EL2)])
    mu = np.array([m["E"] / (2 * (1 + m["nu"])) for m in (EL1, EL2)])
    frac = np.array([np.mean(layers == 0), np.mean(layers == 1)])
    M = lam + 2 * mu
    Cxxxx = 1.0 / np.sum(frac / M)
    Cyyxx = np.sum(frac * lam / M) * Cxxxx
    S = g.homogenized_stress()
    assert abs(S[0, 0] - Cxxxx * 1e-3) < 1e-10 * Cxxxx * 1e-3
    assert abs(S[1, 1] - Cyyxx * 1e-3) < 1e-10 * Cyyxx * 1e-3


def test_homogeneous_cell_on_gpu():
    require_gpu()
    announce("homogeneous")
    shape = (8, 8, 8)
    g, _ = _pair(shape, np.zeros(shape, np.uint8), [EL2])
    dE = np.array([[1e-3, 2e-4, 0], [2e-4, -3e-4, 1e-4], [0, 1e-4, 5e-4]])
    g.apply_load_step(dE)
    rep = g.solve_increment()
    assert rep["converged"] and rep["newton_iters"] == 0
    lam = 7.0 * 0.2 / (1.2 * 0.6)
    mu = 7.0 / 2.4
    ref = lam * np.trace(dE) * np.eye(3) + 2 * mu * dE
    assert rel_err(g.homogenized_stress(), ref) < 1e-13


def _lockstep(name, steps, params=None):
    w = workload(name, steps=steps)
    g, o = _pair(w.shape, w.phase, w.materials)
    results = []
    for n, dE in enumerate(w.load_path):
        announce(name, "step", n)
        g.apply_load_step(dE)
        o.apply_load_step(dE)
        rg = g.solve_increment(params)
        ro = o.solve_increment(params)
        glog = g.newton_log()
        results.append((n, rg, ro, glog))
        # identical decisions
        assert [r["flag"] for r in glog] == ro["flags"], (n, [r["flag"] for r in glog], ro["flags"])
        assert [r["cg_iters"] for r in glog] == ro["cg_per_newton"], n
        assert rg["converged"] == ro["converged"], n
        assert rg["rejected"] == ro["rejected"], n
        # results
        Sg, So = g.homogenized_stress(), o.homogenized_stress()
        assert rel_err(Sg, So) < TOL or np.abs(Sg - So).max() < 1e-14 * max(np.abs(So).max(), 1e-30) + 1e-22, (n, Sg, So)
        assert rel_err(g.gradient(), o.H) < TOL, n
        dg, do = g.damage(), o.damage()
        if np.linalg.norm(do) > 0:
            assert rel_err(dg, do) < TOL, n
        else:
            assert np.abs(dg).max() < TOL, n
    return results


def test_lockstep_2d_workload_full_path():
    """2D 32x32, P1 triangles, 20 uniaxial steps to 0.5% (the small workload)."""
    require_gpu()
    _lockstep("c0_2d32", None)


def test_lockstep_3d_workload_16():
    """3D Q1 inclusion cell at 16^3, first 8 steps of the 0.6% path."""
    require_gpu()
    _lockstep("c1_3d16", 8)
