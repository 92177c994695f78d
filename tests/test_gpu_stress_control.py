"""Mean-stress control on the GPU (Sec. 3.3: zero mean stress through the
modified projector G + M; hfe_set_mean_stress_control) against closed forms
and the oracle (oracle/solver.py, pinned in test_oracle_stress_control.py):

* a homogeneous cell under uniaxial stress and a free-expansion laminate
  with eigenstrains: the closed forms at 1e-10;
* an elastic inclusion cell with all six components free under an
  eigenstrain, with Powell's reset forced after every CG step (the restart
  path recomputes the uniform part of the residual on the host): the
  oracle's stress, strain and macroscopic strain at 1e-10;
* the expanding-site workload under free expansion, each load step from the
  oracle's state: the same Newton decisions (or a certified rounding tie)
  and the results at the parity bar.
"""
import copy

import numpy as np
import pytest

from oracle import material
from oracle.solver import CellSolver
from synthetic import laminate_microstructure, workload
from tests.gpu_util import require_gpu, announce, rel_err
from tests.oracle_rounding import step_outcome

pytestmark = pytest.mark.gpu

EL1 = {"kind": "elastic", "E": 1.0, "nu": 0.3, "kappa0": 0.0, "kappaf": 0.0}
EL2 = {"kind": "elastic", "E": 7.0, "nu": 0.2, "kappa0": 0.0, "kappaf": 0.0}
TIGHT = {"eta_eq": 1e-12, "eta_nr": 1e-14, "eta_cg": 1e-12}


def _solver(shape, phase, mats):
    from paper_2207_10657_amd import Solver
    g = Solver(shape, "q1")
    g.setup(phase, mats)
    return g


def test_uniaxial_stress_of_a_homogeneous_cell():
    require_gpu()
    announce("stress control: uniaxial stress")
    shape = (4, 4, 8)
    g = _solver(shape, np.zeros(shape, np.uint8), [EL2])
    free = np.zeros((3, 3), dtype=bool)
    free[1, 1] = free[2, 2] = True
    g.set_mean_stress_control(free)
    e = 1e-3
    dE = np.zeros((3, 3))
    dE[0, 0] = e
    g.apply_load_step(dE)
    rep = g.solve_increment(TIGHT)
    assert rep["converged"]
    S, E = g.homogenized_stress(), g.get_state()["E"]
    Em, nu = EL2["E"], EL2["nu"]
    assert abs(S[0, 0] - Em * e) < 1e-10 * Em * e
    assert abs(S[1, 1]) < 1e-10 * Em * e and abs(S[2, 2]) < 1e-10 * Em * e
    assert abs(E[1, 1] + nu * e) < 1e-10 * e and abs(E[2, 2] + nu * e) < 1e-10 * e


def test_free_expansion_laminate():
    require_gpu()
    announce("stress control: free-expansion laminate")
    layers = np.array([0, 0, 1, 1, 1, 0, 1, 0], dtype=np.uint8)
    shape = (4, 4, 8)
    phase = laminate_microstructure(shape, layers)
    th = np.array([0.0, 2e-3])
    g = _solver(shape, phase, [EL1, dict(EL2, eig=th[1] * np.eye(3))])
    g.set_mean_stress_control(np.eye(3, dtype=bool))
    g.apply_load_step(np.zeros((3, 3)))
    rep = g.solve_increment(TIGHT)
    assert rep["converged"]
    f = np.array([np.mean(layers == 0), np.mean(layers == 1)])
    lam, mu = material.lame(np.array([EL1["E"], EL2["E"]]), np.array([EL1["nu"], EL2["nu"]]))
    M = lam + 2 * mu
    b = (3 * lam + 2 * mu) * th
    eta = -np.sum(f * b * (1 - lam / M)) / np.sum(f * (2 * lam + 2 * mu - 2 * lam ** 2 / M))
    exx = -np.sum(f * (b + 2 * lam * eta) / M)
    S, E = g.homogenized_stress(), g.get_state()["E"]
    assert np.max(np.abs(S)) < 1e-10 * np.max(b)
    assert abs(E[1, 1] - eta) < 1e-10 * abs(eta) and abs(E[2, 2] - eta) < 1e-10 * abs(eta)
    assert abs(E[0, 0] - exx) < 1e-10 * abs(exx)


def test_all_components_free_with_resets_against_oracle():
    require_gpu()
    announce("stress control: six free components, reset after every CG step")
    rng = np.random.default_rng(4)
    shape = (6, 8, 4)
    phase = (rng.random(shape) < 0.35).astype(np.uint8)
    eig = np.array([[1.0, 0.4, -0.2], [0.4, -0.5, 0.3], [-0.2, 0.3, 0.7]]) * 1e-3
    mats = [EL1, dict(EL2, eig=eig)]
    g = _solver(shape, phase, mats)
    o = CellSolver(phase, mats, "q1")
    free = np.ones((3, 3), dtype=bool)
    g.set_mean_stress_control(free)
    o.set_mean_stress_control(free)
    dE = np.zeros((3, 3))
    g.apply_load_step(dE)
    o.apply_load_step(dE)
    prm = {"restart": -1.0, "j_cg_max": 60, "eta_cg": 1e-10, "eta_eq": 1e-10, "i_nr_max": 200}
    rg = g.solve_increment(prm)
    ro = o.solve_increment(prm)
    print("[stress] six free: Newton %d/%d, CG %d/%d, restarts %d/%d"
          % (rg["newton_iters"], ro["newton_iters"], rg["cg_iters"], ro["cg_iters"],
             rg["restarts"], ro["restarts"]), flush=True)
    assert rg["converged"] and ro["converged"]
    assert rg["restarts"] > 0 and rg["restarts"] == ro["restarts"]
    assert [r["flag"] for r in g.newton_log()] == ro["flags"]
    scale = np.max(np.abs(eig)) * 10.0
    assert np.max(np.abs(g.homogenized_stress() - o.homogenized_stress())) < 1e-10 * scale
    assert np.max(np.abs(g.get_state()["E"] - o.E)) < 1e-10 * np.max(np.abs(o.E))
    assert rel_err(g.gradient(), o.H) < 1e-10


def test_free_expansion_of_the_expanding_site_workload_against_oracle():
    require_gpu()
    w = workload("gel_3d16", steps=4)
    g = _solver(w.shape, w.phase, w.materials)
    o = CellSolver(w.phase, w.materials, "q1")
    g.set_mean_stress_control(np.eye(3, dtype=bool))
    o.set_mean_stress_control(np.eye(3, dtype=bool))
    for n, dE in enumerate(w.load_path):
        announce("stress control: gel_3d16 free expansion, step", n)
        if n > 0:
            ck = o.checkpoint()
            g.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
        g.set_eigenstrain(w.eig_phase, w.eig_path[n])
        o.set_eigenstrain(w.eig_phase, w.eig_path[n])
        g.apply_load_step(dE)
        o.apply_load_step(dE)
        o_start = copy.deepcopy(o)
        olog = []
        rg = g.solve_increment()
        ro = o.solve_increment(log=olog)
        lam, mu = material.lame(10.0, 0.3)
        eig = w.eig_path[n]
        scale = np.linalg.norm(lam * np.trace(eig) * np.eye(3) + 2 * mu * eig)
        dS = np.linalg.norm(g.homogenized_stress() - o.homogenized_stress()) / scale
        dE_rel = np.max(np.abs(g.get_state()["E"] - o.E)) / max(np.max(np.abs(o.E)), 1e-300)
        dd = float(np.abs(g.damage() - o.damage()).max())
        dH = rel_err(g.gradient(), o.H)
        same, certified, what = step_outcome(g, rg, o_start, ro, olog)   # may restart g
        print("[stress] gel free expansion step %d: Newton %d/%d, %s, |dSigma|/scale %.2e, "
              "E %.2e, damage %.2e, grad %.2e, E_xx %.3e, max damage %.3f"
              % (n, rg["newton_iters"], ro["newton_iters"], what, dS, dE_rel, dd, dH, o.E[0, 0],
                 float(o.damage().max())), flush=True)
        assert rg["converged"] and ro["converged"], n
        assert certified, (n, what)
        if same:
            assert dS < 1e-10 and dE_rel < 1e-10 and dd < 1e-10 and dH < 1e-10, (n, dS, dE_rel, dd, dH)
        else:
            assert dS < 1e-8 and dE_rel < 1e-7 and dd < 1e-7 and dH < 1e-7, (n, dS, dE_rel, dd, dH)
        # the free components carry zero mean stress
        S = g.homogenized_stress()
        assert np.max(np.abs(np.diag(S))) < 1e-7 * scale
