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


def _load_scale(w, dE, eig=None):
    """Stress magnitude of the applied strain (or eigenstrain) in the stiffest
    phase: the scale against which stress differences are measured (a fully
    cracked cell has a homogenized stress of zero up to rounding)."""
    m = max(w.materials, key=lambda m: m["E"])
    lam = m["E"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"]))
    mu = m["E"] / (2 * (1 + m["nu"]))
    load = np.asarray(dE) if eig is None else np.asarray(dE) + np.asarray(eig)
    return np.linalg.norm(lam * np.trace(load) * np.eye(3) + 2 * mu * load)


# Rounding noise of the algorithm itself on the 3D workload: the oracle run
# against itself with only the summation order of its inner products changed
# drifts by 3-5% in the CG traces within a few load steps and flips CG stopping
# decisions (tests/test_oracle_cell.py::test_rounding_sensitivity_of_the_method).
ROUNDING_DRIFT = 0.1


def _certify_tie(glog, gtrace, olog, eta_cg, max_drift=ROUNDING_DRIFT):
    """At the first Newton iteration whose decisions differ, check that the
    difference is a threshold tie explained by rounding drift.

    CG stop: the Newton path agreed up to this iteration; at the last common
    CG iteration the stopping threshold eta_cg lies between the two values of
    ||r_{j+1}||/||r_0|| and their relative drift is below the rounding drift
    the method shows against itself. rho: the two ratios straddle the
    threshold and differ by less than that drift.
    Returns (certified, description)."""
    o_cg = [e for e in olog if e[0] == "cg"]
    o_nt = [e for e in olog if e[0] == "newton"]
    pos = 0
    for i, (gr, on) in enumerate(zip(glog, o_nt)):
        if gr["flag"] != on[2] or gr["cg_iters"] != on[3]:
            jmax = min(gr["cg_iters"], on[3])
            g = np.array([gtrace[pos + j][1] for j in range(jmax)])
            o = np.array([o_cg[pos + j][3] for j in range(jmax)])
            if not (np.isfinite(g[-1]) and np.isfinite(o[-1])):
                return False, "Newton %d: flag %d vs %d" % (i, gr["flag"], on[2])
            fin = np.isfinite(g) & np.isfinite(o)
            dev = np.abs(g[fin] - o[fin]) / o[fin]
            straddle = (g[-1] - eta_cg) * (o[-1] - eta_cg) <= 0.0
            ok = dev[-1] < max_drift and straddle
            return ok, ("Newton %d, CG stop after %d/%d iterations: ratios %.6e / %.6e vs eta %.1e, "
                        "trace drift %.1e at start -> %.2e at the stop"
                        % (i, gr["cg_iters"], on[3], g[-1], o[-1], eta_cg, dev[0], dev[-1]))
        rho_g, rho_o = gr["rho"], on[6]
        for t in (0.15, 0.25, 0.75):
            if (rho_g > t) != (rho_o > t):
                ok = abs(rho_g - rho_o) < max_drift
                return ok, "Newton %d: rho %.9f / %.9f across %.2f" % (i, rho_g, rho_o, t)
        pos += gr["cg_iters"]
    return False, "decisions differ after the last Newton iteration"


def _lockstep(name, steps, params=None, max_tie_frac=0.5):
    """Per load step, start the GPU from the oracle's state (checkpoint /
    restart through the C ABI), solve the same increment on both, and compare
    decisions and results. A step whose decisions differ must show that the
    differing decision sat on its threshold (certified tie); its results are
    then not compared."""
    w = workload(name, steps=steps)
    g, o = _pair(w.shape, w.phase, w.materials)
    p = dict(params or {})
    eta_cg = p.get("eta_cg", 1e-6)
    compared, ties = 0, []
    for n, dE in enumerate(w.load_path):
        announce(name, "step", n)
        if n > 0:
            ck = o.checkpoint()
            g.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
        eig = None
        if w.eig_path is not None:     # a growing eigenstrain drives this load step
            eig = w.eig_path[n]
            g.set_eigenstrain(w.eig_phase, eig)
            o.set_eigenstrain(w.eig_phase, eig)
        g.apply_load_step(dE)
        o.apply_load_step(dE)
        olog = []
        rg = g.solve_increment(p)
        ro = o.solve_increment(p, log=olog)
        glog = g.newton_log()
        same = ([r["flag"] for r in glog] == ro["flags"] and
                [r["cg_iters"] for r in glog] == ro["cg_per_newton"] and
                [r["accepted"] for r in glog] == [1 if x > 0.15 else 0 for x in ro["rho"]] and
                rg["converged"] == ro["converged"])
        if not same:
            ok, what = _certify_tie(glog, g.cg_trace(), olog, eta_cg)
            print("[lockstep] %s step %d: decisions differ, %s -> %s"
                  % (name, n, what, "certified tie" if ok else "NOT a tie"), flush=True)
            assert ok, (n, what)
            ties.append(n)
            if rg["converged"] and ro["converged"]:
                # two inexact-Newton paths from the same state to the same
                # equilibrium: stress and damage still at the parity bar, the
                # gradient (which a fully damaged band leaves free) to 1e-8
                scale = _load_scale(w, o.E, eig)
                dS = np.linalg.norm(g.homogenized_stress() - o.homogenized_stress()) / scale
                dH = rel_err(g.gradient(), o.H)
                dd = float(np.abs(g.damage() - o.damage()).max())
                print("[lockstep]   after the tie: |dSigma|/scale %.2e, grad rel %.2e, damage %.2e"
                      % (dS, dH, dd), flush=True)
                assert dS < TOL and dd < TOL and dH < 1e-8, (n, dS, dH, dd)
            continue
        compared += 1
        scale = _load_scale(w, o.E, eig)
        Sg, So = g.homogenized_stress(), o.homogenized_stress()
        assert np.linalg.norm(Sg - So) <= TOL * scale, (n, Sg, So)
        Hg = g.gradient()
        assert rel_err(Hg, o.H) < TOL, (n, rel_err(Hg, o.H))
        dg, do = g.damage(), o.damage()
        assert np.abs(dg - do).max() < TOL, (n, np.abs(dg - do).max())
        # Newton-level ratios agree loosely: rho is a ratio of two differences
        # that vanish at convergence, and the inexact CG steps inherit the
        # rounding drift of the CG traces, while the converged fields do not
        # (they are compared at 1e-10 above)
        for gr, rho_o in zip(glog, ro["rho"]):
            if np.isfinite(rho_o):
                assert abs(gr["rho"] - rho_o) <= 1e-2 * max(1.0, abs(rho_o)), (n, gr["rho"], rho_o)
    print("[lockstep] %s: %d steps compared, certified ties at steps %s"
          % (name, compared, ties), flush=True)
    assert len(ties) <= max_tie_frac * len(w.load_path)
    return compared, ties


def test_lockstep_2d_workload_full_path():
    """2D 32x32, P1 triangles, 20 uniaxial steps to 0.5% (the small workload)."""
    require_gpu()
    _lockstep("c0_2d32", None)


def test_lockstep_3d_workload_16():
    """3D Q1 inclusion cell at 16^3, first 10 steps of the 0.6% path."""
    require_gpu()
    _lockstep("c1_3d16", 10)


def test_lockstep_3d_workload_16_solved_to_tolerance():
    """The same cell with the benchmark's Newton limit (2000): the first four
    steps each solved to the 1e-8 residual, through the damage onset that the
    default limit of 50 cuts short (59 Newton iterations in step 2)."""
    require_gpu()
    compared, ties = _lockstep("c1_3d16", 4, {"i_nr_max": 2000})
    assert compared + len(ties) == 4


def test_checkpoint_restart_is_exact():
    """Solve 4 steps; save after 2, restore into a fresh context, redo steps
    3-4: identical bits."""
    require_gpu()
    announce("checkpoint")
    w = workload("c0_2d32", steps=4)
    from paper_2207_10657_amd import Solver
    a = Solver(w.shape, w.element)
    a.setup(w.phase, w.materials)
    for n in range(2):
        a.apply_load_step(w.load_path[n])
        a.solve_increment()
    st = a.get_state()
    for n in range(2, 4):
        a.apply_load_step(w.load_path[n])
        a.solve_increment()
    b = Solver(w.shape, w.element)
    b.setup(w.phase, w.materials)
    b.set_state(st["u"], st["kappa_hist"], st["E"], st["R"], st["Rmax"])
    for n in range(2, 4):
        b.apply_load_step(w.load_path[n])
        b.solve_increment()
    np.testing.assert_array_equal(a.displacement(), b.displacement())
    np.testing.assert_array_equal(a.homogenized_stress(), b.homogenized_stress())
    np.testing.assert_array_equal(a.field(4), b.field(4))


def test_expanding_sites_16_against_oracle():
    """Eigenstrain loading (Algorithm 2's eps_eval = eps + eps_eig): sites
    inside the inclusions expand by 2.5e-4 per step at zero macroscopic
    strain and crack the damaging matrix. Each step starts from the oracle's
    state; the converged results must agree at the parity bar.

    Newton decisions are not compared here: a point that loaded at the end of
    the previous step has kappa_t = kappa_hist when its strain does not change
    (most matrix points away from the sites), so whether it loads (strict >)
    is decided by rounding, and the two sides may take different, equally
    valid Newton paths to the same equilibrium. Two iterates that both meet
    the stopping test (r_eq or r_NR <= 1e-8) differ by O(1e-8) in relative
    terms, so the results are compared at 10x the tolerance (stress 1e-8 of
    the load scale, damage and gradient 1e-7); steps whose Newton paths
    coincide reach the 1e-10 parity bar (logged)."""
    require_gpu()
    w = workload("gel_3d16", steps=6)
    g, o = _pair(w.shape, w.phase, w.materials)
    compared = 0
    for n, dE in enumerate(w.load_path):
        announce("gel_3d16", "step", n)
        if n > 0:
            ck = o.checkpoint()
            g.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
        eig = w.eig_path[n]
        g.set_eigenstrain(w.eig_phase, eig)
        o.set_eigenstrain(w.eig_phase, eig)
        g.apply_load_step(dE)
        o.apply_load_step(dE)
        rg = g.solve_increment()
        ro = o.solve_increment()
        scale = _load_scale(w, o.E, eig)
        dS = np.linalg.norm(g.homogenized_stress() - o.homogenized_stress()) / scale
        dd = float(np.abs(g.damage() - o.damage()).max())
        dH = rel_err(g.gradient(), o.H)
        print("[gel] step %d: converged %s/%s, Newton %d/%d, |dSigma|/scale %.2e, damage %.2e, "
              "grad %.2e, max damage %.3f" % (n, rg["converged"], ro["converged"], rg["newton_iters"],
                                              len(ro["flags"]), dS, dd, dH, float(o.damage().max())),
              flush=True)
        assert rg["converged"] and ro["converged"], n
        assert dS < 1e-8 and dd < 1e-7 and dH < 1e-7, (n, dS, dd, dH)
        compared += 1
    assert compared == len(w.load_path)


def test_eigenstrain_laminate_on_gpu():
    """The expanding-laminate closed form (layers normal to x, phase 1 with
    eigenstrain theta I, E = 0) on the GPU."""
    require_gpu()
    announce("eigenstrain laminate")
    shape = (4, 4, 8)
    layers = np.array([0, 0, 1, 1, 1, 0, 1, 0], dtype=np.uint8)
    phase = laminate_microstructure(shape, layers)
    theta = 2e-3
    g, _ = _pair(shape, phase, [EL1, dict(EL2, eig=theta * np.eye(3))])
    g.apply_load_step(np.zeros((3, 3)))
    rep = g.solve_increment({"eta_eq": 1e-12, "eta_nr": 1e-14, "eta_cg": 1e-10})
    assert rep["converged"]
    f = np.array([np.mean(layers == 0), np.mean(layers == 1)])
    lam = np.array([m["E"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"])) for m in (EL1, EL2)])
    mu = np.array([m["E"] / (2 * (1 + m["nu"])) for m in (EL1, EL2)])
    M = lam + 2 * mu
    b = (3 * lam + 2 * mu) * np.array([0.0, theta])
    sxx = np.sum(f * b / M) / np.sum(f / M)
    exx = (sxx - b) / M
    syy = np.sum(f * (lam * exx + b))
    S = g.homogenized_stress()
    assert abs(S[0, 0] - sxx) < 1e-10 * abs(syy)
    assert abs(S[1, 1] - syy) < 1e-10 * abs(syy) and abs(S[2, 2] - syy) < 1e-10 * abs(syy)
