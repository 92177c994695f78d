"""GPU parity of whole load steps (Algorithm 2 around Algorithm 1) against the
strain-space oracle, in lockstep: the same Newton decisions (exit flags, CG
iteration counts, accept/reject) and, per step, the homogenized stress and the
gradient, stress and damage fields to a relative 1e-10 in FP64.

Closed forms first (homogeneous cell, laminate), then trajectories of the two
benchmark workloads: the 2D 32x32 plane-strain cell with 20 load steps (full
path) and the 3D inclusion cell at 16^3 (same recipe as the 64^3 workload).
"""
import copy

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


from tests.oracle_rounding import step_outcome as _step_outcome  # noqa: E402


def _lockstep(name, steps, params=None, max_tie_frac=0.5, stats=False):
    """Per load step, start the GPU from the oracle's state (checkpoint /
    restart through the C ABI), solve the same increment on both, and compare
    decisions and results. A step whose decisions differ must show that the
    differing decision sat on its threshold (a tie certified by
    tests/oracle_rounding.step_outcome: a straddled threshold within the
    rounding drift of the method or of the oracle against itself, or a
    loading decision at a threshold of the law); its results are then
    compared only where both sides converged."""
    w = workload(name, steps=steps)
    g, o = _pair(w.shape, w.phase, w.materials)
    p = dict(params or {})
    eta_cg = p.get("eta_cg", 1e-6)
    compared, ties = 0, []
    restarts = [0, 0]
    stalls = [0, 0]
    for n, dE in enumerate(w.load_path):
        announce(name, "step", n, p)
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
        o_start = copy.deepcopy(o)
        olog = []
        rg = g.solve_increment(p)
        ro = o.solve_increment(p, log=olog)
        glog = g.newton_log()
        restarts[0] += rg["restarts"]
        restarts[1] += ro["restarts"]
        stalls[0] += rg["stall_exits"]
        stalls[1] += ro["stall_exits"]
        same = ([r["flag"] for r in glog] == ro["flags"] and
                [r["cg_iters"] for r in glog] == ro["cg_per_newton"] and
                [r["restarts"] for r in glog] == ro["restarts_per_newton"] and
                [r["accepted"] for r in glog] == [1 if x > 0.15 else 0 for x in ro["rho"]] and
                rg["converged"] == ro["converged"])
        if not same:
            # the GPU's results first: the certificate may restart the GPU solver
            Sg, Hg, Dg = g.homogenized_stress(), g.gradient(), g.damage()
            _, ok, what = _step_outcome(g, rg, o_start, ro, olog, p, eta_cg)
            print("[lockstep] %s step %d: decisions differ, %s -> %s"
                  % (name, n, what, "certified tie" if ok else "NOT a tie"), flush=True)
            assert ok, (n, what)
            ties.append(n)
            if rg["converged"] and ro["converged"]:
                # two inexact-Newton paths from the same state to the same
                # equilibrium: stress and damage still at the parity bar, the
                # gradient (which a fully damaged band leaves free) to 1e-8
                scale = _load_scale(w, o.E, eig)
                dS = np.linalg.norm(Sg - o.homogenized_stress()) / scale
                dH = rel_err(Hg, o.H)
                dd = float(np.abs(Dg - o.damage()).max())
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
        # rho_bar of every Newton step: to 1e-8 where the CG iterates of the
        # two sides agree to rounding; a long CG solve carries the rounding
        # drift of the method (its residual-ratio trace drifts between the
        # two sides, as between two summation orders of the oracle), and the
        # step, hence rho_bar, moves with it: there the bound is 10x the drift
        # of the trace measured on that solve
        gtr = g.cg_trace()
        o_cg = [e[3] for e in olog if e[0] == "cg"]
        pos, worst = 0, 0.0
        for gr, rho_o in zip(glog, ro["rho"]):
            k = gr["cg_iters"]
            gt = np.array([gtr[pos + j][1] for j in range(k)])
            ot = np.array(o_cg[pos:pos + k])
            pos += k
            fin = np.isfinite(gt) & np.isfinite(ot)
            drift = float(np.max(np.abs(gt[fin] - ot[fin]) / ot[fin])) if fin.any() else 0.0
            if np.isfinite(rho_o):
                d_rho = abs(gr["rho"] - rho_o) / max(1.0, abs(rho_o))
                worst = max(worst, d_rho)
                assert d_rho <= max(1e-8, 10.0 * drift), (n, gr["rho"], rho_o, drift)
        print("[lockstep] %s step %d: max |d rho| %.1e" % (name, n, worst), flush=True)
    print("[lockstep] %s: %d steps compared, certified ties at steps %s, restarts %d / %d"
          % (name, compared, ties, restarts[0], restarts[1]), flush=True)
    assert len(ties) <= max_tie_frac * len(w.load_path)
    if stats:
        return {"compared": compared, "ties": ties, "restarts": restarts, "stalls": stalls}
    return compared, ties


def test_lockstep_2d_workload_full_path():
    """2D 32x32, P1 triangles, 20 uniaxial steps to 0.5% (the small workload)."""
    require_gpu()
    _lockstep("c0_2d32", None)


def test_free_running_2d_workload_full_path():
    """The 2D workload's 20 load steps run on the GPU and on the oracle side
    by side with no restart from the oracle's state in between (Algorithm 2's
    load loop, Sec. 2.2): per step the same Newton decisions, and the
    homogenized stress and damage field at the 1e-10 parity bar."""
    require_gpu()
    w = workload("c0_2d32")
    g, o = _pair(w.shape, w.phase, w.materials)
    for n, dE in enumerate(w.load_path):
        announce("free-running c0_2d32 step", n)
        g.apply_load_step(dE)
        o.apply_load_step(dE)
        rg = g.solve_increment()
        ro = o.solve_increment()
        glog = g.newton_log()
        assert [r["flag"] for r in glog] == ro["flags"], n
        assert [r["cg_iters"] for r in glog] == ro["cg_per_newton"], n
        assert rg["converged"] == ro["converged"], n
        scale = _load_scale(w, o.E)
        dS = np.linalg.norm(g.homogenized_stress() - o.homogenized_stress()) / scale
        dd = float(np.abs(g.damage() - o.damage()).max())
        print("[free] c0_2d32 step %d: Newton %d, converged %s, |dSigma|/scale %.2e, damage %.2e"
              % (n, rg["newton_iters"], rg["converged"], dS, dd), flush=True)
        assert dS < TOL and dd < TOL, (n, dS, dd)


def test_lockstep_3d_workload_16():
    """3D Q1 inclusion cell at 16^3, first 5 steps of the 0.6% path (through
    the damage onset; the later steps take the oracle minutes each)."""
    require_gpu()
    _lockstep("c1_3d16", 5)


def test_lockstep_3d_workload_8_into_full_damage():
    """The same cell at 8^3, first 15 steps: the damage reaches 1 at step 3
    and the later steps solve the cracked cell with long CG runs. Those runs
    (150-280 iterations) end within the method's rounding drift of the CG
    threshold, so most of the cracked-cell steps are certified ties (on some
    of them the oracle itself decides differently once its summation order
    is reversed); the steps before the crack are compared at the parity bar."""
    require_gpu()
    compared, ties = _lockstep("c1_3d8", 15, max_tie_frac=0.7)
    assert compared >= 4, (compared, ties)


def test_lockstep_3d_workload_16_solved_to_tolerance():
    """The same cell with the benchmark's Newton limit (2000): the first four
    steps each solved to the 1e-8 residual, through the damage onset that the
    default limit of 50 cuts short (59 Newton iterations in step 2)."""
    require_gpu()
    compared, ties = _lockstep("c1_3d16", 4, {"i_nr_max": 2000})
    assert compared + len(ties) == 4


@pytest.mark.parametrize("name,steps", [("c0_2d32", 1), ("c1_3d16", 2)])
def test_lockstep_with_a_reset_after_every_cg_step(name, steps):
    """Powell's reset of Algorithm 1 (eq. 1) forced after every CG step
    (restart constant -1): the GPU recomputes the true residual A z + g on
    the host's request, restarts along it (beta = 0) and continues the fused
    iteration from the resumed device state. Every Newton decision, every
    per-step restart count and the results must match the oracle, which then
    runs steepest descent with exact line search inside each Newton step
    (pinned in tests/test_oracle_solver.py). j_CG,max = 40 keeps the oracle
    fast; the steps compared are those that converge under it (steepest
    descent drifts apart by rounding faster than CG, and the later 2D steps
    run into boundary-exit ties)."""
    require_gpu()
    st = _lockstep(name, steps, {"restart": -1.0, "j_cg_max": 40}, max_tie_frac=0.0, stats=True)
    assert st["compared"] == steps
    assert st["restarts"][0] == st["restarts"][1] >= 40 * steps


def test_lockstep_2d_with_the_stall_exit():
    """The optional stall exit of the CG (a window of 25 iterations, short
    enough to fire on the damaged states of the 2D workload from its fourth
    load step on): the same Newton decisions, stall exits and results as the
    oracle's implementation of the same rule."""
    require_gpu()
    st = _lockstep("c0_2d32", 6, {"cg_stall": 25}, max_tie_frac=0.0, stats=True)
    assert st["compared"] == 6
    assert st["stalls"][0] == st["stalls"][1] > 0


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

    Steps whose Newton decisions coincide are held to the 1e-10 parity bar.
    Where they differ, the step must be rounding-decided: the first differing
    decision is a CG stop or ratio test within the method's rounding drift of
    its threshold, or the oracle re-solving the step with its inner products
    summed in reversed order decides differently too (a point that loaded at
    the end of the previous step has kappa_t = kappa_hist when its strain does
    not change, so whether it loads, strict >, is decided by rounding). Two
    iterates that both meet the stopping test (r_eq or r_NR <= 1e-8) differ
    by O(1e-8) in relative terms, so such steps are compared at 10x the
    tolerance (stress 1e-8 of the load scale, damage and gradient 1e-7)."""
    import copy
    from tests.oracle_rounding import step_outcome
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
        o_start = copy.deepcopy(o)
        olog = []
        rg = g.solve_increment()
        ro = o.solve_increment(log=olog)
        scale = _load_scale(w, o.E, eig)
        dS = np.linalg.norm(g.homogenized_stress() - o.homogenized_stress()) / scale
        dd = float(np.abs(g.damage() - o.damage()).max())
        dH = rel_err(g.gradient(), o.H)
        same, certified, what = step_outcome(g, rg, o_start, ro, olog)   # may restart g
        print("[gel] step %d: converged %s/%s, Newton %d/%d, %s, |dSigma|/scale %.2e, damage "
              "%.2e, grad %.2e, max damage %.3f"
              % (n, rg["converged"], ro["converged"], rg["newton_iters"], len(ro["flags"]), what,
                 dS, dd, dH, float(o.damage().max())), flush=True)
        assert rg["converged"] and ro["converged"], n
        assert certified, (n, what)
        if same:
            assert dS < TOL and dd < TOL and dH < TOL, (n, dS, dd, dH)
        else:
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


def test_step_norm_recurrences_at_64cubed():
    """The CG of Algorithm 1 tracks ||z||^2 and <z, d> in displacement
    coordinates by recurrences (no stencil pass); the trust-region exits put
    the step on ||p|| = R with them. On the 64^3 workload's damage-onset
    load steps (hundreds of boundary exits at a growing iteration count),
    the step norm the trial pass sums directly over the 2,097,152 points
    must equal R at every boundary and negative-curvature exit to 1e-10."""
    require_gpu()
    from paper_2207_10657_amd import Solver
    w = workload("c1_3d64", steps=4)
    s = Solver(w.shape, w.element)
    s.setup(w.phase, w.materials)
    worst, exits = 0.0, 0
    for n, dE in enumerate(w.load_path):
        announce("step norm recurrences 64^3, step", n)
        s.apply_load_step(dE)
        s.solve_increment({"i_nr_max": 60})
        for r in s.newton_log():
            if r["flag"] in (2, 3):
                exits += 1
                worst = max(worst, abs(r["p_norm"] - r["R_before"]) / r["R_before"])
    print("[recurrence] 64^3: %d exits on the sphere, max | ||p|| - R | / R = %.2e" % (exits, worst),
          flush=True)
    assert exits >= 20
    assert worst < 1e-10
