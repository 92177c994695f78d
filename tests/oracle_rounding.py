"""Rounding certificates for lockstep comparisons (test infrastructure).

Where a Newton decision of the GPU differs from the oracle's, the step is
re-solved by the oracle itself with only the summation order of its inner
products reversed. If the oracle's own decisions then change too, the step
is decided by rounding: the method, not the GPU path, is sensitive there."""
import contextlib

import numpy as np


def decisions_gpu(glog, rep):
    return ([r["flag"] for r in glog], [r["cg_iters"] for r in glog],
            [r["accepted"] for r in glog], bool(rep["converged"]))


def decisions_oracle(ro, eta_up=0.15):
    return (list(ro["flags"]), list(ro["cg_per_newton"]),
            [1 if x > eta_up else 0 for x in ro["rho"]], bool(ro["converged"]))


@contextlib.contextmanager
def reversed_summation():
    """Inside this block the oracle's solver sums every inner product in
    reversed element order."""
    from oracle import solver as S
    orig_st, orig_inner = S.steihaug, S.inner

    def rev(X, Y):
        return float(np.sum((X * Y).ravel()[::-1]))

    def st(apply_A, g, R, eta, jmax, dot=None, log=None, **kw):
        return orig_st(apply_A, g, R, eta, jmax, dot=rev, log=log, **kw)

    S.steihaug, S.inner = st, rev
    try:
        yield
    finally:
        S.steihaug, S.inner = orig_st, orig_inner


def oracle_is_rounding_sensitive(o_start, params, ro):
    """o_start: a copy of the oracle taken before the solve that produced
    `ro`. True if the same solve with reversed summation order takes other
    decisions."""
    with reversed_summation():
        ro2 = o_start.solve_increment(params)
    return decisions_oracle(ro2) != decisions_oracle(ro)


# Rounding noise of the algorithm itself on the 3D workload: the oracle run
# against itself with only the summation order of its inner products changed
# drifts by 3-5% in the CG traces within a few load steps and flips CG stopping
# decisions (tests/test_oracle_cell.py::test_rounding_sensitivity_of_the_method).
ROUNDING_DRIFT = 0.1


def certify_tie(glog, gtrace, olog, eta_cg, max_drift=ROUNDING_DRIFT):
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


def first_difference(glog, ro, eta_up=0.15):
    """Index of the first Newton iteration whose decisions (exit flag, CG
    count, acceptance) differ, or the common length if one log is a prefix of
    the other."""
    acc = [1 if x > eta_up else 0 for x in ro["rho"]]
    n = min(len(glog), len(ro["flags"]))
    for i in range(n):
        if (glog[i]["flag"] != ro["flags"][i] or glog[i]["cg_iters"] != ro["cg_per_newton"][i]
                or glog[i]["accepted"] != acc[i]):
            return i
    return n


def _oracle_stop_drift(o_start, params, olog, i):
    """The oracle re-solving the step with reversed summation order: (its
    decisions differ from the default run's, the relative drift of its
    residual-ratio trace against the default run's at the end of Newton
    iteration i's CG)."""
    import copy
    o2 = copy.deepcopy(o_start)
    log2 = []
    with reversed_summation():
        o2.solve_increment(params, log=log2)
    n1 = [e for e in olog if e[0] == "newton"]
    n2 = [e for e in log2 if e[0] == "newton"]
    differ = [(e[2], e[3]) for e in n1] != [(e[2], e[3]) for e in n2]
    c1 = [e[3] for e in olog if e[0] == "cg"]
    c2 = [e[3] for e in log2 if e[0] == "cg"]
    pos = sum(e[3] for e in n1[:i])
    m = min(len(c1), len(c2))
    a = np.array(c1[pos:m])
    b = np.array(c2[pos:m])
    if i < len(n1):
        a, b = a[: n1[i][3]], b[: n1[i][3]]
    fin = np.isfinite(a) & np.isfinite(b) & (a != 0)
    drift = float(np.max(np.abs(a[fin] - b[fin]) / np.abs(a[fin]))) if fin.any() else 0.0
    return differ, drift


# Relative distance to a threshold of the damage law within which the GPU's
# and numpy's evaluations of kappa_t at one state may fall on either side:
# both form kappa_t from the same strain in a different operation order.
LAW_ROUNDING = 1e-12


def _thresholds(mat, kappa_hist):
    return [kappa_hist, mat.k0, mat.kf]


def _near_threshold(kappa_t, thr, tol=LAW_ROUNDING):
    near = np.zeros(kappa_t.shape, dtype=bool)
    for t in thr:
        near |= np.abs(kappa_t - t) <= tol * np.maximum(np.abs(t), 1e-300)
    return near


def loading_tie(g, o_start, params, i):
    """Restart the GPU solver g and a copy of the oracle from the step's
    start and run both to Newton iteration i (the first whose decisions
    differ; the earlier ones coincide). Where the points whose tangent
    carries the softening term differ, the decision must be a threshold tie
    between the two (nearly equal) states:
    - the oracle's law evaluated on the GPU's gradient field and history
      reproduces the GPU's mask, except at points within rounding of a
      threshold (kappa_hist, kappa0, kappaf);
    - at every differing point the equivalent strains of the two states lie
      on either side of such a threshold, or one of them within rounding of
      it. A point that loaded at the end of the previous step and whose
      strain the new load leaves unchanged sits exactly at kappa_hist.
    Returns (certified, text)."""
    import copy
    from oracle import material
    o = copy.deepcopy(o_start)
    ck = o.checkpoint()
    g.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
    if i > 0:
        prm = dict(params or {}, i_nr_max=i)
        g.solve_increment(prm)
        o.solve_increment(prm)
    gm = g.field(5) > 0.5
    om = o.state["cprime"] > 0.0
    diff = gm != om
    nd = int(np.count_nonzero(diff))
    Hg = g.gradient()
    khg = g.get_state()["kappa_hist"]
    dstate = float(np.linalg.norm(Hg - o.H) / np.linalg.norm(o.H))
    if nd == 0:
        return False, "the softening points agree at Newton %d" % i
    stg = material.evaluate(o.mat, Hg, khg)
    bad = ((stg["cprime"] > 0.0) != gm) & ~_near_threshold(stg["kappa_t"], _thresholds(o.mat, khg))
    if np.any(bad):
        return False, ("%d GPU softening point(s) differ from the law at the GPU's own state away "
                       "from its thresholds" % int(np.count_nonzero(bad)))
    kg, ko = stg["kappa_t"][diff], o.state["kappa_t"][diff]
    thr_o = [t[diff] for t in _thresholds(o.mat, o.kappa_hist)]
    thr_g = [t[diff] for t in _thresholds(o.mat, khg)]
    straddle = _near_threshold(kg, thr_g) | _near_threshold(ko, thr_o)
    for tg, to in zip(thr_g, thr_o):
        straddle |= (kg - tg) * (ko - to) <= 0.0
    gap = np.abs(kg - ko) / np.maximum(np.abs(ko), 1e-300)
    ok = bool(np.all(straddle))
    return ok, ("%d point(s) soften on one side only at Newton %d (states %.1e apart), their "
                "equivalent strains %s a threshold of the law (|dkappa|/kappa <= %.1e)"
                % (nd, i, dstate, "straddle" if ok else "do NOT all straddle", float(gap.max())))


def step_outcome(g, rg, o_start, ro, olog, params=None, eta_cg=1e-6):
    """(same, certified, text) for one load step solved by the GPU solver g
    (report rg) and the oracle (report ro, log olog; o_start a copy of the
    oracle right after apply_load_step, before the solve). same: identical
    Newton decisions. Otherwise certified if the first differing decision is
    (a) a CG stop or ratio test whose two values straddle the threshold, with
        a trace drift within the method's rounding drift, or within 10x the
        drift of the oracle against itself with reversed summation order;
    (b) one the oracle itself takes differently with reversed summation order;
    (c) a loading decision at points whose equivalent strains straddle a
        threshold of the law between the two states (loading_tie; this
        restarts g from the step's start, so read g's results first)."""
    glog = g.newton_log()
    if decisions_gpu(glog, rg) == decisions_oracle(ro):
        return True, True, "same decisions"
    i = first_difference(glog, ro)
    ok, what = certify_tie(glog, g.cg_trace(), olog, eta_cg)
    if ok:
        return False, True, what + " (tie)"
    differ, drift_oo = _oracle_stop_drift(o_start, params, olog, i)
    if differ:
        return False, True, what + "; the oracle with reversed summation order decides differently"
    ok2, _ = certify_tie(glog, g.cg_trace(), olog, eta_cg, max_drift=10.0 * drift_oo)
    if ok2:
        return False, True, what + ("; within 10x the oracle's own drift (%.1e) with reversed "
                                    "summation" % drift_oo)
    ok3, why = loading_tie(g, o_start, params, i)
    if ok3:
        return False, True, what + "; " + why
    return False, False, what + "; oracle self-drift %.1e; " % drift_oo + why + "; not a tie"
