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


def loading_tie(g, o_start, params, i, rel=1e-13):
    """Restart the GPU solver g and a copy of the oracle from the step's
    start, run both to Newton iteration i (the first whose decisions
    differ; the earlier ones coincide), and compare the points whose tangent
    carries the softening term. Returns (certified, text): certified if the
    two masks differ, and at every differing point the loading decision is a
    rounding tie of the law, |kappa_t - kappa_hist| <= rel kappa_hist."""
    import copy
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
    if nd == 0:
        return False, "the softening points agree at Newton %d" % i
    kt = o.state["kappa_t"][diff]
    kh = o.kappa_hist[diff]
    gap = np.abs(kt - kh) / np.maximum(kh, 1e-300)
    ok = bool(np.all(gap <= rel))
    return ok, ("%d point(s) load on one side only at Newton %d, |kappa_t - kappa_hist| / "
                "kappa_hist <= %.1e there" % (nd, i, float(gap.max())))


def step_verdict(g, rg, o_start, ro, olog, params=None, eta_cg=1e-6):
    """(same, certified, text) for one load step solved by the GPU solver g
    (report rg) and the oracle (report ro, log olog; o_start a copy of the
    oracle right after apply_load_step, before the solve). same: identical
    Newton decisions. Otherwise certified if the first differing decision is
    a CG-stop or ratio tie within the rounding drift of the method, if it
    follows a loading decision that is a rounding tie of the law at some
    points (loading_tie: this restarts g from the step's start, so call it
    after reading g's results), or if the oracle itself decides differently
    with reversed summation order."""
    glog = g.newton_log()
    if decisions_gpu(glog, rg) == decisions_oracle(ro):
        return True, True, "same decisions"
    ok, what = certify_tie(glog, g.cg_trace(), olog, eta_cg)
    if ok:
        return False, True, what + " (tie)"
    ok, why = loading_tie(g, o_start, params, first_difference(glog, ro))
    if ok:
        return False, True, what + "; " + why
    if oracle_is_rounding_sensitive(o_start, params, ro):
        return False, True, what + "; the oracle with reversed summation order decides differently"
    return False, False, what + "; " + why + "; not a tie"
