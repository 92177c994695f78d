"""The loading-tie certificate of tests/oracle_rounding.py on the CPU, with
the oracle standing in for the GPU solver (test infrastructure checks).

On the expanding-site cell, a load step that changes only the sites'
eigenstrain leaves the matrix strain unchanged at its first Newton iterate:
every matrix point that loaded at the end of the previous step starts with
kappa_t equal to kappa_hist, and whether it loads (strict >) is decided by
rounding. The certificate must accept a softening mask that differs there
and reject one that differs at a point far from every threshold of the law."""
import copy

import numpy as np
import pytest

from oracle.solver import CellSolver
from synthetic import workload
from tests import oracle_rounding as R


class OracleAsSolver:
    """The calls loading_tie makes on the GPU solver, served by an oracle
    restored from the checkpoint it is given; `flip` toggles mask entries."""

    def __init__(self, like, flip=()):
        self.o = copy.deepcopy(like)
        self.flip = list(flip)

    def set_state(self, u, kappa_hist, E, Rr, Rmax):
        self.o.restore({"u": u, "kappa_hist": kappa_hist, "E": E, "R": Rr, "Rmax": Rmax})
        self.o.apply_load_step(np.zeros((3, 3)))

    def solve_increment(self, params=None):
        return self.o.solve_increment(params)

    def field(self, which):
        assert which == 5
        m = (self.o.state["cprime"] > 0.0).astype(np.float64)
        for idx in self.flip:
            m[idx] = 1.0 - m[idx]
        return m

    def gradient(self):
        return self.o.H.copy()

    def get_state(self):
        return {"kappa_hist": self.o.kappa_hist.copy()}


@pytest.fixture(scope="module")
def eigenstrain_step_start():
    """The oracle right after apply_load_step of the first eigenstrain step
    that follows a step with matrix points loading in its last iterate."""
    w = workload("gel_3d8", steps=8)
    o = CellSolver(w.phase, w.materials, "q1")
    for n, dE in enumerate(w.load_path):
        o.set_eigenstrain(w.eig_phase, w.eig_path[n])
        o.apply_load_step(dE)
        st = o.state
        ties = o.mat.damage & (st["kappa_t"] == o.kappa_hist) & (o.kappa_hist > o.mat.k0)
        if n > 0 and np.count_nonzero(ties) > 0:
            return copy.deepcopy(o), ties
        o.solve_increment()
    pytest.fail("no step with matrix points at kappa_t = kappa_hist")


def test_equality_ties_are_certified(eigenstrain_step_start):
    o_start, ties = eigenstrain_step_start
    idx = tuple(a[0] for a in np.nonzero(ties))
    ok, text = R.loading_tie(OracleAsSolver(o_start, flip=[idx]), o_start, None, 0)
    assert ok, text


def test_a_mask_error_away_from_thresholds_is_rejected(eigenstrain_step_start):
    o_start, _ = eigenstrain_step_start
    st = o_start.state
    thr = R._thresholds(o_start.mat, o_start.kappa_hist)
    dist = np.min([np.abs(st["kappa_t"] - t) / np.maximum(np.abs(t), 1e-300) for t in thr], axis=0)
    dist = np.where(o_start.mat.damage, dist, -1.0)
    idx = np.unravel_index(int(np.argmax(dist)), dist.shape)
    assert dist[idx] > 1e-3
    ok, text = R.loading_tie(OracleAsSolver(o_start, flip=[idx]), o_start, None, 0)
    assert not ok and "away from its thresholds" in text, text


def test_near_threshold_uses_a_relative_rounding_band():
    t = np.array([1.0, 1.0, 2e-4])
    k = np.array([1.0 + 5e-13, 1.0 + 5e-12, 2e-4 * (1 - 1e-13)])
    assert list(R._near_threshold(k, [t])) == [True, False, True]
