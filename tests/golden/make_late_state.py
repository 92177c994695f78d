"""Writes tests/golden/c1_3d8_state19.npz: the oracle's state after load step
19 of the 3D inclusion recipe at 8^3 (the 64^3 workload's recipe, radii
scaled), each step solved to the 1e-8 residual (i_NR,max 2000). Calls the
oracle only. Run from the repository root:

    python tests/golden/make_late_state.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.solver import CellSolver  # noqa: E402
from synthetic import workload  # noqa: E402

STEPS = 20


def main():
    w = workload("c1_3d8")
    o = CellSolver(w.phase, w.materials, "q1")
    newton = []
    for dE in w.load_path[:STEPS]:
        o.apply_load_step(dE)
        r = o.solve_increment({"i_nr_max": 2000})
        assert r["converged"]
        newton.append(r["newton_iters"])
    ck = o.checkpoint()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_3d8_state19.npz")
    np.savez_compressed(out, u=ck["u"], kappa_hist=ck["kappa_hist"], E=ck["E"],
                        radius=np.array([ck["R"], ck["Rmax"]]), newton=np.array(newton))
    print("wrote", out, "Newton iterations per step:", newton)


if __name__ == "__main__":
    main()
