"""Plain FP64 CPU oracle for the FE-projection trust-region solver.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, links or runs
this package: only the test suite, the smoke check and the CPU-baseline leg of
the benchmark do. It shares no code with the HIP path (only the seeded input
generators in ``synthetic`` serve both).

It works in strain space, as the paper states the method: the unknown is the
full displacement gradient at the quadrature points, compatibility is imposed
with the explicit per-wave-vector projector built from the finite-element
derivative operator (Sec. 2.1, eq. proj_operator), Newton steps come from
Steihaug's truncated CG with Powell's restart (Sec. 2.2, Algorithm 1), and the
trust-region ratio uses the first-order incremental energy (eq.
incr_energy_func, eq. rho_bar, Algorithm 2).

Modules:
  fe          shape-function gradients, real-space D and D^T, Fourier symbol of D
  projection  the compatibility projector G (explicit, per wave vector)
  material    isotropic energy-norm damage law: stress, tangent, exact energy
  solver      Steihaug-CG with restart, trust-region Newton with FAIEF ratio
  spring      the periodic 1D damage-spring system of Sec. 3.1

Parity status of each function is stated in its docstring ("pinned by ...");
the pins live in ``tests/test_oracle_*.py``.
"""
from . import fe, projection, material, solver, spring  # noqa: F401
