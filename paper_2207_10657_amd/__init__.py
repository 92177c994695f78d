"""MI355X-native FE-projection homogenization solver (trust region + FAIEF).

The solver itself is the HIP library ``libhfe.so`` built from ``csrc/`` (C ABI
in ``include/hfe.h``); ``hfe`` is its ctypes binding. Importing the package
does not load the library; ``Solver(...)`` or ``hfe.load_library()`` does,
and fails with ImportError when it has not been built.
"""
from .hfe import (Solver, HfeError, effective_stiffness, load_library, solve_batch,  # noqa: F401
                  workspace_bytes)
