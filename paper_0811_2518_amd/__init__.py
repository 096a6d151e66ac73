"""Synchronous Gaussian belief propagation for sparse symmetric A x = b on MI355X.

The solver is the HIP library ``libgabp.so`` (C ABI in include/gabp.h); this
package holds its sources, the build script and a thin ctypes binding.
"""
from .binding import (AugmentedSolver, BatchedSolver, GabpError, Solver, default_opts, lib,  # noqa: F401
                      last_create_error, try_create)
from .autograd import GaBPSolve, gabp_solve  # noqa: F401
