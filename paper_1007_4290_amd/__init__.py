"""Sweeping preconditioner for the Helmholtz equation (2D, and 3D face by face) on MI355X (gfx950).

The numerical work lives in libhsweep.so (HIP C++, C-ABI declared in
include/hsweep.h); this package only marshals arguments.  Importing the
package does not load the library; the first Solver does, and it raises if
the library has not been built.
"""
from ._lib import HsweepError, EXPORTED  # noqa: F401


def __getattr__(name):
    if name in ("Solver", "Solver3", "helmholtz_solve", "factor_batch", "solve_batch"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
