"""Mixed-precision restarted GMRES(m) on MI355X (gfx950).

Method: Lindquist, Luszczek, Dongarra, "Improving the Performance of the
GMRES Method using Mixed-Precision Techniques" (arXiv 2011.01850).  The
solver is the C-ABI library libgmres.so (include/gmres.h) built from the
HIP sources in csrc/; this package only marshals arguments to it.
"""
from ._lib import (CGSR, CONVERGED, FP64, MAXITER, MGS, MIXED_BF16, MIXED_FP16, MIXED_FP32,  # noqa: F401
                   STALLED, GmresError, load)
from .solver import BatchSolver, Solver, encode, release_cached_memory  # noqa: F401
