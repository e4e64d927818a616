"""MI355X-native primal-dual solver of the generalized Hopf formula for
time-optimal control of linear systems (arXiv 1712.08226).

The solver is the C-ABI library libhopfpd.so (include/hopfpd.h) built from
csrc/ for gfx950; ``hopfpd`` is its thin Python binding.
"""
from .hopfpd import (Solver, HopfError, load, default_opts,  # noqa: F401
                     PT_OK, PT_INSIDE, PT_UNREACH, PT_NOCONV, PT_NONFINITE)
