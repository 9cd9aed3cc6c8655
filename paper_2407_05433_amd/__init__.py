"""MI355X (gfx950) solver for linear equality-constrained LQR problems.

The HIP library ``libeclqr.so`` (C ABI in ``include/eclqr.h``) implements
Algorithm 1 of the paper: the associative suffix scan over affine endpoint
relations, the stage-parallel elimination, an associative-scan Riccati solve
of the reduced LQR, primal recovery and the multipliers of Section VII, with
batching over instances of uneven horizons and dimensions, and the adjoint
used by ``ECLQRFunction``.  This package is its Python binding.
"""

from ._lib import EclqrError, STATUS_BITS, status_names  # noqa: F401
from .solver import (IpmSolution, Plan, Solution, allocate_solution, autotune, backward, default_options,  # noqa: F401
                     get_tuning, ipm_default_params, ipm_solve, ipm_workspace, kkt_residual, pack, pack_bounds, set_tuning,
                     solve, solve_noalloc, unpack)


def __getattr__(name):
    if name in ("ECLQRFunction", "eclqr_layer"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
