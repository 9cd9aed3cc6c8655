"""Seeded synthetic equality-constrained LQR instances.

This package is the only code shared by the CPU oracle and the GPU path.  It
draws problem data and holds none of the solver's arithmetic: no relation
projection, no elimination, no Riccati recursion, no multiplier recovery.
"""

from .generate import (  # noqa: F401
    Problem,
    config_c0,
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    config_mpc,
    config_paper,
    random_problem,
    make_config,
    CONFIG_SEEDS,
)
