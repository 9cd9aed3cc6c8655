"""CPU oracle for the equality-constrained LQR solve (FP64, NumPy/LAPACK).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP path and never imports it; the product path does not call it.

Contents (each function cites the passage of the paper it follows):

* ``relations``   -- Lemma 1 (existential projection), eq. (composition-matrix),
                     the base and terminal relations of Section IV.
* ``sequential``  -- the method of Algorithm 1 run sequentially: suffix
                     relations composed right to left, state parameterization
                     (Section IV), stage elimination (Section V), textbook
                     Riccati recursion on the reduced problem, recovery.
* ``dense``       -- the plain definition: the KKT system of eq. (problem)
                     solved densely by SVD least squares (minimum-norm
                     multipliers).  Tiny inputs only.
* ``multipliers`` -- canonical (minimum-norm) multipliers at any size, by
                     solving the minimum-norm stationarity problem of
                     Section VII as an equality-constrained LQR in reversed time.
* ``residual``    -- the KKT residual of Section IX.
* ``gradients``   -- implicit-differentiation gradients and central finite
                     differences.

Parity pins: every function above is pinned by ``tests/test_oracle_*.py``
against closed forms, brute force, exact rational arithmetic, invariants of the
paper (Lemma 2, Theorems 1-2, Propositions 2-3) or an independent route.
"""

from .relations import Relation  # noqa: F401
from .sequential import rows_independent, solve_sequential, SequentialResult  # noqa: F401
from .dense import dense_kkt, solve_dense  # noqa: F401
from .multipliers import dual_problem, minnorm_multipliers, solve_with_multipliers  # noqa: F401
from .residual import kkt_residual  # noqa: F401
