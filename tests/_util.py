"""Small helpers shared by the tests (comparisons and tiny problem builders)."""

from __future__ import annotations

import numpy as np

from workloads.generate import Problem, random_problem


def flat(blocks) -> np.ndarray:
    return np.concatenate([np.asarray(b, dtype=np.float64).ravel() for b in blocks]) if len(blocks) else np.zeros(0)


def rel_err(a, b) -> float:
    """||a - b||_2 / max(||b||_2, 1e-300) over a list of blocks (b = reference)."""
    fa, fb = flat(a), flat(b)
    return float(np.linalg.norm(fa - fb) / max(np.linalg.norm(fb), 1e-300))


def tiny_problem(seed: int, N=5, n=3, m=2, kinds=None, terminal_rows=1, redundant=(), g_mode="trajectory",
                 nx=None, nu=None, with_M=False) -> Problem:
    rng = np.random.default_rng(seed)
    nx = list(nx) if nx is not None else [n] * (N + 1)
    nu = list(nu) if nu is not None else [m] * N
    N = len(nu)
    if kinds is None:
        kinds = []
        for i in range(N):
            k = int(rng.integers(0, min(nu[i], 3) + 1))
            kinds.append(["state" if rng.random() < 0.5 else "mixed" for _ in range(k)])
    return random_problem(rng, nx, nu, kinds, terminal_rows=terminal_rows, redundant_stages=redundant,
                          g_mode=g_mode, with_M=with_M)


def problem_family():
    """(name, problem) pairs covering the structural cases of the paper: mixed and
    state-only rows, redundant rows, varying dimensions, empty rows, N = 1,
    fully pinned states (n-bar = 0), no free input (m-bar = 0)."""
    out = []
    for s in range(6):
        out.append((f"mixed-state-{s}", tiny_problem(100 + s, N=6, n=4, m=2, terminal_rows=2)))
    for s in range(4):
        out.append((f"redundant-{s}", tiny_problem(200 + s, N=6, n=4, m=3, terminal_rows=1, redundant=(1, 3, 4))))
    out.append(("varying-dims", tiny_problem(300, nx=[3, 4, 2, 5, 3, 4], nu=[2, 3, 2, 2, 3], terminal_rows=1)))
    out.append(("varying-dims-2", tiny_problem(301, nx=[2, 5, 5, 3, 1, 4, 2], nu=[3, 1, 4, 2, 2, 3], terminal_rows=1)))
    out.append(("no-rows", tiny_problem(302, N=5, n=3, m=2, kinds=[[]] * 5, terminal_rows=0)))
    out.append(("N1", tiny_problem(303, N=1, n=3, m=2, kinds=[["mixed"]], terminal_rows=1)))
    out.append(("N1-full-terminal", tiny_problem(304, N=1, n=2, m=2, kinds=[[]], terminal_rows=2)))
    # every state pinned at stage 2 (n-bar_2 = 0)
    out.append(("pinned-state", tiny_problem(305, N=4, n=2, m=2, kinds=[[], [], ["state", "state"], []],
                                             terminal_rows=0)))
    # inputs fully determined (m-bar = 0): as many mixed rows as inputs
    out.append(("no-free-input", tiny_problem(306, N=4, n=3, m=2, kinds=[["mixed", "mixed"]] * 4,
                                              terminal_rows=0, g_mode="random")))
    out.append(("with-M", tiny_problem(307, N=5, n=3, m=2, terminal_rows=1, with_M=True)))
    out.append(("random-g-mixed", tiny_problem(308, N=7, n=3, m=3, kinds=[["mixed"]] * 7, terminal_rows=2,
                                               g_mode="random")))
    # one input and a state row per stage: long-interval relations keep rows
    out.append(("state-heavy", tiny_problem(309, N=8, n=4, m=1, kinds=[["state"]] * 8, terminal_rows=2)))
    return out


def indefinite_cost_problems():
    """Instances whose costs are indefinite only along directions the
    constraints fix, so the reduced problem is strictly convex: R_i with
    eigenvalue -2 along the u-direction of a mixed row, and Q_i with
    eigenvalue -2 along the normal of a state row (stages 1..N, terminal row
    included).  A third instance leaves the negative direction of R_1 free."""
    p1 = tiny_problem(1301, N=5, n=3, m=2, kinds=[["mixed"]] * 5, terminal_rows=0)
    for i in range(p1.N):
        d = p1.F[i][0] / np.linalg.norm(p1.F[i][0])
        p1.R[i] = np.eye(2) - 3.0 * np.outer(d, d)
    p2 = tiny_problem(1302, N=5, n=3, m=2, kinds=[["state"]] * 5, terminal_rows=1)
    for i in range(1, p2.N + 1):
        e = p2.E[i][0] / np.linalg.norm(p2.E[i][0])
        p2.Q[i] = np.eye(3) - 3.0 * np.outer(e, e)
    p3 = tiny_problem(1303, N=4, n=3, m=2, kinds=[[]] * 4, terminal_rows=0)
    p3.R[1] = np.diag([1.0, -1.0])
    return p1, p2, p3
