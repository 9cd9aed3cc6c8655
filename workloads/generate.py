"""Seeded generators for equality-constrained LQR instances (FP64, NumPy).

The problem is the one of the paper's Section II, eq. (problem), with the mixed
rows ``C_i x_i + D_i u_i + d_i = 0`` and the state-only rows
``E_i x_i + e_i = 0`` of a stage merged into one block

    E_i x_i + F_i u_i + g_i = 0        (k_i rows; a state-only row has F = 0)

and the terminal rows ``E_N x_N + g_N = 0``.  Dimensions may vary by stage:
``x_i`` has ``n_i`` entries (i = 0..N), ``u_i`` has ``m_i`` (i < N).

Every draw uses ``numpy.random.Generator(PCG64(seed))``; batched workloads give
instance ``b`` the stream ``SeedSequence(seed).spawn(B)[b]``.  Offsets ``g`` are
either drawn directly or taken from a random feasible trajectory so that state
rows are consistent (the trajectory is steered with minimum-norm inputs that
return the state to the origin at the end of short windows, which keeps it
bounded under unstable ``A_i = I + 0.1 randn``).

Nothing here solves the constrained problem: the module only draws data.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

CONFIG_SEEDS = {"c0": 1000, "c1": 1001, "c2": 1002, "c3": 1003, "c4": 1004, "paper": 1005, "mpc": 1006}


@dataclass
class Problem:
    """One instance.  Lists are indexed by stage; ``Q, q, E, g`` have N+1 entries
    (the last one is the terminal block), the others N."""

    Q: List[np.ndarray]
    q: List[np.ndarray]
    R: List[np.ndarray]
    r: List[np.ndarray]
    M: List[np.ndarray]
    A: List[np.ndarray]
    B: List[np.ndarray]
    c: List[np.ndarray]
    E: List[np.ndarray]
    F: List[np.ndarray]
    g: List[np.ndarray]
    x0: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return len(self.R)

    @property
    def nx(self) -> List[int]:
        return [int(Qi.shape[0]) for Qi in self.Q]

    @property
    def nu(self) -> List[int]:
        return [int(Ri.shape[0]) for Ri in self.R]

    @property
    def nc(self) -> List[int]:
        return [int(Ei.shape[0]) for Ei in self.E]

    def copy(self) -> "Problem":
        cp = lambda L: [np.array(a, dtype=np.float64, copy=True) for a in L]  # noqa: E731
        return Problem(cp(self.Q), cp(self.q), cp(self.R), cp(self.r), cp(self.M),
                       cp(self.A), cp(self.B), cp(self.c), cp(self.E), cp(self.F),
                       cp(self.g), np.array(self.x0, copy=True), dict(self.meta))

    def n_stages(self) -> int:
        return self.N


# ----------------------------------------------------------------------------
# primitive draws
# ----------------------------------------------------------------------------

def _spd(rng: np.random.Generator, d: int) -> np.ndarray:
    """L L^T + 1e-2 I with L standard normal."""
    L = rng.standard_normal((d, d))
    return L @ L.T + 1e-2 * np.eye(d)


def _dynamics(rng, n0: int, n1: int, m: int):
    A = np.eye(n1, n0) + 0.1 * rng.standard_normal((n1, n0))
    B = rng.standard_normal((n1, m))
    c = 0.1 * rng.standard_normal(n1)
    return A, B, c


def feasible_trajectory(rng, A, B, c, x0, noise: float = 0.5, bound: float = 1e4, extra: int = 2):
    """A random trajectory of ``x_{i+1} = A_i x_i + B_i u_i + c_i`` that stays bounded.

    Receding-horizon minimum-energy steering: at every stage the inputs of the
    next W stages are the minimum-norm solution of "state after W stages = 0"
    (W = the fewest stages whose inputs outnumber the end state, plus ``extra``),
    only the first of them is applied, and ``noise * randn`` is added to it.
    """
    N = len(A)
    xs = [np.asarray(x0, dtype=np.float64)]
    us: List[Optional[np.ndarray]] = [None] * N
    for i in range(N):
        W, tot = 0, 0
        while i + W < N:
            tot += B[i + W].shape[1]
            W += 1
            if tot >= A[i + W - 1].shape[0] + 1:
                break
        W = min(N - i, W + extra)
        n_end = A[i + W - 1].shape[0]
        blocks, free = [], np.zeros(n_end)
        Phi = np.eye(n_end)
        for j in range(i + W - 1, i - 1, -1):
            blocks.append(Phi @ B[j])
            free = free + Phi @ c[j]
            Phi = Phi @ A[j]
        blocks.reverse()
        free = free + Phi @ xs[i]
        Rm = np.hstack(blocks)
        mi = B[i].shape[1]
        if Rm.shape[1] > 0:
            uw = np.linalg.lstsq(Rm, -free, rcond=None)[0][:mi]
        else:
            uw = np.zeros(mi)
        ui = uw + noise * rng.standard_normal(mi)
        us[i] = ui
        xs.append(A[i] @ xs[i] + B[i] @ ui + c[i])
    mx = max(float(np.max(np.abs(x))) if x.size else 0.0 for x in xs)
    mu = max((float(np.max(np.abs(u))) if u.size else 0.0) for u in us) if us else 0.0
    if not (mx < bound and mu < bound):
        raise RuntimeError(f"generated trajectory left the box: |x|max={mx:.3g} |u|max={mu:.3g}")
    return xs, us


# ----------------------------------------------------------------------------
# generic builder
# ----------------------------------------------------------------------------

def random_problem(
    rng: np.random.Generator,
    nx: Sequence[int],
    nu: Sequence[int],
    row_kinds: Sequence[Sequence[str]],
    terminal_rows: int = 0,
    redundant_stages: Sequence[int] = (),
    g_mode: str = "trajectory",
    custom_rows=None,
    with_M: bool = False,
) -> Problem:
    """Draw one instance.

    ``row_kinds[i]`` lists the kind of each constraint row of stage i:
    ``'state'`` (F row zero) or ``'mixed'`` ([E F] standard normal).
    ``custom_rows(i, rng) -> (E_i, F_i) or None`` overrides the rows of a stage.
    ``redundant_stages`` get one extra row, a Gaussian combination of the other
    rows of the stage *including* their offsets (so it stays consistent).
    ``g_mode``: 'trajectory' (offsets from a bounded random feasible trajectory)
    or 'random' (standard normal offsets).
    """
    N = len(nu)
    assert len(nx) == N + 1 and len(row_kinds) == N
    A, B, c, Q, R, M, q, r, E, F = [], [], [], [], [], [], [], [], [], []
    for i in range(N):
        Ai, Bi, ci = _dynamics(rng, nx[i], nx[i + 1], nu[i])
        A.append(Ai); B.append(Bi); c.append(ci)
        if with_M:
            # joint stage Hessian [[Q, M], [M^T, R]] = L L^T + 1e-2 I (convex, with a cross term)
            Hj = _spd(rng, nx[i] + nu[i])
            Q.append(Hj[:nx[i], :nx[i]].copy()); R.append(Hj[nx[i]:, nx[i]:].copy())
            M.append(Hj[:nx[i], nx[i]:].copy())
        else:
            Q.append(_spd(rng, nx[i])); R.append(_spd(rng, nu[i]))
            M.append(np.zeros((nx[i], nu[i])))
        q.append(rng.standard_normal(nx[i])); r.append(rng.standard_normal(nu[i]))
        rows = custom_rows(i, rng) if custom_rows is not None else None
        if rows is None:
            Er = np.zeros((len(row_kinds[i]), nx[i]))
            Fr = np.zeros((len(row_kinds[i]), nu[i]))
            for j, kind in enumerate(row_kinds[i]):
                Er[j] = rng.standard_normal(nx[i])
                if kind == "mixed":
                    Fr[j] = rng.standard_normal(nu[i])
                elif kind != "state":
                    raise ValueError(kind)
        else:
            Er, Fr = rows
        E.append(Er); F.append(Fr)
    Q.append(_spd(rng, nx[N])); q.append(rng.standard_normal(nx[N]))
    E.append(rng.standard_normal((terminal_rows, nx[N])))
    x0 = rng.standard_normal(nx[0])

    traj = None
    if g_mode == "trajectory":
        xs, us = feasible_trajectory(rng, A, B, c, x0)
        traj = (xs, us)
        g = [-(E[i] @ xs[i] + F[i] @ us[i]) for i in range(N)]
        g.append(-(E[N] @ xs[N]))
    elif g_mode == "random":
        g = [rng.standard_normal(E[i].shape[0]) for i in range(N + 1)]
    else:
        raise ValueError(g_mode)

    for i in sorted(set(redundant_stages)):
        k = E[i].shape[0]
        if k == 0:
            continue
        a = rng.standard_normal(k)
        E[i] = np.vstack([E[i], a @ E[i]])
        F[i] = np.vstack([F[i], a @ F[i]])
        g[i] = np.concatenate([g[i], [a @ g[i]]])

    p = Problem(Q, q, R, r, M, A, B, c, E, F, g, x0)
    if traj is not None:
        p.meta["trajectory"] = traj  # a feasible (x, u), for workloads that need an interior point
    return p


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def _stream(seed: int, count: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(count)]


def config_c0(seed: int = CONFIG_SEEDS["c0"]) -> List[Problem]:
    """Tiny plain case: N=16, n=4, m=2, one mixed row per stage, 2 terminal rows,
    standard normal offsets (always feasible: 1 free input per stage reaches R^4)."""
    rng = _stream(seed, 1)[0]
    N, n, m = 16, 4, 2
    p = random_problem(rng, [n] * (N + 1), [m] * N, [["mixed"]] * N, terminal_rows=2, g_mode="random")
    p.meta = {"config": "c0"}
    return [p]


def _c1_law(rng, N, n, m, kmax, terminal_rows, redundant_frac=0.1):
    kinds = []
    for _ in range(N):
        k = int(rng.integers(0, kmax + 1))
        kinds.append(["state" if rng.random() < 0.5 else "mixed" for _ in range(k)])
    cand = [i for i in range(N) if len(kinds[i]) >= 1]
    nred = min(len(cand), int(np.ceil(redundant_frac * N)))
    red = sorted(rng.choice(cand, size=nred, replace=False).tolist()) if nred else []
    return random_problem(rng, [n] * (N + 1), [m] * N, kinds, terminal_rows=terminal_rows,
                          redundant_stages=red, g_mode="trajectory")


def config_c1(seed: int = CONFIG_SEEDS["c1"], N: int = 1024) -> List[Problem]:
    """N=1024, n=12, m=6, k_i uniform in {0..4} (each row state-only w.p. 1/2),
    a redundant row on 10% of the stages, 3 terminal rows, trajectory offsets."""
    rng = _stream(seed, 1)[0]
    p = _c1_law(rng, N, 12, 6, 4, 3)
    p.meta = {"config": "c1"}
    return [p]


def config_c2(seed: int = CONFIG_SEEDS["c2"], N: int = 8192) -> List[Problem]:
    """Long DAE-like horizon: N=8192, n=32, m=16.  The last 6 inputs are algebraic
    variables tied by 6 mixed rows F = [randn(6x10), I_6 + 0.1 randn(6x6)];
    stages 8, 16, ..., N-8 carry 4 more state-only rows; no terminal rows."""
    rng = _stream(seed, 1)[0]
    n, m = 32, 16

    def rows(i, rg):
        Ea = rg.standard_normal((6, n))
        Fa = np.hstack([rg.standard_normal((6, 10)), np.eye(6) + 0.1 * rg.standard_normal((6, 6))])
        if i > 0 and i % 8 == 0 and i <= N - 8:
            Es = rg.standard_normal((4, n))
            return np.vstack([Ea, Es]), np.vstack([Fa, np.zeros((4, m))])
        return Ea, Fa

    kinds = [["mixed"] * 6 for _ in range(N)]
    p = random_problem(rng, [n] * (N + 1), [m] * N, kinds, terminal_rows=0, g_mode="trajectory",
                       custom_rows=rows)
    p.meta = {"config": "c2"}
    return [p]


def config_c3(seed: int = CONFIG_SEEDS["c3"], B: int = 512, N_range=(32, 512)) -> List[Problem]:
    """512 instances: N uniform in [32,512], n in [6,24], m in [3,12] per instance,
    k_i uniform in {0..m-1} per stage, otherwise the N=1024 law; terminal rows min(3, n-1)."""
    out = []
    for rng in _stream(seed, B):
        N = int(rng.integers(N_range[0], N_range[1] + 1))
        n = int(rng.integers(6, 25))
        m = int(rng.integers(3, 13))
        p = _c1_law(rng, N, n, m, m - 1, min(3, n - 1))
        p.meta = {"config": "c3"}
        out.append(p)
    return out


def config_c4(seed: int = CONFIG_SEEDS["c4"], B: int = 256, N: int = 128) -> List[Problem]:
    """Differentiable batch: 256 instances, N=128, n=16, m=8, 3 mixed rows per stage,
    standard normal offsets, no state-only or terminal rows."""
    out = []
    for rng in _stream(seed, B):
        p = random_problem(rng, [16] * (N + 1), [8] * N, [["mixed"] * 3] * N, terminal_rows=0,
                           g_mode="random")
        p.meta = {"config": "c4"}
        out.append(p)
    return out


def config_paper(N: int, seed: int = CONFIG_SEEDS["paper"]) -> List[Problem]:
    """The paper's benchmark shape (Section IX): n=8, m=4, two state-only rows on
    every nonterminal stage, trajectory offsets."""
    rng = _stream(seed, 1)[0]
    p = random_problem(rng, [8] * (N + 1), [4] * N, [["state", "state"]] * N, terminal_rows=0,
                       g_mode="trajectory")
    p.meta = {"config": "paper", "N": N}
    return [p]


def config_mpc(seed: int = CONFIG_SEEDS["mpc"], B: int = 256, N: int = 128, width: float = 0.5) -> List[Problem]:
    """Bound-constrained batch for the interior-point driver: the differentiable
    batch's shape (256 instances, N=128, n=16, m=8, 3 mixed rows per stage),
    offsets from a bounded random feasible trajectory, and box bounds on every
    input at +-width around that trajectory's inputs, so the bounded problem is
    feasible with the trajectory strictly inside (p.meta["bounds"]: u_lo, u_hi
    per stage)."""
    out = []
    for rng in _stream(seed, B):
        p = random_problem(rng, [16] * (N + 1), [8] * N, [["mixed"] * 3] * N, terminal_rows=0,
                           g_mode="trajectory")
        us = p.meta.pop("trajectory")[1]
        p.meta = {"config": "mpc", "bounds": {"u_lo": [v - width for v in us], "u_hi": [v + width for v in us]}}
        out.append(p)
    return out


def make_config(name: str, **kw) -> List[Problem]:
    return {"c0": config_c0, "c1": config_c1, "c2": config_c2, "c3": config_c3,
            "c4": config_c4, "paper": config_paper, "mpc": config_mpc}[name](**kw)
