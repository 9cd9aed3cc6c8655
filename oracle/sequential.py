"""The method of Algorithm 1 executed sequentially on the CPU (FP64).

Steps, in the paper's order:

1. base relations R_i (Section IV eq. (base-system)/(base-relation), Lemma 1) and
   the terminal relation R_N (eq. (terminal-relation));
2. suffix relations S_i = R_i o S_{i+1} (eq. (suffix-relation)), composed right to
   left with eq. (composition-matrix) -- one valid parenthesization
   (Proposition 1); S_i is the unary relation H_i x_i + h_i = 0
   (eq. (domain-equations));
3. state parameterization T_i, t_i, S_i (eqs. (state-param), (state-domain),
   (left-inverse)): T_i an orthonormal basis of null(H_i), t_i the minimum-norm
   point, S_i = T_i^T;
4. initial feasibility (eq. (initial-feasibility)) and z_0 (eq. (reduced-initial));
5. stage elimination (Section V): Gamma_i, Phi_i, gamma_i
   (eq. (local-control-matrices)), Y_i, Z_i, y_i (Lemma 2 with the Moore-Penrose
   inverse), reduced dynamics (eq. (reduced-dynamics-data)), reduced costs
   (eqs. (state-cost-data), (reduced-cost-data), (stage-constant),
   (terminal-cost-data));
6. the reduced unconstrained LQR solved by the textbook backward Riccati
   recursion and a forward rollout (Section VI allows any LQR solver);
7. recovery x_i = T_i z_i + t_i, u_i = Y_i z_i + Z_i v_i + y_i (eq. (recovery-maps)).

The mixed and state-only rows of a stage are merged (E_i x + F_i u + g_i = 0);
a state-only row is one whose F part is zero.  Including such rows in Gamma_i
adds zero rows whose Phi/gamma parts vanish on X_i, which is the consistency
check the paper suggests after Lemma 2.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .relations import (CONS_TOL, RANK_TOL, Relation, base_relation, compose,
                        numerical_rank, terminal_relation)


@dataclass
class SequentialResult:
    status: str
    stage: int = -1
    x: List[np.ndarray] = field(default_factory=list)
    u: List[np.ndarray] = field(default_factory=list)
    # intermediates (basis dependent; used by invariant tests only)
    H: List[np.ndarray] = field(default_factory=list)
    h: List[np.ndarray] = field(default_factory=list)
    T: List[np.ndarray] = field(default_factory=list)
    t: List[np.ndarray] = field(default_factory=list)
    Gam: List[np.ndarray] = field(default_factory=list)
    Phi: List[np.ndarray] = field(default_factory=list)
    gam: List[np.ndarray] = field(default_factory=list)
    Y: List[np.ndarray] = field(default_factory=list)
    Z: List[np.ndarray] = field(default_factory=list)
    y: List[np.ndarray] = field(default_factory=list)
    Abar: List[np.ndarray] = field(default_factory=list)
    Bbar: List[np.ndarray] = field(default_factory=list)
    cbar: List[np.ndarray] = field(default_factory=list)
    Qbar: List[np.ndarray] = field(default_factory=list)
    Mbar: List[np.ndarray] = field(default_factory=list)
    Rbar: List[np.ndarray] = field(default_factory=list)
    qbar: List[np.ndarray] = field(default_factory=list)
    rbar: List[np.ndarray] = field(default_factory=list)
    kappa: List[float] = field(default_factory=list)
    P: List[np.ndarray] = field(default_factory=list)
    p: List[np.ndarray] = field(default_factory=list)
    z: List[np.ndarray] = field(default_factory=list)
    v: List[np.ndarray] = field(default_factory=list)
    relations: List[Relation] = field(default_factory=list)
    suffix: List[Relation] = field(default_factory=list)
    objective: float = float("nan")
    reduced_objective: float = float("nan")


def objective(prob, x, u) -> float:
    """Objective of eq. (problem) with the stage cost of eq. (stage-cost)."""
    N = prob.N
    f = 0.0
    for i in range(N):
        f += 0.5 * x[i] @ prob.Q[i] @ x[i] + x[i] @ prob.M[i] @ u[i] + 0.5 * u[i] @ prob.R[i] @ u[i]
        f += prob.q[i] @ x[i] + prob.r[i] @ u[i]
    f += 0.5 * x[N] @ prob.Q[N] @ x[N] + prob.q[N] @ x[N]
    return float(f)


def _null_basis(H: np.ndarray, n: int) -> np.ndarray:
    """Orthonormal basis of null(H) for H with orthonormal rows."""
    r = H.shape[0]
    if r == 0:
        return np.eye(n)
    _, _, Vt = np.linalg.svd(H, full_matrices=True)
    return Vt[r:].T.copy()


def solve_sequential(prob, rank_tol: float = RANK_TOL, cons_tol: float = CONS_TOL,
                     keep_relations: bool = False, check_lemma2: bool = True) -> SequentialResult:
    """Algorithm 1, sequentially.  ``check_lemma2`` turns a failed consistency
    check after Lemma 2 into the status 'rank_inconsistent' (otherwise it is
    only a diagnostic)."""
    N = prob.N
    nx = prob.nx
    res = SequentialResult(status="ok")

    # -- step 1: base relations and the terminal relation (Section IV) --------
    rel = [base_relation(prob.A[i], prob.B[i], prob.c[i], prob.E[i], prob.F[i], prob.g[i],
                         rank_tol, cons_tol) for i in range(N)]
    rel.append(terminal_relation(prob.E[N], prob.g[N], rank_tol, cons_tol))

    # -- step 2: suffix relations, right to left ------------------------------
    S: List[Optional[Relation]] = [None] * (N + 1)
    S[N] = rel[N]
    for i in range(N - 1, -1, -1):
        S[i] = compose(rel[i], S[i + 1], rank_tol, cons_tol)
    if keep_relations:
        res.relations, res.suffix = rel, S
    bad = [i for i in range(N + 1) if not S[i].consistent]
    if bad:
        res.status, res.stage = "infeasible_suffix", max(bad)
        return res

    # -- step 3: state parameterization (eqs. state-param, left-inverse) ------
    for i in range(N + 1):
        H, h = S[i].L, S[i].ell
        res.H.append(H); res.h.append(h)
        res.T.append(_null_basis(H, nx[i]))
        res.t.append(-H.T @ h)

    # -- step 4: initial feasibility and reduced initial state ---------------
    x0 = prob.x0
    resid0 = res.H[0] @ x0 + res.h[0]
    scale0 = max(1.0, float(np.max(np.abs(x0))) if x0.size else 0.0,
                 float(np.max(np.abs(res.h[0]))) if res.h[0].size else 0.0)
    if resid0.size and float(np.max(np.abs(resid0))) > cons_tol * scale0:
        res.status, res.stage = "infeasible_initial", 0
        return res
    z0 = res.T[0].T @ (x0 - res.t[0])

    # -- step 5: stage elimination (Section V) --------------------------------
    for i in range(N):
        A, B, c, E, F, g = prob.A[i], prob.B[i], prob.c[i], prob.E[i], prob.F[i], prob.g[i]
        Q, M, R, q, r = prob.Q[i], prob.M[i], prob.R[i], prob.q[i], prob.r[i]
        T, t, T1, t1 = res.T[i], res.t[i], res.T[i + 1], res.t[i + 1]
        H1, h1 = res.H[i + 1], res.h[i + 1]
        Gam = np.vstack([F, H1 @ B])
        Phi = np.vstack([E @ T, H1 @ A @ T])
        gam = np.concatenate([E @ t + g, H1 @ (A @ t + c) + h1])
        # scale rows by the norms of their original coefficients [Gamma, Psi] with
        # Phi = Psi T, before the rank test (Section VIII item 1)
        Psi = np.vstack([E, H1 @ A])
        nrm = np.linalg.norm(np.hstack([Gam, Psi]), axis=1)
        sc = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 1.0)
        Gs, Ps, gs = Gam * sc[:, None], Phi * sc[:, None], gam * sc
        m = B.shape[1]
        if Gs.shape[0] and m:
            U, s, Vt = np.linalg.svd(Gs, full_matrices=True)
            rk = numerical_rank(s, rank_tol)
        else:
            U, s, Vt, rk = np.eye(Gs.shape[0]), np.zeros(0), np.eye(m), 0
        # Lemma 2 with the (rank-truncated) Moore-Penrose inverse
        Gpinv = Vt[:rk].T @ np.diag(1.0 / s[:rk]) @ U[:, :rk].T if rk else np.zeros((m, Gs.shape[0]))
        Y = -Gpinv @ Ps
        y = -Gpinv @ gs
        Z = Vt[rk:].T.copy()
        # consistency of the rank decisions (remark after Lemma 2)
        rY = Gs @ Y + Ps
        ry = Gs @ y + gs
        sc_res = max(1.0, float(np.max(np.abs(gs))) if gs.size else 0.0)
        if check_lemma2 and (
                (rY.size and float(np.max(np.abs(rY))) > cons_tol * max(1.0, float(np.max(np.abs(Ps))))) or
                (ry.size and float(np.max(np.abs(ry))) > cons_tol * sc_res)):
            res.status, res.stage = "rank_inconsistent", i
            return res
        res.Gam.append(Gam); res.Phi.append(Phi); res.gam.append(gam)
        res.Y.append(Y); res.Z.append(Z); res.y.append(y)
        # reduced dynamics, eq. (reduced-dynamics-data), S_{i+1} = T_{i+1}^T
        S1 = T1.T
        res.Abar.append(S1 @ (A @ T + B @ Y))
        res.Bbar.append(S1 @ B @ Z)
        res.cbar.append(S1 @ (A @ t + B @ y + c - t1))
        # reduced costs, eqs. (state-cost-data), (reduced-cost-data), (stage-constant)
        Qz = T.T @ Q @ T
        Mz = T.T @ M
        qz = T.T @ (Q @ t + q)
        rz = M.T @ t + r
        res.Qbar.append(Qz + Mz @ Y + Y.T @ Mz.T + Y.T @ R @ Y)
        res.Mbar.append(Mz @ Z + Y.T @ R @ Z)
        res.Rbar.append(Z.T @ R @ Z)
        res.qbar.append(qz + Mz @ y + Y.T @ (R @ y + rz))
        res.rbar.append(Z.T @ (R @ y + rz))
        res.kappa.append(float(0.5 * t @ Q @ t + q @ t + 0.5 * y @ R @ y + rz @ y))
    TN, tN = res.T[N], res.t[N]
    QbN = TN.T @ prob.Q[N] @ TN
    qbN = TN.T @ (prob.Q[N] @ tN + prob.q[N])
    res.kappa.append(float(0.5 * tN @ prob.Q[N] @ tN + prob.q[N] @ tN))

    # -- step 6: reduced unconstrained LQR, textbook Riccati recursion --------
    P = [None] * (N + 1)
    p = [None] * (N + 1)
    Kg = [None] * N
    kg = [None] * N
    P[N], p[N] = QbN, qbN
    for i in range(N - 1, -1, -1):
        Ab, Bb, cb = res.Abar[i], res.Bbar[i], res.cbar[i]
        Pn, pn = P[i + 1], p[i + 1]
        Huu = res.Rbar[i] + Bb.T @ Pn @ Bb
        Hux = res.Mbar[i].T + Bb.T @ Pn @ Ab
        hu = res.rbar[i] + Bb.T @ (Pn @ cb + pn)
        mb = Bb.shape[1]
        if mb:
            try:
                Lc = np.linalg.cholesky(0.5 * (Huu + Huu.T))
            except np.linalg.LinAlgError:
                res.status, res.stage = "not_convex", i
                return res
            Kg[i] = -np.linalg.solve(Lc.T, np.linalg.solve(Lc, Hux))
            kg[i] = -np.linalg.solve(Lc.T, np.linalg.solve(Lc, hu))
        else:
            Kg[i] = np.zeros((0, Ab.shape[1]))
            kg[i] = np.zeros(0)
        Pi = res.Qbar[i] + Ab.T @ Pn @ Ab + Hux.T @ Kg[i]
        P[i] = 0.5 * (Pi + Pi.T)
        p[i] = res.qbar[i] + Ab.T @ (Pn @ cb + pn) + Hux.T @ kg[i]
    res.P, res.p = P, p

    # forward rollout of the reduced system, eq. (reduced-dynamics)
    z = [z0]
    v = []
    for i in range(N):
        v.append(Kg[i] @ z[i] + kg[i])
        z.append(res.Abar[i] @ z[i] + res.Bbar[i] @ v[i] + res.cbar[i])
    res.z, res.v = z, v

    # -- step 7: recovery, eq. (recovery-maps) --------------------------------
    res.x = [res.T[i] @ z[i] + res.t[i] for i in range(N + 1)]
    res.u = [res.Y[i] @ z[i] + res.Z[i] @ v[i] + res.y[i] for i in range(N)]
    res.objective = objective(prob, res.x, res.u)
    fr = 0.0
    for i in range(N):
        fr += 0.5 * z[i] @ res.Qbar[i] @ z[i] + z[i] @ res.Mbar[i] @ v[i] + 0.5 * v[i] @ res.Rbar[i] @ v[i]
        fr += res.qbar[i] @ z[i] + res.rbar[i] @ v[i]
    fr += 0.5 * z[N] @ QbN @ z[N] + qbN @ z[N]
    res.reduced_objective = float(fr)
    res.Qbar.append(QbN); res.qbar.append(qbN)
    return res


def rows_independent(prob, res: SequentialResult) -> bool:
    """LICQ from the sequential method's rank decisions (any size).  The
    feasible trajectories are parameterized by the free inputs v_i alone (z_0
    is fixed by x_0 = s_0 and the map v -> (x, u) is injective), so the
    feasible set has dimension sum_i m-bar_i and rank J = dim(w) - sum_i
    m-bar_i.  J has n_0 + sum_i (n_{i+1} + k_i) + k_N rows, hence full row rank
    exactly when sum_{i<N} (m_i - m-bar_i) = sum_{i<=N} k_i.  Needs a solved
    instance (res.status == 'ok')."""
    N = prob.N
    eliminated = sum(prob.nu[i] - res.Z[i].shape[1] for i in range(N))
    return eliminated == sum(prob.nc[i] for i in range(N + 1))
