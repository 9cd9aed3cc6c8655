"""Multipliers by the contraction-expansion procedure of Section VII, written
plainly with the oracle's relations (TEST INFRASTRUCTURE ONLY, like the rest
of ``oracle/``).

Steps, in the paper's order:

1. dual base relations: stage i's stationarity equations
   (eq. (stage-stationarity), with the mixed and state-only rows merged)
       [E_i'; F_i'] mu_i + [[-I, A_i'], [0, B_i']] (lambda_i, lambda_{i+1}) + [g^x_i; g^u_i] = 0
   with mu_i projected out (eq. (dual-base-system), Lemma 1), a relation over
   (lambda_i, lambda_{i+1}); the terminal equations g^x_N - lambda_N + E_N' mu_N = 0
   (eq. (terminal-stationarity)) give one over (lambda_N, nothing);
2. contraction: the relations of leaves 0..N and one empty leaf after them
   composed pairwise, level by level, an odd last node passing up unchanged
   (a balanced composition, as in Section IV);
3. the root relation constrains lambda_0 alone; lambda_0 is its minimum-norm
   point;
4. expansion from the root: at a composition node whose outer costates are
   known, the shared costate solves the two operand relations; the free
   coordinates are set to zero by taking the minimum-norm solution
   (eq. (middle-dual-map) with rho_j = 0);
5. leaf solves: mu_i is the minimum-norm solution of stage i's stationarity
   rows at the recovered costates.

Where the multipliers are unique (independent constraint rows) this is the
minimum-norm multiplier; otherwise it is another valid one (Proposition
(multipliers): every stationarity equation holds).
"""

from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

from .multipliers import DUAL_CONS_TOL, objective_gradients
from .relations import RANK_TOL, Relation, compose, make_relation, project_out, scale_rows


def _pinv(M: np.ndarray, rank_tol: float = RANK_TOL) -> np.ndarray:
    if M.size == 0:
        return np.zeros((M.shape[1], M.shape[0]))
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    r = int(np.sum(s > rank_tol * max(1.0, s[0]))) if s.size else 0
    return Vt[:r].T @ np.diag(1.0 / s[:r]) @ U[:, :r].T


def dual_base_relations(prob, gx, gu, rank_tol=RANK_TOL, cons_tol=DUAL_CONS_TOL) -> List[Relation]:
    """Step 1: relations D_0..D_N over (lambda_i, lambda_{i+1}) (D_N over
    (lambda_N, nothing))."""
    N = prob.N
    out = []
    for i in range(N + 1):
        n = prob.nx[i]
        if i < N:
            n1, m = prob.nx[i + 1], prob.nu[i]
            Fm = np.vstack([prob.E[i].T, prob.F[i].T])
            Gm = np.block([[-np.eye(n), prob.A[i].T], [np.zeros((m, n)), prob.B[i].T]])
            gv = np.concatenate([gx[i], gu[i]])
        else:
            n1 = 0
            Fm = prob.E[N].T
            Gm = -np.eye(n)
            gv = gx[N].copy()
        full, gv = scale_rows(np.hstack([Fm, Gm]), gv)
        Fm, Gm = full[:, :Fm.shape[1]], full[:, Fm.shape[1]:]
        Gp, gp = project_out(Fm, Gm, gv, rank_tol)
        out.append(make_relation(Gp, gp, n, rank_tol, cons_tol))
        assert out[-1].R.shape[1] == n1
    return out


def contraction_expansion(prob, x, u, rank_tol: float = RANK_TOL, cons_tol: float = DUAL_CONS_TOL) -> Dict:
    N = prob.N
    gx, gu = objective_gradients(prob, x, u)
    leaves = dual_base_relations(prob, gx, gu, rank_tol, cons_tol)
    # the empty leaf after the terminal one: a relation over (nothing, nothing)
    leaves.append(Relation(np.zeros((0, 0)), np.zeros((0, 0)), np.zeros(0)))
    dims = list(prob.nx) + [0, 0]  # costate dims at leaf boundaries 0..N+2

    # step 2: balanced contraction, keeping every composition node
    # node: (start, end, relation, left child, right child)
    level = [(j, j + 1, rel, None, None) for j, rel in enumerate(leaves)]
    consistent = all(r.consistent for r in leaves)
    while len(level) > 1:
        nxt = []
        for j in range(0, len(level), 2):
            if j + 1 < len(level):
                a, c = level[j], level[j + 1]
                rel = compose(a[2], c[2], rank_tol, cons_tol)
                consistent = consistent and rel.consistent
                nxt.append((a[0], c[1], rel, a, c))
            else:
                nxt.append(level[j])
        level = nxt
    root = level[0]

    # step 3: minimum-norm lambda_0 of the root relation L lambda_0 + ell = 0
    lam: List[Optional[np.ndarray]] = [None] * (N + 2)
    lam[0] = -_pinv(root[2].L, rank_tol) @ root[2].ell
    lam[N + 1] = np.zeros(0)

    # step 4: expansion, top-down
    def expand(node):
        s, e, rel, a, c = node
        if a is None:
            return
        mid = a[1]
        la, lc = a[2], c[2]
        ls = lam[s]
        le = lam[e] if e <= N + 1 else np.zeros(0)
        Mm = np.vstack([la.R, lc.L])
        rhs = -np.concatenate([la.L @ ls + la.ell, lc.R @ le + lc.ell])
        lam[mid] = _pinv(Mm, rank_tol) @ rhs if dims[mid] else np.zeros(0)
        expand(a)
        expand(c)

    expand(root)

    # step 5: leaf solves
    mu = []
    for i in range(N + 1):
        if i < N:
            Mm = np.vstack([prob.E[i].T, prob.F[i].T])
            rhs = -np.concatenate([gx[i] - lam[i] + prob.A[i].T @ lam[i + 1], gu[i] + prob.B[i].T @ lam[i + 1]])
        else:
            Mm = prob.E[N].T
            rhs = lam[N] - gx[N]
        mu.append(_pinv(Mm, rank_tol) @ rhs)
    return {"status": "ok" if consistent else "dual_inconsistent", "lam": lam[:N + 1], "mu": mu}
