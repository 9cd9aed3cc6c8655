"""Affine endpoint relations (paper Section III) and the per-stage relations of
Section IV, computed with LAPACK SVDs.

A relation over endpoints (a, b) is the set {(a, b) : L a + R b + ell = 0}
(Definition 1).  A unary relation has an empty right endpoint (R has 0 columns).

Numerical policy (Section VIII): rows are scaled before rank tests; a singular
value counts toward the rank when it exceeds ``rank_tol * max(sigma_1, 1)``; every
relation is replaced by an orthonormal row basis after each projection; a row
whose coefficients vanish is redundant when its offset is below
``cons_tol * max(1, |offsets|_inf)`` and inconsistent otherwise.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

RANK_TOL = 1e-10
CONS_TOL = 1e-8


@dataclass
class Relation:
    L: np.ndarray      # rows x n_a
    R: np.ndarray      # rows x n_b (n_b = 0 for a unary relation)
    ell: np.ndarray    # rows
    consistent: bool = True

    @property
    def rows(self) -> int:
        return self.L.shape[0]


def numerical_rank(s: np.ndarray, rank_tol: float = RANK_TOL) -> int:
    """Count of singular values above the relative threshold (Section VIII, item 2)."""
    if s.size == 0:
        return 0
    return int(np.sum(s > rank_tol * max(float(s[0]), 1.0)))


def scale_rows(Cm: np.ndarray, off: np.ndarray):
    """Section VIII item 1: divide each equation by the 2-norm of its coefficients."""
    nrm = np.linalg.norm(Cm, axis=1) if Cm.shape[1] else np.zeros(Cm.shape[0])
    s = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 1.0)
    return Cm * s[:, None], off * s


def project_out(Fm: np.ndarray, Gm: np.ndarray, gv: np.ndarray, rank_tol: float = RANK_TOL):
    """Lemma 1: exists y with F y + G z + g = 0  <=>  W^T (G z + g) = 0, where the
    columns of W are a basis of null(F^T).  W is read off a full SVD of F."""
    p = Fm.shape[0]
    if Fm.shape[1] == 0 or p == 0:
        return Gm.copy(), gv.copy()
    U, s, _ = np.linalg.svd(Fm, full_matrices=True)
    rk = numerical_rank(s, rank_tol)
    W = U[:, rk:]
    return W.T @ Gm, W.T @ gv


def row_basis(Gm: np.ndarray, gv: np.ndarray, rank_tol: float = RANK_TOL, cons_tol: float = CONS_TOL):
    """Section VIII items 3-4: replace G z + g = 0 by an orthonormal row basis
    Vt_r z + h = 0 and report whether the dropped rows read 0 = 0 (consistent)
    or 0 = gamma with gamma != 0 (inconsistent)."""
    p, ncol = Gm.shape
    if p == 0:
        return np.zeros((0, ncol)), np.zeros(0), True
    scale = max(1.0, float(np.max(np.abs(gv)))) if gv.size else 1.0
    if ncol == 0:
        return np.zeros((0, 0)), np.zeros(0), bool(np.all(np.abs(gv) <= cons_tol * scale))
    U, s, Vt = np.linalg.svd(Gm, full_matrices=True)
    r = numerical_rank(s, rank_tol)
    beta = U.T @ gv
    consistent = bool(np.all(np.abs(beta[r:]) <= cons_tol * scale))
    return Vt[:r].copy(), beta[:r] / s[:r], consistent


def make_relation(Gm: np.ndarray, gv: np.ndarray, n_a: int, rank_tol=RANK_TOL, cons_tol=CONS_TOL) -> Relation:
    H, h, ok = row_basis(Gm, gv, rank_tol, cons_tol)
    return Relation(H[:, :n_a], H[:, n_a:], h, ok)


def base_relation(A, B, c, E, F, g, rank_tol=RANK_TOL, cons_tol=CONS_TOL) -> Relation:
    """Section IV eq. (base-system) and (base-relation), with the stage's mixed and
    state-only rows merged into E x + F u + g = 0:

        [B; F] u + [[A, -I], [E, 0]] (x_i, x_{i+1}) + [c; g] = 0,

    and u projected out with Lemma 1."""
    n1, n = A.shape
    k = E.shape[0]
    Fm = np.vstack([B, F])
    Gm = np.block([[A, -np.eye(n1)], [E, np.zeros((k, n1))]])
    gv = np.concatenate([c, g])
    full, gv = scale_rows(np.hstack([Fm, Gm]), gv)
    Fm, Gm = full[:, :Fm.shape[1]], full[:, Fm.shape[1]:]
    Gp, gp = project_out(Fm, Gm, gv, rank_tol)
    return make_relation(Gp, gp, n, rank_tol, cons_tol)


def terminal_relation(EN, gN, rank_tol=RANK_TOL, cons_tol=CONS_TOL) -> Relation:
    """Section IV eq. (terminal-relation): {x_N : E_N x_N + e_N = 0}, a relation to a
    zero-dimensional endpoint."""
    Gm, gv = scale_rows(EN, gN)
    return make_relation(Gm, gv, EN.shape[1], rank_tol, cons_tol)


def compose(rab: Relation, rbc: Relation, rank_tol=RANK_TOL, cons_tol=CONS_TOL) -> Relation:
    """Section III eq. (composition-matrix): stack F = [R_ab; L_bc],
    G = blkdiag(L_ab, R_bc), offsets [ell_ab; ell_bc], and project out the shared
    endpoint b with Lemma 1."""
    n_a = rab.L.shape[1]
    n_c = rbc.R.shape[1]
    Fm = np.vstack([rab.R, rbc.L])
    Gm = np.block([[rab.L, np.zeros((rab.rows, n_c))],
                   [np.zeros((rbc.rows, n_a)), rbc.R]])
    gv = np.concatenate([rab.ell, rbc.ell])
    Gp, gp = project_out(Fm, Gm, gv, rank_tol)
    out = make_relation(Gp, gp, n_a, rank_tol, cons_tol)
    out.consistent = out.consistent and rab.consistent and rbc.consistent
    return out


def same_set(r1: Relation, r2: Relation, tol: float = 1e-9) -> bool:
    """Two affine relations describe the same set (Definition 1 equivalence):
    equal row spaces (compared through orthogonal projectors) and equal
    minimum-norm points."""
    H1 = np.hstack([r1.L, r1.R]); H2 = np.hstack([r2.L, r2.R])
    if H1.shape[0] != H2.shape[0]:
        return False
    if H1.shape[0] == 0:
        return True
    P1 = np.linalg.pinv(H1) @ H1
    P2 = np.linalg.pinv(H2) @ H2
    p1 = -np.linalg.pinv(H1) @ r1.ell
    p2 = -np.linalg.pinv(H2) @ r2.ell
    return bool(np.allclose(P1, P2, atol=tol) and np.allclose(p1, p2, atol=tol * max(1, np.abs(p1).max())))
