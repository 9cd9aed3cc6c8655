"""The two multiplier routes of the kernels, restated in NumPy on the oracle's
sequential intermediates (domains H_i, bases T_i, reduced value functions and
states), checked against the oracle's minimum-norm multipliers (the plain
definition: minimum-norm solution of the stationarity equations of Section
VII).  This pins the derivations the kernels follow, not the kernels:

* factor-reusing route: lambda_i = T_i lambda-bar_i + H_i' theta_i, the stage
  systems in (mu_i, theta_{i+1}) solved one after another from theta_0 = 0 --
  a valid multiplier vector (stationarity residual at rounding level), equal
  to the minimum-norm one where the constraint Jacobian has full row rank;
* theta LQR: the minimum-norm solutions and null spaces of the same stage
  systems, then a Riccati recursion over theta (identity input cost) with a
  free initial state -- the minimum-norm multiplier itself.
"""

from __future__ import annotations

import numpy as np

from oracle import solve_with_multipliers
from oracle.dense import dense_kkt
from oracle.residual import kkt_residual
from oracle.sequential import solve_sequential
from tests._util import problem_family, rel_err


def _pinv_null(M, tol=1e-10):
    U, s, Vt = np.linalg.svd(M, full_matrices=True)
    r = int(np.sum(s > tol * max(1.0, s[0]))) if s.size else 0
    return Vt[:r].T @ np.diag(1.0 / s[:r]) @ U[:, :r].T, Vt[r:].T


def _stage_systems(prob, r):
    """Per stage: (coefficients M, normal columns [H_i'; 0], constant c)."""
    N = prob.N
    x, u = r.x, r.u
    w = [r.T[i] @ (r.P[i] @ r.z[i] + r.p[i]) for i in range(N + 1)]
    out = []
    for i in range(N + 1):
        H = r.H[i]
        gx = prob.Q[i] @ x[i] + prob.q[i]
        if i < N:
            gx = gx + prob.M[i] @ u[i]
            gu = prob.M[i].T @ x[i] + prob.R[i] @ u[i] + prob.r[i]
            H1 = r.H[i + 1]
            M = np.vstack([np.hstack([prob.E[i].T, (H1 @ prob.A[i]).T]),
                           np.hstack([prob.F[i].T, (H1 @ prob.B[i]).T])])
            Hx = np.vstack([H.T, np.zeros((prob.nu[i], H.shape[0]))])
            c = np.concatenate([w[i] - gx - prob.A[i].T @ w[i + 1], -gu - prob.B[i].T @ w[i + 1]])
        else:
            M, Hx, c = prob.E[N].T, H.T, w[N] - gx
        out.append((M, Hx, c))
    return w, out


def factor_reusing_multipliers(prob):
    r = solve_sequential(prob)
    w, sysm = _stage_systems(prob, r)
    theta = np.zeros(r.H[0].shape[0])
    lam, mu = [], []
    for i, (M, Hx, c) in enumerate(sysm):
        y, *_ = np.linalg.lstsq(M, Hx @ theta + c, rcond=None)
        k = prob.E[i].shape[0]
        lam.append(w[i] + r.H[i].T @ theta)
        mu.append(y[:k])
        theta = y[k:]
    return r.x, r.u, lam, mu


def theta_lqr_multipliers(prob):
    r = solve_sequential(prob)
    N = prob.N
    w, sysm = _stage_systems(prob, r)
    st = []
    for i, (M, Hx, c) in enumerate(sysm):
        Mp, Nb = _pinv_null(M)
        st.append((Mp @ Hx, Mp @ c, Nb if i < N else np.zeros((M.shape[1], 0)), prob.E[i].shape[0]))
    YN, yN, _, _ = st[N]
    P, p = YN.T @ YN, YN.T @ yN
    gains = [None] * N
    for i in range(N - 1, -1, -1):
        Y, y0, Nb, k = st[i]
        A, B, c = Y[k:], Nb[k:], y0[k:]
        Huu = np.eye(Nb.shape[1]) + B.T @ P @ B
        Hux, hu = B.T @ P @ A, B.T @ (P @ c + p)
        K = -np.linalg.solve(Huu, Hux) if Huu.size else np.zeros((0, A.shape[1]))
        kk = -np.linalg.solve(Huu, hu) if Huu.size else np.zeros(0)
        gains[i] = (K, kk)
        Pn = Y.T @ Y + A.T @ P @ A + Hux.T @ K
        pn = Y.T @ y0 + A.T @ (P @ c + p) + Hux.T @ kk
        P, p = 0.5 * (Pn + Pn.T), pn
    theta = -np.linalg.solve(np.eye(P.shape[0]) + P, p) if P.size else np.zeros(0)
    lam, mu = [], []
    for i in range(N + 1):
        Y, y0, Nb, k = st[i]
        lam.append(w[i] + r.H[i].T @ theta)
        if i < N:
            K, kk = gains[i]
            y = Y @ theta + Nb @ (K @ theta + kk) + y0
            mu.append(y[:k])
            theta = y[k:]
        else:
            mu.append(Y @ theta + y0)
    return r.x, r.u, lam, mu


def _unique(prob):
    _, _, J, _, _ = dense_kkt(prob)
    return J.shape[0] == 0 or np.linalg.matrix_rank(J) == J.shape[0]


def _scale(lam, mu):
    return max(1.0, max(np.abs(v).max(initial=0.0) for v in lam), max(np.abs(v).max(initial=0.0) for v in mu))


def test_factor_reusing_route_is_valid_and_unique_where_licq():
    fam = problem_family()
    kinds = set()
    for name, p in fam:
        x, u, lam, mu = factor_reusing_multipliers(p)
        o = solve_with_multipliers(p)
        assert kkt_residual(p, x, u, lam, mu)["stationarity"] <= 1e-8 * _scale(lam, mu), name
        uq = _unique(p)
        kinds.add(uq)
        if uq:
            assert rel_err(lam, o["lam"]) <= 1e-10, name
            if sum(p.nc):
                assert rel_err(mu, o["mu"]) <= 1e-10, name
    assert kinds == {True, False}


def test_theta_lqr_gives_the_minimum_norm_multiplier():
    from workloads import config_c1, config_c3
    cases = [p for _, p in problem_family()] + config_c1(N=48) + config_c3(B=2, N_range=(32, 40))
    for p in cases:
        x, u, lam, mu = theta_lqr_multipliers(p)
        o = solve_with_multipliers(p)
        assert rel_err(lam, o["lam"]) <= 1e-9
        if sum(p.nc):
            assert rel_err(mu, o["mu"]) <= 1e-9
