"""KKT residual of Section IX: initial condition, dynamics, equality feasibility
and stationarity (eqs. (stage-stationarity), (terminal-stationarity)), infinity
norm.  Each equality row is divided by the maximum of one and the magnitudes of
its coefficients and offset."""

from __future__ import annotations

from typing import Dict

import numpy as np


def _inf(v) -> float:
    v = np.asarray(v)
    return float(np.max(np.abs(v))) if v.size else 0.0


def kkt_residual(prob, x, u, lam, mu) -> Dict[str, float]:
    N = prob.N
    init = _inf(x[0] - prob.x0)
    dyn = max([_inf(prob.A[i] @ x[i] + prob.B[i] @ u[i] + prob.c[i] - x[i + 1]) for i in range(N)] + [0.0])
    eq = 0.0
    for i in range(N + 1):
        E, g = prob.E[i], prob.g[i]
        F = prob.F[i] if i < N else np.zeros((E.shape[0], 0))
        uu = u[i] if i < N else np.zeros(0)
        for j in range(E.shape[0]):
            row = E[j] @ x[i] + F[j] @ uu + g[j]
            den = max(1.0, _inf(E[j]), _inf(F[j]), abs(float(g[j])))
            eq = max(eq, abs(float(row)) / den)
    stat = 0.0
    if lam is not None:
        for i in range(N):
            gx = prob.Q[i] @ x[i] + prob.M[i] @ u[i] + prob.q[i]
            gu = prob.M[i].T @ x[i] + prob.R[i] @ u[i] + prob.r[i]
            sx = gx - lam[i] + prob.A[i].T @ lam[i + 1] + prob.E[i].T @ mu[i]
            su = gu + prob.B[i].T @ lam[i + 1] + prob.F[i].T @ mu[i]
            stat = max(stat, _inf(sx), _inf(su))
        gxN = prob.Q[N] @ x[N] + prob.q[N]
        stat = max(stat, _inf(gxN - lam[N] + prob.E[N].T @ mu[N]))
    return {"initial": init, "dynamics": dyn, "equality": eq, "stationarity": stat,
            "total": max(init, dyn, eq, stat)}
