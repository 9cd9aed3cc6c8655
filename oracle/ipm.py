"""Primal-dual interior-point driver for bound-constrained LQR problems
(TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``).

The paper's motivation (Section I) is that interior-point and SQP methods
solve a sequence of equality-constrained LQR problems with the same
structure and new diagonal weights.  This module states that use plainly:
eq. (problem) plus bounds lo <= u_i <= hi on the inputs and lo <= x_i <= hi
on the states after x_0 (an infinite bound is absent), solved by a
primal-dual path-following method whose Newton step is one such LQR,
solved by the oracle's sequential method with minimum-norm multipliers.

With bound multipliers z_lo, z_hi >= 0 and barrier target sigma * mu,
eliminating dz from the linearised optimality conditions
    grad f(w) + J' nu - z_lo + z_hi = 0,  c(w) = 0,
    z_lo (w - lo) = sigma mu,  z_hi (hi - w) = sigma mu
gives, for the step dw and the new equality multipliers nu+, the
equality-constrained quadratic problem
    min 1/2 dw' (H + S) dw + g' dw   s.t.  J dw + c(w) = 0,
    S = diag(z_lo / (w - lo) + z_hi / (hi - w)),
    g = grad f(w) - sigma mu / (w - lo) + sigma mu / (hi - w),
whose multipliers are nu+; then
    dz_lo = sigma mu / (w - lo) - z_lo - (z_lo / (w - lo)) dw,
    dz_hi = sigma mu / (hi - w) - z_hi + (z_hi / (hi - w)) dw.
Every instance takes the largest step alpha <= 1 that keeps w strictly
inside the bounds and z positive (fraction to the boundary tau); mu is the
mean complementarity product of the instance.  At most a fixed number of
iterations is taken (the device driver runs the same count); an instance
stops once its mean complementarity is below MU_STOP.
"""

from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

from .multipliers import objective_gradients, solve_with_multipliers

SIGMA = 0.1
TAU = 0.995
MU0 = 1.0
MU_STOP = 1e-10  # an instance stops once its mean complementarity is below this
INTERIOR = 0.05  # initial point: at least this fraction of the bound gap inside


def _blocks(prob, bounds):
    """Per-variable bound lists (lo, hi) as flat blocks: u_i (i < N), x_i (1 <= i <= N)."""
    N = prob.N
    ulo = bounds.get("u_lo") or [np.full(prob.nu[i], -np.inf) for i in range(N)]
    uhi = bounds.get("u_hi") or [np.full(prob.nu[i], np.inf) for i in range(N)]
    xlo = bounds.get("x_lo") or [np.full(prob.nx[i], -np.inf) for i in range(N + 1)]
    xhi = bounds.get("x_hi") or [np.full(prob.nx[i], np.inf) for i in range(N + 1)]
    xlo = [np.full(prob.nx[0], -np.inf)] + [np.asarray(v, float) for v in xlo[1:]]  # x_0 = x0 is fixed
    xhi = [np.full(prob.nx[0], np.inf)] + [np.asarray(v, float) for v in xhi[1:]]
    return [np.asarray(v, float) for v in ulo], [np.asarray(v, float) for v in uhi], xlo, xhi


def _interior(v, lo, hi):
    """Move v inside [lo, hi]: at least INTERIOR of the gap (two-sided) or
    INTERIOR * max(1, |bound|) (one-sided) from each finite bound."""
    v = np.array(v, float)
    two = np.isfinite(lo) & np.isfinite(hi)
    gap = np.where(two, hi - lo, 0.0)
    off_lo = np.where(two, INTERIOR * gap, INTERIOR * np.maximum(1.0, np.abs(np.where(np.isfinite(lo), lo, 0.0))))
    off_hi = np.where(two, INTERIOR * gap, INTERIOR * np.maximum(1.0, np.abs(np.where(np.isfinite(hi), hi, 0.0))))
    v = np.where(np.isfinite(lo), np.maximum(v, lo + off_lo), v)
    v = np.where(np.isfinite(hi), np.minimum(v, hi - off_hi), v)
    return v


def ipm_solve(prob, bounds: Dict[str, Optional[List[np.ndarray]]], iterations: int = 30) -> Dict:
    """Returns x, u, lam, mu (equality multipliers), z (bound multipliers per
    block: u_lo, u_hi, x_lo, x_hi), mu_history (mean complementarity per
    iteration) and the Newton LQR status of each iteration."""
    N = prob.N
    ulo, uhi, xlo, xhi = _blocks(prob, bounds)
    start = solve_with_multipliers(prob)
    if start["status"] != "ok":
        return {"status": "start_" + start["status"]}
    x = [v.copy() for v in start["x"]]
    u = [_interior(start["u"][i], ulo[i], uhi[i]) for i in range(N)]
    x = [x[0]] + [_interior(x[i], xlo[i], xhi[i]) for i in range(1, N + 1)]
    lam = [v.copy() for v in start["lam"]]
    mu = [v.copy() for v in start["mu"]]

    def zinit(v, lo, hi):
        zl = np.where(np.isfinite(lo), MU0 / np.where(np.isfinite(lo), v - lo, 1.0), 0.0)
        zh = np.where(np.isfinite(hi), MU0 / np.where(np.isfinite(hi), hi - v, 1.0), 0.0)
        return zl, zh

    zu = [zinit(u[i], ulo[i], uhi[i]) for i in range(N)]
    zx = [zinit(x[i], xlo[i], xhi[i]) for i in range(N + 1)]
    hist = []
    for _ in range(iterations):
        # mean complementarity over the finite bounds
        prods, count = 0.0, 0
        for v, lo, hi, (zl, zh) in [(u[i], ulo[i], uhi[i], zu[i]) for i in range(N)] + \
                                   [(x[i], xlo[i], xhi[i], zx[i]) for i in range(N + 1)]:
            fl, fh = np.isfinite(lo), np.isfinite(hi)
            prods += float(np.sum(zl[fl] * (v - lo)[fl]) + np.sum(zh[fh] * (hi - v)[fh]))
            count += int(fl.sum() + fh.sum())
        mu_b = prods / max(count, 1)
        hist.append(mu_b)
        if mu_b < MU_STOP:
            break
        target = SIGMA * mu_b
        gx, gu = objective_gradients(prob, x, u)

        def weights(v, lo, hi, zl, zh):
            fl, fh = np.isfinite(lo), np.isfinite(hi)
            dl = np.where(fl, v - lo, 1.0)
            dh = np.where(fh, hi - v, 1.0)
            S = np.where(fl, zl / dl, 0.0) + np.where(fh, zh / dh, 0.0)
            gb = np.where(fl, -target / dl, 0.0) + np.where(fh, target / dh, 0.0)
            return S, gb

        newton = prob.copy()
        for i in range(N):
            S, gb = weights(u[i], ulo[i], uhi[i], *zu[i])
            newton.R[i] = prob.R[i] + np.diag(S)
            newton.r[i] = gu[i] + gb
            newton.c[i] = prob.A[i] @ x[i] + prob.B[i] @ u[i] + prob.c[i] - x[i + 1]
            newton.g[i] = prob.E[i] @ x[i] + prob.F[i] @ u[i] + prob.g[i]
        for i in range(N + 1):
            S, gb = weights(x[i], xlo[i], xhi[i], *zx[i])
            newton.Q[i] = prob.Q[i] + np.diag(S)
            newton.q[i] = gx[i] + gb
        newton.g[N] = prob.E[N] @ x[N] + prob.g[N]
        newton.x0 = prob.x0 - x[0]
        st = solve_with_multipliers(newton)
        if st["status"] != "ok":
            return {"status": "newton_" + st["status"], "mu_history": hist}
        dx, du = st["x"], st["u"]

        def dz(v, lo, hi, zl, zh, dv):
            fl, fh = np.isfinite(lo), np.isfinite(hi)
            dl = np.where(fl, v - lo, 1.0)
            dh = np.where(fh, hi - v, 1.0)
            dzl = np.where(fl, target / dl - zl - zl / dl * dv, 0.0)
            dzh = np.where(fh, target / dh - zh + zh / dh * dv, 0.0)
            return dzl, dzh

        alpha = 1.0
        steps = []
        for v, lo, hi, (zl, zh), dv in [(u[i], ulo[i], uhi[i], zu[i], du[i]) for i in range(N)] + \
                                       [(x[i], xlo[i], xhi[i], zx[i], dx[i]) for i in range(N + 1)]:
            dzl, dzh = dz(v, lo, hi, zl, zh, dv)
            steps.append((dzl, dzh))
            fl, fh = np.isfinite(lo), np.isfinite(hi)
            for ok, num, den in ((fl & (dv < 0), v - lo, -dv), (fh & (dv > 0), hi - v, dv),
                                 (fl & (dzl < 0), zl, -dzl), (fh & (dzh < 0), zh, -dzh)):
                if np.any(ok):
                    alpha = min(alpha, TAU * float(np.min(num[ok] / den[ok])))
        for i in range(N):
            u[i] = u[i] + alpha * du[i]
            zu[i] = (zu[i][0] + alpha * steps[i][0], zu[i][1] + alpha * steps[i][1])
        for i in range(N + 1):
            x[i] = x[i] + alpha * dx[i]
            zx[i] = (zx[i][0] + alpha * steps[N + i][0], zx[i][1] + alpha * steps[N + i][1])
        lam = [a + alpha * (b - a) for a, b in zip(lam, st["lam"])]
        mu = [a + alpha * (b - a) for a, b in zip(mu, st["mu"])]
    return {"status": "ok", "x": x, "u": u, "lam": lam, "mu": mu, "z_u": zu, "z_x": zx, "mu_history": hist}


def bound_kkt_residual(prob, bounds, sol) -> Dict[str, float]:
    """Residuals of the optimality conditions of the bound-constrained
    problem at sol: stationarity grad f + J' nu - z_lo + z_hi (inf norm),
    equality feasibility (dynamics, rows, initial state), bound violation,
    negative multipliers and complementarity (max of z * gap)."""
    N = prob.N
    ulo, uhi, xlo, xhi = _blocks(prob, bounds)
    x, u, lam, mu = sol["x"], sol["u"], sol["lam"], sol["mu"]
    gx, gu = objective_gradients(prob, x, u)
    stat = 0.0
    for i in range(N + 1):
        zl, zh = sol["z_x"][i]
        sx = gx[i] - lam[i] + prob.E[i].T @ mu[i] - zl + zh
        if i < N:
            sx = sx + prob.A[i].T @ lam[i + 1]
            zul, zuh = sol["z_u"][i]
            su = gu[i] + prob.B[i].T @ lam[i + 1] + prob.F[i].T @ mu[i] - zul + zuh
            stat = max(stat, float(np.max(np.abs(su), initial=0.0)))
        stat = max(stat, float(np.max(np.abs(sx), initial=0.0)))
    feas = float(np.max(np.abs(x[0] - prob.x0), initial=0.0))
    for i in range(N):
        feas = max(feas, float(np.max(np.abs(prob.A[i] @ x[i] + prob.B[i] @ u[i] + prob.c[i] - x[i + 1]), initial=0.0)))
        feas = max(feas, float(np.max(np.abs(prob.E[i] @ x[i] + prob.F[i] @ u[i] + prob.g[i]), initial=0.0)))
    feas = max(feas, float(np.max(np.abs(prob.E[N] @ x[N] + prob.g[N]), initial=0.0)))
    viol, neg, comp = 0.0, 0.0, 0.0
    for v, lo, hi, (zl, zh) in [(u[i], ulo[i], uhi[i], sol["z_u"][i]) for i in range(N)] + \
                               [(x[i], xlo[i], xhi[i], sol["z_x"][i]) for i in range(1, N + 1)]:
        fl, fh = np.isfinite(lo), np.isfinite(hi)
        if np.any(fl):
            viol = max(viol, float(np.max(lo[fl] - v[fl])))
            neg = max(neg, float(np.max(-zl[fl])))
            comp = max(comp, float(np.max(zl[fl] * (v - lo)[fl])))
        if np.any(fh):
            viol = max(viol, float(np.max(v[fh] - hi[fh])))
            neg = max(neg, float(np.max(-zh[fh])))
            comp = max(comp, float(np.max(zh[fh] * (hi - v)[fh])))
    return {"stationarity": stat, "feasibility": feas, "bound_violation": max(viol, 0.0),
            "negative_multiplier": max(neg, 0.0), "complementarity": comp}
