"""Primal-dual interior-point driver for bound-constrained LQR problems
(TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``).

The paper's motivation (Section I) is that interior-point and SQP methods
solve a sequence of equality-constrained LQR problems with the same
structure and new diagonal weights.  This module states that use plainly:
eq. (problem) plus bounds lo <= u_i <= hi on the inputs and lo <= x_i <= hi
on the states after x_0 (an infinite bound is absent), solved by Mehrotra's
predictor-corrector primal-dual method (S. Mehrotra, "On the implementation
of a primal-dual interior point method", SIAM J. Optim. 2(4), 1992), whose
two linear systems per iteration are each one such LQR, solved by the
oracle's sequential method with minimum-norm multipliers.

With bound multipliers z_lo, z_hi >= 0, d_lo = w - lo, d_hi = hi - w and
per-bound complementarity targets t_lo, t_hi, eliminating dz from the
linearised optimality conditions
    grad f(w) + J' nu - z_lo + z_hi = 0,  c(w) = 0,
    z_lo d_lo = t_lo,  z_hi d_hi = t_hi
gives, for the step dw and the new equality multipliers nu+, the
equality-constrained quadratic problem
    min 1/2 dw' (H + S) dw + g' dw   s.t.  J dw + c(w) = 0,
    S = diag(z_lo / d_lo + z_hi / d_hi),
    g = grad f(w) - t_lo / d_lo + t_hi / d_hi,
whose multipliers are nu+; then
    dz_lo = t_lo / d_lo - z_lo - (z_lo / d_lo) dw,
    dz_hi = t_hi / d_hi - z_hi + (z_hi / d_hi) dw.
One iteration, with mu the instance's mean complementarity product:
  1. predictor: targets 0; its largest step a_aff <= 1 keeping d and z
     non-negative, and mu_aff, the mean complementarity after that step;
  2. sigma = min(1, (mu_aff / mu)^3);
  3. corrector: the same matrices with targets
         t_lo = sigma mu - dz_lo_aff dw_aff,  t_hi = sigma mu + dz_hi_aff dw_aff
     (the second-order term of the complementarity products);
  4. step a = min(1, tau * largest step keeping d and z non-negative) for
     (w, z), and nu <- nu + a (nu+ - nu).
The start point is the equality-constrained solution moved inside the
bounds with z = MU0 / distance.  At most a fixed number of iterations is
taken (the device driver runs the same count); an instance stops once its
mean complementarity is below MU_STOP.
"""

from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

from .multipliers import objective_gradients, solve_with_multipliers

TAU = 0.995
MU0 = 100.0
MU_STOP = 1e-8  # an instance stops once its mean complementarity is below this
INTERIOR = 0.25  # initial point: at least this fraction of the bound gap inside


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


def _interior(v, lo, hi, frac=INTERIOR):
    """Move v inside [lo, hi]: at least frac of the gap (two-sided) or
    frac * max(1, |bound|) (one-sided) from each finite bound."""
    v = np.array(v, float)
    two = np.isfinite(lo) & np.isfinite(hi)
    gap = np.where(two, hi - lo, 0.0)
    off_lo = np.where(two, frac * gap, frac * np.maximum(1.0, np.abs(np.where(np.isfinite(lo), lo, 0.0))))
    off_hi = np.where(two, frac * gap, frac * np.maximum(1.0, np.abs(np.where(np.isfinite(hi), hi, 0.0))))
    v = np.where(np.isfinite(lo), np.maximum(v, lo + off_lo), v)
    v = np.where(np.isfinite(hi), np.minimum(v, hi - off_hi), v)
    return v


class _Var:
    """One block of bounded variables (u_i or x_i) with its bounds and bound
    multipliers; absent bounds are masked out of every product."""

    def __init__(self, v, lo, hi):
        self.v, self.lo, self.hi = v, lo, hi
        self.fl, self.fh = np.isfinite(lo), np.isfinite(hi)
        self.zl = np.zeros_like(v)
        self.zh = np.zeros_like(v)

    def gaps(self, v=None):
        v = self.v if v is None else v
        return np.where(self.fl, v - np.where(self.fl, self.lo, 0.0), 1.0), \
            np.where(self.fh, np.where(self.fh, self.hi, 0.0) - v, 1.0)

    def products(self):
        dl, dh = self.gaps()
        return float(np.sum((self.zl * dl)[self.fl]) + np.sum((self.zh * dh)[self.fh])), \
            int(self.fl.sum() + self.fh.sum())

    def newton_terms(self, tl, th):
        """Diagonal S and the barrier part of the linear term for targets tl, th."""
        dl, dh = self.gaps()
        S = np.where(self.fl, self.zl / dl, 0.0) + np.where(self.fh, self.zh / dh, 0.0)
        gb = np.where(self.fl, -tl / dl, 0.0) + np.where(self.fh, th / dh, 0.0)
        return S, gb

    def dz(self, dv, tl, th):
        dl, dh = self.gaps()
        return (np.where(self.fl, tl / dl - self.zl - self.zl / dl * dv, 0.0),
                np.where(self.fh, th / dh - self.zh + self.zh / dh * dv, 0.0))

    def max_step(self, dv, dzl, dzh):
        """Largest a with v + a dv inside the bounds and z + a dz >= 0 (inf if none binds)."""
        dl, dh = self.gaps()
        a = np.inf
        for ok, num, den in ((self.fl & (dv < 0), dl, -dv), (self.fh & (dv > 0), dh, dv),
                             (self.fl & (dzl < 0), self.zl, -dzl), (self.fh & (dzh < 0), self.zh, -dzh)):
            if np.any(ok):
                a = min(a, float(np.min(num[ok] / den[ok])))
        return a

    def products_after(self, a, dv, dzl, dzh):
        dl, dh = self.gaps(self.v + a * dv)
        return float(np.sum(((self.zl + a * dzl) * dl)[self.fl]) + np.sum(((self.zh + a * dzh) * dh)[self.fh]))


def ipm_solve(prob, bounds: Dict[str, Optional[List[np.ndarray]]], iterations: int = 30, mu_stop: float = MU_STOP,
              tau: float = TAU, mu0: float = MU0, interior: float = INTERIOR) -> Dict:
    """Returns x, u, lam, mu (equality multipliers), z_u, z_x (bound
    multipliers per block: (lower, upper)), mu_history (mean complementarity
    at the start of each iteration) and steps (Newton iterations taken)."""
    N = prob.N
    ulo, uhi, xlo, xhi = _blocks(prob, bounds)
    start = solve_with_multipliers(prob)
    if start["status"] != "ok":
        return {"status": "start_" + start["status"]}
    U = [_Var(_interior(start["u"][i], ulo[i], uhi[i], interior), ulo[i], uhi[i]) for i in range(N)]
    X = [_Var(np.array(start["x"][0], float), xlo[0], xhi[0])] + \
        [_Var(_interior(start["x"][i], xlo[i], xhi[i], interior), xlo[i], xhi[i]) for i in range(1, N + 1)]
    blocks = U + X  # u_0..u_{N-1}, x_0..x_N
    for b in blocks:
        dl, dh = b.gaps()
        b.zl = np.where(b.fl, mu0 / dl, 0.0)
        b.zh = np.where(b.fh, mu0 / dh, 0.0)
    lam = [v.copy() for v in start["lam"]]
    mu = [v.copy() for v in start["mu"]]
    hist: List[float] = []
    steps = 0

    def newton(targets):
        x = [b.v for b in X]
        u = [b.v for b in U]
        gx, gu = objective_gradients(prob, x, u)
        nw = prob.copy()
        for i in range(N):
            S, gb = U[i].newton_terms(*targets[i])
            nw.R[i] = prob.R[i] + np.diag(S)
            nw.r[i] = gu[i] + gb
            nw.c[i] = prob.A[i] @ x[i] + prob.B[i] @ u[i] + prob.c[i] - x[i + 1]
            nw.g[i] = prob.E[i] @ x[i] + prob.F[i] @ u[i] + prob.g[i]
        for i in range(N + 1):
            S, gb = X[i].newton_terms(*targets[N + i])
            nw.Q[i] = prob.Q[i] + np.diag(S)
            nw.q[i] = gx[i] + gb
        nw.g[N] = prob.E[N] @ x[N] + prob.g[N]
        nw.x0 = prob.x0 - x[0]
        return solve_with_multipliers(nw)

    for _ in range(iterations):
        prods = [b.products() for b in blocks]
        count = sum(c for _, c in prods)
        mu_b = sum(p for p, _ in prods) / max(count, 1)
        hist.append(mu_b)
        if mu_b < mu_stop:
            break
        # 1. predictor (affine scaling direction)
        zero = [(np.zeros_like(b.v), np.zeros_like(b.v)) for b in blocks]
        aff = newton(zero)
        if aff["status"] != "ok":
            return {"status": "newton_" + aff["status"], "mu_history": hist}
        dv_aff = list(aff["u"]) + list(aff["x"])
        dz_aff = [b.dz(dv, 0.0, 0.0) for b, dv in zip(blocks, dv_aff)]
        a_aff = min(1.0, min(b.max_step(dv, *dz) for b, dv, dz in zip(blocks, dv_aff, dz_aff)))
        mu_aff = sum(b.products_after(a_aff, dv, *dz) for b, dv, dz in zip(blocks, dv_aff, dz_aff)) / max(count, 1)
        # 2. centering
        sigma = min(1.0, (mu_aff / mu_b) ** 3)
        # 3. corrector: same matrices, second-order targets
        targets = [(sigma * mu_b - dzl * dv, sigma * mu_b + dzh * dv) for dv, (dzl, dzh) in zip(dv_aff, dz_aff)]
        cor = newton(targets)
        if cor["status"] != "ok":
            return {"status": "newton_" + cor["status"], "mu_history": hist}
        dv = list(cor["u"]) + list(cor["x"])
        dz = [b.dz(d, *t) for b, d, t in zip(blocks, dv, targets)]
        # 4. step
        a = min(1.0, tau * min(b.max_step(d, *z) for b, d, z in zip(blocks, dv, dz)))
        for b, d, (dzl, dzh) in zip(blocks, dv, dz):
            b.v = b.v + a * d
            b.zl = b.zl + a * dzl
            b.zh = b.zh + a * dzh
        lam = [p + a * (q - p) for p, q in zip(lam, cor["lam"])]
        mu = [p + a * (q - p) for p, q in zip(mu, cor["mu"])]
        steps += 1
    return {"status": "ok", "x": [b.v for b in X], "u": [b.v for b in U], "lam": lam, "mu": mu,
            "z_u": [(b.zl, b.zh) for b in U], "z_x": [(b.zl, b.zh) for b in X], "mu_history": hist,
            "steps": steps}
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
