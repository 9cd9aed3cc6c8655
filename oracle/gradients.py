"""Gradients of a loss of the solution with respect to the problem data.

Implicit differentiation of the KKT system K [w; nu] = -[h; b] of eq. (problem)
(K symmetric, constraints J w + b = 0 with b = (-x0, c_i, g_i)): for a loss
L(w, nu), the adjoint (a_w, a_nu) solves K [a_w; a_nu] = -[dL/dw; dL/dnu],
which is the KKT system of the same constrained LQR with linear costs
q_i <- dL/dx_i, r_i <- dL/du_i and offsets b <- dL/dnu: c_i <- dL/dlambda_{i+1},
g_i <- dL/dmu_i and, since the multiplier of x_0 - x0 = 0 is alpha =
-lambda_0, x0 <- dL/dlambda_0 (all offsets zero for a loss of w alone).  Then
dL = a_w^T (dh + dH w + dJ^T nu) + a_nu^T (dJ w + db), i.e.

    dL/dq_i = a_x_i,  dL/dr_i = a_u_i,  dL/dc_i = a_lambda_{i+1},
    dL/dg_i = a_mu_i, dL/dx0 = a_lambda_0 (lambda_0 = -alpha),
    dL/dQ_i = (a_x x^T + x a_x^T)/2,  dL/dR_i = (a_u u^T + u a_u^T)/2,
    dL/dM_i = a_x u^T + x a_u^T,
    dL/dA_i = lambda_{i+1} a_x_i^T + a_lambda_{i+1} x_i^T,
    dL/dB_i = lambda_{i+1} a_u_i^T + a_lambda_{i+1} u_i^T,
    dL/dE_i = mu_i a_x_i^T + a_mu_i x_i^T,  dL/dF_i = mu_i a_u_i^T + a_mu_i u_i^T.

Valid where the multipliers are unique (LICQ) and the rank pattern is locally
constant.  The central finite difference along a direction is the independent
check.
"""

from __future__ import annotations

from typing import Callable, Dict, List

import numpy as np

from .multipliers import correction_problem, solve_with_multipliers
from .sequential import solve_sequential

FIELDS = ("Q", "q", "R", "r", "M", "A", "B", "c", "E", "F", "g")


def adjoint_problem(prob, dLdx: List[np.ndarray], dLdu: List[np.ndarray], dLdlam=None, dLdmu=None):
    adj = prob.copy()
    N = prob.N
    adj.q = [np.array(dLdx[i], dtype=np.float64) for i in range(N + 1)]
    adj.r = [np.array(dLdu[i], dtype=np.float64) for i in range(N)]
    if dLdlam is None:
        adj.c = [np.zeros_like(ci) for ci in prob.c]
        adj.x0 = np.zeros_like(prob.x0)
    else:
        adj.c = [np.array(dLdlam[i + 1], dtype=np.float64) for i in range(N)]
        adj.x0 = np.array(dLdlam[0], dtype=np.float64)
    if dLdmu is None:
        adj.g = [np.zeros_like(gi) for gi in prob.g]
    else:
        adj.g = [np.array(dLdmu[i], dtype=np.float64) for i in range(N + 1)]
    return adj


def adjoint_gradients(prob, sol: Dict, dLdx, dLdu, dLdlam=None, dLdmu=None) -> Dict[str, list]:
    """Gradients of L with respect to every field, given the forward solution
    ``sol`` (x, u, lam, mu), dL/dx, dL/du and optionally dL/dlam, dL/dmu."""
    N = prob.N
    a = solve_with_multipliers(adjoint_problem(prob, dLdx, dLdu, dLdlam, dLdmu))
    if a["status"] != "ok":
        raise RuntimeError("adjoint solve failed: " + a["status"])
    x, u, lam, mu = sol["x"], sol["u"], sol["lam"], sol["mu"]
    ax, au, al, am = a["x"], a["u"], a["lam"], a["mu"]
    G: Dict[str, list] = {}
    G["q"] = [ax[i].copy() for i in range(N + 1)]
    G["r"] = [au[i].copy() for i in range(N)]
    G["c"] = [al[i + 1].copy() for i in range(N)]
    G["g"] = [am[i].copy() for i in range(N + 1)]
    G["x0"] = al[0].copy()
    G["Q"] = [0.5 * (np.outer(ax[i], x[i]) + np.outer(x[i], ax[i])) for i in range(N + 1)]
    G["R"] = [0.5 * (np.outer(au[i], u[i]) + np.outer(u[i], au[i])) for i in range(N)]
    G["M"] = [np.outer(ax[i], u[i]) + np.outer(x[i], au[i]) for i in range(N)]
    G["A"] = [np.outer(lam[i + 1], ax[i]) + np.outer(al[i + 1], x[i]) for i in range(N)]
    G["B"] = [np.outer(lam[i + 1], au[i]) + np.outer(al[i + 1], u[i]) for i in range(N)]
    G["E"] = [np.outer(mu[i], ax[i]) + np.outer(am[i], x[i]) for i in range(N + 1)]
    G["F"] = [np.outer(mu[i], au[i]) + np.outer(am[i], u[i]) for i in range(N)]
    return G


def sumsq_loss(x, u) -> float:
    """L = sum_i |x_i|^2 + sum_i |u_i|^2."""
    return float(sum(float(xi @ xi) for xi in x) + sum(float(ui @ ui) for ui in u))


def sumsq_loss_grad(x, u):
    return [2.0 * xi for xi in x], [2.0 * ui for ui in u]


def sumsq_all_loss(sol) -> float:
    """L = sum |x_i|^2 + sum |u_i|^2 + sum |lambda_i|^2 + sum |mu_i|^2 (a loss
    that also reads the multipliers)."""
    return float(sum(float(v @ v) for k in ("x", "u", "lam", "mu") for v in sol[k]))


def fd_directional_all(prob, d, h: float = 1e-4) -> float:
    """Central difference of ``sumsq_all_loss`` through two full solves with
    multipliers (valid where the multipliers are unique)."""
    sp = solve_with_multipliers(perturbed(prob, d, h))
    sm = solve_with_multipliers(perturbed(prob, d, -h))
    if sp["status"] != "ok" or sm["status"] != "ok":
        raise RuntimeError("finite-difference solve failed")
    return (sumsq_all_loss(sp) - sumsq_all_loss(sm)) / (2.0 * h)


def perturbed(prob, d: Dict[str, list], h: float):
    p = prob.copy()
    for f in FIELDS:
        if f in d:
            setattr(p, f, [a + h * da for a, da in zip(getattr(p, f), d[f])])
    if "x0" in d:
        p.x0 = p.x0 + h * d["x0"]
    return p


def random_direction(prob, rng, fields=FIELDS + ("x0",)) -> Dict[str, list]:
    """A Gaussian direction over the given fields (Q, R symmetrised), unit 2-norm.

    Entries of F that are exactly zero stay zero: a state-only row that picks up
    an input coefficient changes the rank pattern of the reduction, where the
    solution map is not differentiable in the sense used here."""
    d: Dict[str, list] = {}
    for f in fields:
        if f == "x0":
            d[f] = rng.standard_normal(prob.x0.shape)
            continue
        out = []
        for a in getattr(prob, f):
            z = rng.standard_normal(a.shape)
            if f in ("Q", "R"):
                z = 0.5 * (z + z.T)
            if f == "F":
                z = np.where(a != 0.0, z, 0.0)
            out.append(z)
        d[f] = out
    tot = 0.0
    for f, v in d.items():
        tot += float(np.sum(v * v)) if f == "x0" else sum(float(np.sum(z * z)) for z in v)
    s = 1.0 / np.sqrt(tot)
    return {f: (v * s if f == "x0" else [z * s for z in v]) for f, v in d.items()}


def directional(G: Dict[str, list], d: Dict[str, list]) -> float:
    tot = 0.0
    for f, v in d.items():
        if f == "x0":
            tot += float(G["x0"] @ v)
        else:
            tot += sum(float(np.sum(ga * da)) for ga, da in zip(G[f], v))
    return tot


def fd_directional(prob, d, h: float = 1e-6,
                   loss: Callable = sumsq_loss) -> float:
    """Central difference (L(theta + h d) - L(theta - h d)) / 2h through the
    sequential oracle."""
    sp = solve_sequential(perturbed(prob, d, h))
    sm = solve_sequential(perturbed(prob, d, -h))
    if sp.status != "ok" or sm.status != "ok":
        raise RuntimeError("finite-difference solve failed")
    return (loss(sp.x, sp.u) - loss(sm.x, sm.u)) / (2.0 * h)


def effective_direction(prob, d, h: float):
    """The direction the rounded perturbations actually apply:
    (fl(theta + h d) - fl(theta - h d)) / 2h (the subtraction is exact), so
    that the difference quotient is compared with the derivative along the
    perturbation that was really made."""
    pp, pm = perturbed(prob, d, h), perturbed(prob, d, -h)
    out = {}
    for f, v in d.items():
        if f == "x0":
            out[f] = (pp.x0 - pm.x0) / (2.0 * h)
        else:
            out[f] = [(a - b) / (2.0 * h) for a, b in zip(getattr(pp, f), getattr(pm, f))]
    return out


def fd_directional_corrected(prob, sol, d, h: float = 1e-6) -> float:
    """Central difference (L(theta + h d) - L(theta - h d)) / 2h of the sum-of-
    squares loss, with each perturbed solution written w + delta and delta
    obtained from ``correction_problem`` (same quotient, far less cancellation
    than differencing two full solves)."""
    x, u = sol["x"], sol["u"]
    vals = []
    for sgn in (1.0, -1.0):
        cp = correction_problem(perturbed(prob, d, sgn * h), sol)
        s = solve_sequential(cp)
        if s.status != "ok":
            raise RuntimeError("correction solve failed: " + s.status)
        dl = sum(float(2.0 * x[i] @ s.x[i] + s.x[i] @ s.x[i]) for i in range(len(x)))
        dl += sum(float(2.0 * u[i] @ s.u[i] + s.u[i] @ s.u[i]) for i in range(len(u)))
        vals.append(dl)
    return (vals[0] - vals[1]) / (2.0 * h)
