"""Pins of the oracle's interior-point driver for bound-constrained problems
against the plain definition of its result (the optimality conditions of the
bound-constrained quadratic problem, which fix the unique minimiser of a
strictly convex problem), against SciPy's SLSQP on a tiny instance, and
against the equality-constrained solution when no bound is active."""

from __future__ import annotations

import warnings

import numpy as np
import pytest

from oracle import solve_with_multipliers
from oracle.dense import dense_kkt, split_primal
from oracle.ipm import bound_kkt_residual, ipm_solve
from tests._util import rel_err, tiny_problem


def _box(p, frac, seed=0):
    o = solve_with_multipliers(p)
    umax = frac * max(np.abs(v).max() for v in o["u"])
    return o, {"u_lo": [np.full(p.nu[i], -umax) for i in range(p.N)],
               "u_hi": [np.full(p.nu[i], umax) for i in range(p.N)]}


@pytest.mark.parametrize("kinds,frac", [(0, 0.5), (1, 0.7), (2, 0.8)])
def test_ipm_meets_the_optimality_conditions(kinds, frac):
    p = tiny_problem(2001 + kinds, N=20, n=6, m=4, kinds=[["mixed"] * kinds] * 20, terminal_rows=0, g_mode="random")
    o, b = _box(p, frac)
    s = ipm_solve(p, b, 40)
    assert s["status"] == "ok" and s["mu_history"][-1] < 1e-8
    r = bound_kkt_residual(p, b, s)
    assert r["stationarity"] < 1e-9 and r["feasibility"] < 1e-9, r
    assert r["bound_violation"] == 0.0 and r["negative_multiplier"] == 0.0 and r["complementarity"] < 1e-7, r
    active = sum(int(np.sum(np.abs(u) > b["u_hi"][0][0] * (1 - 1e-6))) for u in s["u"])
    assert active >= 1  # the bounds bind: the solution differs from the equality-constrained one
    assert rel_err(s["u"], o["u"]) > 1e-3


def test_ipm_matches_slsqp_on_a_tiny_instance():
    from scipy.optimize import minimize
    p = tiny_problem(2010, N=4, n=3, m=2, kinds=[["mixed"]] * 4, terminal_rows=0, g_mode="random")
    o, b = _box(p, 0.6)
    s = ipm_solve(p, b, 60, mu_stop=1e-13)  # run to the optimum: the pin is the method's limit
    H, h, J, bb, layout = dense_kkt(p)
    xo, uo = layout[0], layout[1]
    nw = H.shape[0]
    lo, hi = np.full(nw, -np.inf), np.full(nw, np.inf)
    for i in range(p.N):
        lo[uo[i]:uo[i] + p.nu[i]] = b["u_lo"][i]
        hi[uo[i]:uo[i] + p.nu[i]] = b["u_hi"][i]
    w0 = np.zeros(nw)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        res = minimize(lambda w: 0.5 * w @ H @ w + h @ w, w0, jac=lambda w: H @ w + h, method="SLSQP",
                       bounds=list(zip(lo, hi)),
                       constraints=[{"type": "eq", "fun": lambda w: J @ w + bb, "jac": lambda w: J}],
                       options={"ftol": 1e-15, "maxiter": 1000})
    ref = split_primal(p, res.x, layout)
    assert rel_err(s["u"], ref["u"]) < 1e-6 and rel_err(s["x"], ref["x"]) < 1e-6


def test_ipm_with_inactive_bounds_is_the_equality_solution():
    p = tiny_problem(2020, N=10, n=4, m=2, kinds=[["mixed"]] * 10, terminal_rows=1, g_mode="random")
    o, b = _box(p, 5.0)
    s = ipm_solve(p, b, 40)
    assert rel_err(s["x"], o["x"]) < 1e-8 and rel_err(s["u"], o["u"]) < 1e-8
    assert rel_err(s["lam"], o["lam"]) < 1e-7


def test_ipm_with_state_bounds_meets_the_optimality_conditions():
    """Upper bounds on a state component (stages 1..N) beside input boxes: the
    returned point satisfies the optimality conditions of the bounded problem
    and the state bound binds somewhere."""
    p = tiny_problem(2003, N=20, n=6, m=4, kinds=[["mixed"] * 2] * 20, terminal_rows=0, g_mode="random")
    o, b = _box(p, 0.8)
    xm = 0.8 * max(abs(v[0]) for v in o["x"][1:])
    b["x_hi"] = [np.concatenate([[xm], np.full(p.nx[i] - 1, np.inf)]) for i in range(p.N + 1)]
    s = ipm_solve(p, b, 40)
    assert s["status"] == "ok" and s["mu_history"][-1] < 1e-8
    r = bound_kkt_residual(p, b, s)
    assert r["stationarity"] < 1e-9 and r["feasibility"] < 1e-9 and r["complementarity"] < 1e-7, r
    assert r["bound_violation"] == 0.0 and r["negative_multiplier"] == 0.0, r
    assert max(v[0] for v in s["x"][1:]) > xm * (1 - 1e-6)  # the state bound is active
    assert max(float(zh[0]) for _, zh in s["z_x"][1:]) > 1e-3  # with a positive multiplier


def test_ipm_without_bounds_takes_no_step():
    """No finite bound: the mean complementarity is zero, so the result is the
    equality-constrained solution itself, with no iteration."""
    p = tiny_problem(2030, N=6, n=3, m=2, kinds=[["mixed"]] * 6, terminal_rows=1, g_mode="random")
    o = solve_with_multipliers(p)
    s = ipm_solve(p, {}, 10)
    assert s["steps"] == 0 and s["mu_history"] == [0.0]
    assert rel_err(s["x"], o["x"]) == 0.0 and rel_err(s["u"], o["u"]) == 0.0
