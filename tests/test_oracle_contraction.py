"""Pins of the oracle's contraction-expansion multipliers (Section VII)
against the plain definition: the stationarity equations of eq. (problem),
assembled densely (J' nu = -(H w + h) at the primal solution), and the
minimum-norm multipliers where the constraint rows are independent (there
the multipliers are unique, so every valid route must return them)."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import rows_independent, solve_sequential, solve_with_multipliers
from oracle.contraction import contraction_expansion
from oracle.dense import _offsets, dense_kkt
from tests._util import problem_family, rel_err, tiny_problem
from workloads import config_c1, config_c4


def _cases():
    out = list(problem_family())
    out += [("c1-40", config_c1(N=40)[0]), ("c4-20", config_c4(B=1, N=20)[0]),
            ("redundant", tiny_problem(1601, N=5, n=3, m=2, kinds=[["mixed"]] * 5, terminal_rows=0, redundant=(2,))),
            ("state-row-0", tiny_problem(1602, N=4, n=3, m=2, kinds=[["state"], [], ["mixed"], []], terminal_rows=0))]
    return out


def _dense_stationarity(p, x, u, lam, mu):
    """|| J' nu + H w + h ||_inf with nu in the dense ordering (alpha = -lambda_0)."""
    H, h, J, b, layout = dense_kkt(p)
    xo, uo, nw, ao, lo, mo, nnu = _offsets(p)
    w = np.zeros(nw)
    for i in range(p.N + 1):
        w[xo[i]:xo[i] + p.nx[i]] = x[i]
    for i in range(p.N):
        w[uo[i]:uo[i] + p.nu[i]] = u[i]
    nu = np.zeros(nnu)
    nu[ao:ao + p.nx[0]] = -lam[0]
    for i in range(1, p.N + 1):
        nu[lo[i]:lo[i] + p.nx[i]] = lam[i]
    for i in range(p.N + 1):
        nu[mo[i]:mo[i] + p.nc[i]] = mu[i]
    return float(np.max(np.abs(J.T @ nu + H @ w + h))), float(np.max(np.abs(nu), initial=1.0))


@pytest.mark.parametrize("name,p", _cases(), ids=[c[0] for c in _cases()])
def test_contraction_expansion_is_a_multiplier(name, p):
    o = solve_with_multipliers(p)
    cx = contraction_expansion(p, o["x"], o["u"])
    assert cx["status"] == "ok"
    if sum(p.nx) + sum(p.nu) <= 800:
        res, scale = _dense_stationarity(p, o["x"], o["u"], cx["lam"], cx["mu"])
        assert res <= 1e-10 * scale, (res, scale)
    if rows_independent(p, solve_sequential(p)):
        assert rel_err(cx["lam"], o["lam"]) <= 1e-10
        if sum(p.nc):
            assert rel_err(cx["mu"], o["mu"]) <= 1e-10


def test_contraction_expansion_differs_where_rows_are_dependent():
    """With dependent rows the route returns a valid representative that is
    not the minimum-norm one (its norm is larger)."""
    p = tiny_problem(309, N=8, n=4, m=1, kinds=[["state"]] * 8, terminal_rows=2)
    assert not rows_independent(p, solve_sequential(p))
    o = solve_with_multipliers(p)
    cx = contraction_expansion(p, o["x"], o["u"])
    res, scale = _dense_stationarity(p, o["x"], o["u"], cx["lam"], cx["mu"])
    assert res <= 1e-10 * scale
    nrm = lambda d: np.sqrt(sum(float(v @ v) for k in ("lam", "mu") for v in d[k]))  # noqa: E731
    assert nrm(cx) > nrm(o) * (1 + 1e-6)
