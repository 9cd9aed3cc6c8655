"""Pins of the oracle's implicit-differentiation gradients: central finite
differences through the sequential solve, and the dense adjoint KKT solve."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import solve_with_multipliers
from oracle.dense import dense_kkt, split_dual, split_primal
from oracle.gradients import (adjoint_gradients, directional, effective_direction, fd_directional,
                              fd_directional_corrected,
                              random_direction, sumsq_loss_grad)
from tests._util import rel_err, tiny_problem


def _cases():
    return [
        ("mixed", tiny_problem(600, N=6, n=4, m=3, kinds=[["mixed"]] * 6, terminal_rows=1, g_mode="random")),
        ("mixed-state", tiny_problem(601, N=5, n=4, m=3, kinds=[["mixed"], ["mixed"], ["mixed", "state"], ["mixed"], ["mixed"]],
                                     terminal_rows=0, g_mode="trajectory")),
        ("c4-like", tiny_problem(602, N=8, n=5, m=3, kinds=[["mixed"] * 2] * 8, terminal_rows=0,
                                 g_mode="random", with_M=True)),
    ]


@pytest.mark.parametrize("name,p", _cases(), ids=[c[0] for c in _cases()])
def test_gradients_vs_central_fd(name, p):
    sol = solve_with_multipliers(p)
    assert sol["status"] == "ok"
    gx, gu = sumsq_loss_grad(sol["x"], sol["u"])
    G = adjoint_gradients(p, sol, gx, gu)
    rng = np.random.default_rng(9)
    for _ in range(5):
        d = random_direction(p, rng)
        an = directional(G, effective_direction(p, d, 1e-6))
        # central difference at h = 1e-6, perturbed solutions written as w + delta
        fd = fd_directional_corrected(p, sol, d, 1e-6)
        assert abs(fd - an) / max(abs(fd), abs(an)) < 1e-6, (fd, an)
        # plain central difference of two full solves at a larger step
        fd2 = fd_directional(p, d, 1e-4)
        assert abs(fd2 - an) / max(abs(fd2), abs(an)) < 1e-4, (fd2, an)


def test_adjoint_matches_dense_adjoint():
    name, p = _cases()[0]
    sol = solve_with_multipliers(p)
    gx, gu = sumsq_loss_grad(sol["x"], sol["u"])
    H, h, J, b, layout = dense_kkt(p)
    nw, nn = H.shape[0], J.shape[0]
    K = np.block([[H, J.T], [J, np.zeros((nn, nn))]])
    gw = np.concatenate([np.concatenate([gx[i], gu[i]]) for i in range(p.N)] + [gx[p.N]])
    a = np.linalg.solve(K, -np.concatenate([gw, np.zeros(nn)]))
    ap = split_primal(p, a[:nw], layout)
    ad = split_dual(p, a[nw:], layout)
    G = adjoint_gradients(p, sol, gx, gu)
    assert rel_err(G["q"], ap["x"]) < 1e-10
    assert rel_err(G["r"], ap["u"]) < 1e-10
    assert rel_err(G["c"], ad["lam"][1:]) < 1e-10
    assert rel_err(G["g"], ad["mu"]) < 1e-10
    assert np.allclose(G["x0"], ad["lam"][0], rtol=1e-10, atol=1e-12)


def test_corrected_fd_equals_plain_fd_at_large_step():
    """The correction route evaluates the same difference quotient."""
    name, p = _cases()[0]
    sol = solve_with_multipliers(p)
    d = random_direction(p, np.random.default_rng(5))
    a = fd_directional_corrected(p, sol, d, 1e-2)
    b = fd_directional(p, d, 1e-2)
    assert abs(a - b) <= 1e-9 * max(1.0, abs(b))
