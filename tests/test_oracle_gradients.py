"""Pins of the oracle's implicit-differentiation gradients: central finite
differences through the sequential solve, and the dense adjoint KKT solve."""

from __future__ import annotations

import numpy as np
import pytest

from oracle import solve_with_multipliers
from oracle.dense import dense_kkt, split_dual, split_primal
from oracle.gradients import (adjoint_gradients, directional, effective_direction, fd_directional,
                              fd_directional_all, fd_directional_corrected,
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


def test_multiplier_cotangents_vs_dense_adjoint():
    """A loss that reads lambda and mu: the oracle's adjoint (offsets from
    dL/dlam, dL/dmu) against K a = -[dL/dw; dL/dnu] solved densely, with
    dL/dalpha = -dL/dlambda_0."""
    name, p = _cases()[0]
    sol = solve_with_multipliers(p)
    rng = np.random.default_rng(77)
    gx = [rng.standard_normal(v.shape) for v in sol["x"]]
    gu = [rng.standard_normal(v.shape) for v in sol["u"]]
    gl = [rng.standard_normal(v.shape) for v in sol["lam"]]
    gm = [rng.standard_normal(v.shape) for v in sol["mu"]]
    H, h, J, b, layout = dense_kkt(p)
    _, _, ao, lo, mo = layout
    nw, nn = H.shape[0], J.shape[0]
    gnu = np.zeros(nn)
    gnu[ao:ao + p.nx[0]] = -gl[0]
    for i in range(1, p.N + 1):
        gnu[lo[i]:lo[i] + p.nx[i]] = gl[i]
    for i in range(p.N + 1):
        gnu[mo[i]:mo[i] + p.nc[i]] = gm[i]
    K = np.block([[H, J.T], [J, np.zeros((nn, nn))]])
    gw = np.concatenate([np.concatenate([gx[i], gu[i]]) for i in range(p.N)] + [gx[p.N]])
    a = np.linalg.solve(K, -np.concatenate([gw, gnu]))
    ap = split_primal(p, a[:nw], layout)
    ad = split_dual(p, a[nw:], layout)
    G = adjoint_gradients(p, sol, gx, gu, gl, gm)
    assert rel_err(G["q"], ap["x"]) < 1e-10
    assert rel_err(G["r"], ap["u"]) < 1e-10
    assert rel_err(G["c"], ad["lam"][1:]) < 1e-10
    assert rel_err(G["g"], ad["mu"]) < 1e-10
    assert np.allclose(G["x0"], ad["lam"][0], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("name,p", _cases(), ids=[c[0] for c in _cases()])
def test_multiplier_loss_gradients_vs_central_fd(name, p):
    """L = sum |x|^2 + |u|^2 + |lambda|^2 + |mu|^2 (unique multipliers: every
    case has independent rows): the adjoint's directional derivative against
    a central difference of two full solves with multipliers."""
    sol = solve_with_multipliers(p)
    gx, gu = sumsq_loss_grad(sol["x"], sol["u"])
    gl = [2.0 * v for v in sol["lam"]]
    gm = [2.0 * v for v in sol["mu"]]
    G = adjoint_gradients(p, sol, gx, gu, gl, gm)
    rng = np.random.default_rng(19)
    for _ in range(3):
        d = random_direction(p, rng)
        an = directional(G, effective_direction(p, d, 1e-4))
        fd = fd_directional_all(p, d, 1e-4)
        assert abs(fd - an) / max(abs(fd), abs(an)) < 1e-5, (fd, an)
