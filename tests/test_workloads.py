"""The seeded generators: determinism, the shapes the configurations promise,
feasibility by construction, and the rank gap that keeps rank decisions
unambiguous."""

from __future__ import annotations

import numpy as np

from oracle import solve_with_multipliers
from oracle.residual import kkt_residual
from workloads import config_c0, config_c1, config_c2, config_c3, config_c4, config_paper


def test_determinism():
    a, b = config_c1()[0], config_c1()[0]
    for f in ("Q", "A", "B", "E", "F", "g"):
        for x, y in zip(getattr(a, f), getattr(b, f)):
            assert np.array_equal(x, y)
    c3a, c3b = config_c3(B=3, N_range=(32, 40)), config_c3(B=3, N_range=(32, 40))
    assert [p.N for p in c3a] == [p.N for p in c3b]


def test_config_shapes():
    p = config_c0()[0]
    assert (p.N, p.nx[0], p.nu[0], p.nc[:-1], p.nc[-1]) == (16, 4, 2, [1] * 16, 2)
    p = config_c1()[0]
    assert p.N == 1024 and set(p.nx) == {12} and set(p.nu) == {6} and p.nc[-1] == 3
    assert max(p.nc[:-1]) <= 5 and min(p.nc[:-1]) == 0
    p = config_c2(N=64)[0]
    assert p.nc[8] == 10 and p.nc[9] == 6 and p.nc[-1] == 0 and p.nc[0] == 6
    ps = config_c4(B=2, N=128)
    assert all(p.N == 128 and set(p.nc[:-1]) == {3} and p.nc[-1] == 0 for p in ps)
    ps = config_c3(B=8)
    for p in ps:
        assert 32 <= p.N <= 512 and 6 <= p.nx[0] <= 24 and 3 <= p.nu[0] <= 12
        assert p.nc[-1] == min(3, p.nx[0] - 1)


def test_c2_algebraic_block_invertible():
    p = config_c2(N=16)[0]
    for i in range(16):
        Fa = p.F[i][:6, 10:]
        assert np.linalg.cond(Fa) < 1e3


def test_redundant_rows_have_rank_gap():
    p = config_c1()[0]
    gaps = []
    for i in range(p.N):
        M = np.hstack([p.E[i], p.F[i]])
        if M.shape[0] < 2:
            continue
        s = np.linalg.svd(M / np.linalg.norm(M, axis=1, keepdims=True), compute_uv=False)
        if s[-1] < 1e-12 * s[0]:
            gaps.append(s[-2] / s[0])
    assert len(gaps) >= 50
    assert min(gaps) > 1e-6


def test_generated_instances_are_feasible():
    for p in config_c0() + config_c1(N=128) + config_c3(B=4, N_range=(32, 64)) + config_paper(32):
        s = solve_with_multipliers(p)
        assert s["status"] == "ok"
        r = kkt_residual(p, s["x"], s["u"], s["lam"], s["mu"])
        assert r["total"] < 1e-8, r
