"""Gradients of the HIP adjoint (through ECLQRFunction and the C ABI) against
the oracle: the oracle's implicit-differentiation gradients (relative error
<= 1e-8 per field) and central finite differences at h = 1e-6 along random
directions over all differentiable inputs jointly (relative error <= 1e-6)."""

from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FIELDS = ("Q", "q", "R", "r", "A", "B", "c", "E", "F", "g")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gpu_grads(probs):
    import paper_2407_05433_amd as ecl
    from paper_2407_05433_amd.autograd import eclqr_layer
    plan = ecl.Plan.for_problems(probs)
    data = ecl.pack(plan, probs)
    leaves = {k: v.clone().requires_grad_(True) for k, v in data.items()}
    x, u, lam, mu, status = eclqr_layer(plan, leaves)
    loss = (x * x).sum() + (u * u).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    # split per instance / stage
    out = []
    for b, p in enumerate(probs):
        out.append({})
    for f in FIELDS + ("M", "x0"):
        if f not in leaves:
            continue
        g = leaves[f].grad.detach().cpu().numpy()
        offs, _ = plan.layout(f)
        s = 0
        for b, p in enumerate(probs):
            if f == "x0":
                out[b]["x0"] = g[offs[b]:offs[b] + p.nx[0]].copy()
                continue
            blocks = getattr(p, f)
            lst = []
            for i, a in enumerate(blocks):
                o = int(offs[s + i])
                lst.append(g[o:o + a.size].reshape(a.shape).copy())
            out[b][f] = lst
            s += p.N + 1
    return out


def _rel(a, b):
    a = np.concatenate([np.ravel(v) for v in a]) if isinstance(a, list) else np.ravel(a)
    b = np.concatenate([np.ravel(v) for v in b]) if isinstance(b, list) else np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_gradients_match_oracle_adjoint_and_fd():
    _need_gpu()
    from oracle import solve_with_multipliers
    from oracle.gradients import (adjoint_gradients, directional, effective_direction, fd_directional_corrected, random_direction,
                                  sumsq_loss_grad)
    from workloads import config_c4
    probs = config_c4(B=3)
    G = _gpu_grads(probs)
    rng = np.random.default_rng(1004)
    for b, p in enumerate(probs):
        sol = solve_with_multipliers(p)
        gx, gu = sumsq_loss_grad(sol["x"], sol["u"])
        Go = adjoint_gradients(p, sol, gx, gu)
        for f in FIELDS + ("x0",):
            assert _rel(G[b][f], Go[f]) < 1e-8, (b, f, _rel(G[b][f], Go[f]))
        fields = ("Q", "q", "R", "r", "A", "B", "c", "E", "F", "g", "x0")
        for _ in range(4):
            d = random_direction(p, rng, fields)
            an = directional(G[b], effective_direction(p, d, 1e-6))
            fd = fd_directional_corrected(p, sol, d, 1e-6)
            assert abs(fd - an) / max(abs(fd), abs(an)) < 1e-6, (b, fd, an)


def test_gradients_full_c4_batch_sampled():
    _need_gpu()
    from oracle import solve_with_multipliers
    from oracle.gradients import directional, effective_direction, fd_directional_corrected, random_direction
    from workloads import config_c4
    probs = config_c4()
    G = _gpu_grads(probs)
    rng = np.random.default_rng(4)
    for b in (0, 97, 255):
        p = probs[b]
        sol = solve_with_multipliers(p)
        for _ in range(3):
            d = random_direction(p, rng)
            d.pop("M", None)
            an = directional(G[b], effective_direction(p, d, 1e-6))
            fd = fd_directional_corrected(p, sol, d, 1e-6)
            assert abs(fd - an) / max(abs(fd), abs(an)) < 1e-6, (b, fd, an)


def test_cross_term_gradient():
    """Nonzero cross terms M_i: the gradient with respect to M (and every
    other field) against the oracle's adjoint, and central differences along
    directions that include M."""
    _need_gpu()
    from oracle import solve_with_multipliers
    from oracle.gradients import (adjoint_gradients, directional, effective_direction, fd_directional_corrected,
                                  random_direction, sumsq_loss_grad)
    from tests._util import tiny_problem
    # joint stage Hessians [[Q, M], [M', R]] = L L' + 1e-2 I (convex, nonzero M)
    probs = [tiny_problem(4099 + b, N=24, n=6, m=3, kinds=[["mixed"] * 2] * 24, terminal_rows=0, g_mode="random",
                          with_M=True) for b in range(3)]
    rng = np.random.default_rng(4099)
    G = _gpu_grads(probs)
    for b, p in enumerate(probs):
        sol = solve_with_multipliers(p)
        gx, gu = sumsq_loss_grad(sol["x"], sol["u"])
        Go = adjoint_gradients(p, sol, gx, gu)
        for f in FIELDS + ("M", "x0"):
            assert _rel(G[b][f], Go[f]) < 1e-8, (b, f, _rel(G[b][f], Go[f]))
        for _ in range(3):
            d = random_direction(p, rng, ("Q", "q", "R", "r", "M", "A", "B", "c", "E", "F", "g", "x0"))
            an = directional(G[b], effective_direction(p, d, 1e-6))
            fd = fd_directional_corrected(p, sol, d, 1e-6)
            assert abs(fd - an) / max(abs(fd), abs(an)) < 1e-6, (b, fd, an)
