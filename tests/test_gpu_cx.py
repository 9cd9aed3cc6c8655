"""The contraction-expansion multiplier route of Section VII on the GPU
(multipliers = 3), through the C ABI, against the oracle's restatement of
the same procedure (same balanced tree, minimum-norm choices at the root, in
the expansion and at the leaves): x, u at 1e-9, lambda and mu at 1e-8
relative, the stationarity residual at rounding level, and the minimum-norm
multipliers at 1e-9 where the constraint rows are independent (there the
multipliers are unique)."""

from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _cases():
    from tests._util import problem_family, tiny_problem
    from workloads import config_c1, config_c3, config_c4
    out = [p for _, p in problem_family()]
    out += [config_c1(N=40)[0], config_c4(B=1, N=20)[0],
            tiny_problem(1601, N=5, n=3, m=2, kinds=[["mixed"]] * 5, terminal_rows=0, redundant=(2,)),
            tiny_problem(1602, N=4, n=3, m=2, kinds=[["state"], [], ["mixed"], []], terminal_rows=0)]
    out += config_c3(B=6, N_range=(32, 90))
    return out


def test_contraction_expansion_route_matches_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_05433_amd as ecl
    from oracle import rows_independent, solve_sequential, solve_with_multipliers
    from oracle.contraction import contraction_expansion
    from oracle.residual import kkt_residual
    from tests._util import rel_err
    probs = _cases()
    for batch in (probs, [probs[0]], [probs[-1]]):
        plan = ecl.Plan.for_problems(batch, multipliers=3)
        data = ecl.pack(plan, batch)
        ws = plan.workspace()
        sol = ecl.solve(plan, data, ws)
        torch.cuda.synchronize()
        st = sol.status.cpu().tolist()
        xs, us = ecl.unpack(plan, sol.x, "q", batch), ecl.unpack(plan, sol.u, "r", batch)
        ls, ms = ecl.unpack(plan, sol.lam, "q", batch), ecl.unpack(plan, sol.mu, "g", batch)
        for b, p in enumerate(batch):
            assert st[b] == 0, (b, st[b])
            o = solve_with_multipliers(p)
            assert rel_err(xs[b], o["x"]) <= 1e-9 and rel_err(us[b], o["u"]) <= 1e-9, b
            cx = contraction_expansion(p, o["x"], o["u"])
            assert rel_err(ls[b], cx["lam"]) <= 1e-8, (b, rel_err(ls[b], cx["lam"]))
            if sum(p.nc):
                assert rel_err(ms[b], cx["mu"]) <= 1e-8, (b, rel_err(ms[b], cx["mu"]))
            r = kkt_residual(p, xs[b], us[b], ls[b], ms[b])
            scale = max(1.0, max(np.abs(v).max(initial=0.0) for v in ls[b]),
                        max(np.abs(v).max(initial=0.0) for v in ms[b]))
            assert r["stationarity"] <= 1e-9 * scale, (b, r)
            if rows_independent(p, solve_sequential(p)):
                assert rel_err(ls[b], o["lam"]) <= 1e-9, b
                if sum(p.nc):
                    assert rel_err(ms[b], o["mu"]) <= 1e-9, b
