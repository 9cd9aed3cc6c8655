"""eclqr_solve_noalloc (the workspace in the library's static per-GPU array)
against eclqr_solve (caller workspace), through the C ABI: two calls in a
row, the second on a smaller problem of another plan, each compared with the
regular entry point's solution to the parity bar (relative 1e-9 per field;
outcome bits and failing stages equal).  Plans whose workspace exceeds the
array are refused with ECLQR_WORKSPACE_TOO_SMALL."""

from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_noalloc_matches_solve_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_05433_amd as ecl
    from workloads import config_c0, config_c1, config_c4
    cases = [config_c1(N=128), config_c0()]
    outs = []
    for probs in cases:
        plan = ecl.Plan.for_problems(probs)
        assert plan.workspace_bytes <= 64 << 20
        data = ecl.pack(plan, probs)
        ref = ecl.solve(plan, data, plan.workspace())
        torch.cuda.synchronize()
        got = ecl.allocate_solution(plan)
        for f in ("x", "u", "lam", "mu"):
            getattr(got, f).fill_(np.nan)
        ecl.solve_noalloc(plan, data, got)
        torch.cuda.synchronize()
        outs.append((plan, data, ref, got))
    for plan, data, ref, got in outs:
        assert torch.equal(got.status, ref.status) and int(ref.status.abs().sum()) == 0
        assert torch.equal(got.info, ref.info)
        for f in ("x", "u", "lam", "mu"):
            assert _rel(getattr(got, f), getattr(ref, f)) <= 1e-9, f
    # back to the first (larger) plan after the second used the array
    plan, data, ref, _ = outs[0]
    again = ecl.allocate_solution(plan)
    ecl.solve_noalloc(plan, data, again)
    torch.cuda.synchronize()
    for f in ("x", "u", "lam", "mu"):
        assert _rel(getattr(again, f), getattr(ref, f)) <= 1e-9, f
    big = config_c4(B=16, N=64)
    bplan = ecl.Plan.for_problems(big)
    assert bplan.workspace_bytes > 64 << 20
    with pytest.raises(ecl.EclqrError, match="status 2"):
        ecl.solve_noalloc(bplan, ecl.pack(bplan, big), ecl.allocate_solution(bplan))
