"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerance: relative 2-norm error <= 1e-9 per instance and field over x, u,
lambda (lambda_0 = -alpha) and mu, against the oracle's primal solution and
minimum-norm multipliers, and the same bound stage by stage (each stage's
block error relative to the larger of its own norm and the field's RMS block
norm, so one bad stage is not averaged away).  Small cases are compared in
full; the single instances of the N=1024, N=8192 (n=32) and the paper-shape
N=8192 workloads are compared in full at their full size; the batched
workloads on sampled instances, and every instance through the KKT residual
of Section IX.
"""

from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-9
# Per-stage bound for the 512-instance law's short batches solved with the
# non-default multiplier routes or scan schedules: their multipliers meet
# 1e-9 per instance, and per stage differ from the oracle by up to 2.3e-9 on
# stages of nearly uncontrollable instances (the reversed-time and the
# overlapped theta routes by the same amount there, so the difference comes
# from the shared primal point, not from either multiplier route).
C3_BLOCK_TOL = 1e-8


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_solve(probs, tuning=None, **opts):
    import paper_2407_05433_amd as ecl
    plan = ecl.Plan.for_problems(probs, **opts)
    if tuning:
        ecl.set_tuning(plan, **tuning)
    data = ecl.pack(plan, probs)
    ws = plan.workspace()
    sol = ecl.solve(plan, data, ws)
    torch.cuda.synchronize()
    out = {
        "status": sol.status.cpu().tolist(),
        "x": ecl.unpack(plan, sol.x, "q", probs),
        "u": ecl.unpack(plan, sol.u, "r", probs),
    }
    if sol.lam is not None:
        out["lam"] = ecl.unpack(plan, sol.lam, "q", probs)
        out["mu"] = ecl.unpack(plan, sol.mu, "g", probs)
    out["_plan"], out["_data"], out["_sol"], out["_ws"] = plan, data, sol, ws
    return out


def blockwise_err(a, b):
    """Largest per-stage error max_i ||a_i - b_i|| / max(||b_i||, RMS_j ||b_j||)
    over the blocks of one field (b = reference)."""
    norms = np.array([np.linalg.norm(v) for v in b])
    if norms.size == 0 or not np.any(norms > 0):
        return 0.0 if all(np.array_equal(np.asarray(x), np.asarray(y)) for x, y in zip(a, b)) else np.inf
    rms = float(np.sqrt(np.mean(norms ** 2)))
    return max(float(np.linalg.norm(np.asarray(x) - np.asarray(y))) / max(float(ny), rms)
               for x, y, ny in zip(a, b, norms))


def check_parity(probs, res, idx=None, tol=TOL, oracle_results=None, block_tol=TOL):
    from oracle import solve_with_multipliers
    from tests._util import rel_err
    idx = range(len(probs)) if idx is None else idx
    for b in idx:
        p = probs[b]
        o = oracle_results[b] if oracle_results is not None else solve_with_multipliers(p)
        assert o["status"] == "ok"
        assert res["status"][b] == 0, (b, res["status"][b])
        for key in ("x", "u", "lam", "mu"):
            if key == "mu" and sum(p.nc) == 0:
                continue
            e = rel_err(res[key][b], o[key])
            assert e <= tol, (b, key, e)
            eb = blockwise_err(res[key][b], o[key])
            assert eb <= block_tol, (b, key, "per stage", eb)


def _check_residuals(res, r, tol=1e-8, stat_tol=1e-7):
    """Initial, dynamics and (normalised) equality residuals absolute (tol);
    the stationarity residual relative to the largest multiplier of the
    instance (stat_tol): on nearly uncontrollable instances the multipliers
    reach 1e3..1e5, and on instance 506 of the 512-instance batch the oracle's
    own relative stationarity residual is 1.8e-7."""
    assert r[:, :3].max() < tol, r[:, :3].max(axis=0)
    for b in range(r.shape[0]):
        scale = max(1.0, max(np.abs(v).max(initial=0.0) for v in res["lam"][b]),
                    max(np.abs(v).max(initial=0.0) for v in res["mu"][b]))
        assert r[b, 3] <= stat_tol * scale, (b, r[b, 3], scale)


def test_c0_tiny():
    _need_gpu()
    from workloads import config_c0
    probs = config_c0()
    check_parity(probs, gpu_solve(probs))


def test_reversed_time_multiplier_route():
    """The minimum-norm multipliers through the reversed-time stationarity
    problem (multiplier_route = 0), with and without the overlapped
    factorization, on the small case, the structural family and a batch."""
    _need_gpu()
    from tests._util import problem_family
    from workloads import config_c0, config_c3
    fam = [p for _, p in problem_family()]
    for tun in ({"multiplier_route": 0, "overlap_dual": 1}, {"multiplier_route": 0, "overlap_dual": 0}):
        probs = config_c0()
        res = gpu_solve(probs, tuning=tun, reversed_time=1)
        assert ecl_tuning(res)["multiplier_route"] == 0
        check_parity(probs, res)
        check_parity(fam, gpu_solve(fam, tuning=tun, reversed_time=1))
    probs = config_c3(B=8, N_range=(32, 90))
    check_parity(probs, gpu_solve(probs, tuning={"multiplier_route": 0}, reversed_time=1), block_tol=C3_BLOCK_TOL)


def ecl_tuning(res):
    import paper_2407_05433_amd as ecl
    return ecl.get_tuning(res["_plan"])


def test_both_scan_schedules():
    """Small problems default to recursive doubling; the balanced up/down
    sweep (scan_schedule = 1) on the same cases, and doubling forced on a
    batch that would default to the balanced sweep."""
    _need_gpu()
    from tests._util import problem_family
    from workloads import config_c0, config_c3
    fam = [p for _, p in problem_family()]
    probs = config_c0()
    check_parity(probs, gpu_solve(probs, scan_schedule=1))
    check_parity(fam, gpu_solve(fam, scan_schedule=1))
    probs = config_c3(B=12, N_range=(150, 250))
    check_parity(probs, gpu_solve(probs, scan_schedule=2), idx=range(0, 12, 3), block_tol=C3_BLOCK_TOL)


def test_structural_family_single_and_batched():
    _need_gpu()
    from tests._util import problem_family
    fam = [p for _, p in problem_family()]
    for p in fam:
        check_parity([p], gpu_solve([p]))
    check_parity(fam, gpu_solve(fam))


def test_singular_state_costs():
    """Q = 0 (value functions identically zero: the value-function combine
    takes its LU form) and a rank-one Q (positive semidefinite value
    functions), single and batched with a regular instance."""
    _need_gpu()
    from tests._util import tiny_problem
    zero = tiny_problem(700, N=9, n=4, m=2, terminal_rows=1)
    for i in range(zero.N + 1):
        zero.Q[i] = np.zeros_like(zero.Q[i])
    rank1 = tiny_problem(701, N=9, n=4, m=2, terminal_rows=1)
    for i in range(rank1.N + 1):
        v = np.ones((4, 1)) / 2.0
        rank1.Q[i] = v @ v.T
    regular = tiny_problem(702, N=9, n=4, m=2, terminal_rows=1)
    probs = [zero, rank1, regular]
    for p in probs:
        check_parity([p], gpu_solve([p]))
    check_parity(probs, gpu_solve(probs))


def test_combine_modes_same_bits():
    """Every LDS mode of the value-function combine (work pool in global
    scratch, pool in LDS, everything in LDS, staged operands with a compact
    pool; one or two wavefronts per combine) gives the same bits, on batches
    whose combines take the factored form and the LU form (Q = 0)."""
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from tests._util import tiny_problem
    from workloads import config_c3
    zero = tiny_problem(710, N=9, n=4, m=2, terminal_rows=1)
    for i in range(zero.N + 1):
        zero.Q[i] = np.zeros_like(zero.Q[i])
    probs = config_c3(B=6, N_range=(32, 70)) + [zero, tiny_problem(711, N=11, n=5, m=3, terminal_rows=1)]
    plan = ecl.Plan.for_problems(probs)
    data = ecl.pack(plan, probs)
    ws = plan.workspace()
    base = {k: v for k, v in ecl.get_tuning(plan).items() if k != "ms_per_solve"}
    ref = None
    for pool in (1, 0, 2, 3):
        for split in (0, 1):
            ecl.set_tuning(plan, **dict(base, pool_in_lds=pool, split_combine=split))
            sol = ecl.solve(plan, data, ws)
            torch.cuda.synchronize()
            got = {f: getattr(sol, f).clone() for f in ("x", "u", "lam", "mu", "status")}
            print(f"[modes] pool {pool} split {split}: status {got['status'].tolist()}", flush=True)
            if ref is None:
                ref = got
                assert int(got["status"].abs().sum()) == 0
                check_parity(probs, {"x": ecl.unpack(plan, sol.x, "q", probs), "u": ecl.unpack(plan, sol.u, "r", probs),
                                     "lam": ecl.unpack(plan, sol.lam, "q", probs),
                                     "mu": ecl.unpack(plan, sol.mu, "g", probs), "status": got["status"].tolist()})
            for f in got:
                assert torch.equal(got[f], ref[f]), (pool, split, f)


def test_buckets_same_bits():
    """A batch of more than 4096 stages launches its LDS-bound stage kernels
    per stage bucket (stages in size order, LDS sized to each range) and its
    wide scan levels per dim or size bucket; with buckets off every kernel
    runs one launch over its whole range.  Both give the same bits, and agree
    with the oracle on sampled instances."""
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from workloads import config_c3
    probs = config_c3(B=24)
    assert sum(p.N + 1 for p in probs) > 4096
    plan = ecl.Plan.for_problems(probs)
    data = ecl.pack(plan, probs)
    ws = plan.workspace()
    base = {k: v for k, v in ecl.get_tuning(plan).items() if k != "ms_per_solve"}
    out = []
    for buckets in (1, 0):
        ecl.set_tuning(plan, **dict(base, level_buckets=buckets))
        sol = ecl.solve(plan, data, ws)
        torch.cuda.synchronize()
        out.append({f: getattr(sol, f).clone() for f in ("x", "u", "lam", "mu", "status")})
        print(f"[buckets] {buckets}: status {int((sol.status != 0).sum())} nonzero", flush=True)
    for f in out[0]:
        assert torch.equal(out[0][f], out[1][f]), f
    res = {"status": out[0]["status"].cpu().tolist(), "x": ecl.unpack(plan, out[0]["x"], "q", probs),
           "u": ecl.unpack(plan, out[0]["u"], "r", probs), "lam": ecl.unpack(plan, out[0]["lam"], "q", probs),
           "mu": ecl.unpack(plan, out[0]["mu"], "g", probs)}
    check_parity(probs, res, idx=[0, 7, 15, 23])


def test_c1_full_size():
    _need_gpu()
    from workloads import config_c1
    probs = config_c1()
    check_parity(probs, gpu_solve(probs))


def test_c2_law_short_horizon():
    _need_gpu()
    from workloads import config_c2
    probs = config_c2(N=512)
    check_parity(probs, gpu_solve(probs))


def test_c3_batched_sample_and_residuals():
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from workloads import config_c3
    probs = config_c3(B=64)
    res = gpu_solve(probs)
    # every 4th instance, plus 47: a nearly uncontrollable reduced system whose
    # value-function scan needs more than one refinement step
    check_parity(probs, res, idx=list(range(0, 64, 4)) + [47])
    steps = res["_plan"].refine_steps(res["_ws"])
    assert steps.min() >= 0 and steps.max() <= 3 and steps[47] >= 1, steps
    r = ecl.kkt_residual(res["_plan"], res["_data"], res["_sol"], res["_ws"]).cpu().numpy()
    torch.cuda.synchronize()
    assert np.all(np.array(res["status"]) == 0)
    _check_residuals(res, r)


def test_c3_full_batch_sampled():
    """The full 512-instance batch in the configuration bench.py times:
    sampled instances against the oracle, every instance through the KKT
    residual."""
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from workloads import config_c3
    probs = config_c3()
    res = bench_config_solve(probs)
    assert np.all(np.array(res["status"]) == 0), np.nonzero(res["status"])
    check_parity(probs, res, idx=range(3, 512, 37))
    r = ecl.kkt_residual(res["_plan"], res["_data"], res["_sol"], res["_ws"]).cpu().numpy()
    _check_residuals(res, r)


def test_refinement_options():
    """refine = 0 (multipliers at the first primal point) and a single
    forced step both stay within tolerance on a well-conditioned instance;
    accept_tol = 0 and refine_tol = 0 force every instance through the
    maximum step count."""
    _need_gpu()
    from workloads import config_c0, config_c3
    probs = config_c0()
    check_parity(probs, gpu_solve(probs, refine=0))
    check_parity(probs, gpu_solve(probs, refine=1))
    probs = config_c3(B=4, N_range=(32, 64))
    res = gpu_solve(probs, refine=2, refine_tol=0.0, accept_tol=0.0)
    assert np.all(res["_plan"].refine_steps(res["_ws"]) == 2)
    check_parity(probs, res)


def test_batched_equals_single():
    _need_gpu()
    from workloads import config_c3
    probs = config_c3(B=6, N_range=(32, 80))
    batch = gpu_solve(probs)
    for b, p in enumerate(probs):
        single = gpu_solve([p])
        for key in ("x", "u", "lam", "mu"):
            a = np.concatenate([v.ravel() for v in batch[key][b]])
            s = np.concatenate([v.ravel() for v in single[key][0]])
            assert np.array_equal(a, s), (b, key)


def test_c4_forward_sample():
    _need_gpu()
    from workloads import config_c4
    probs = config_c4(B=32)
    res = gpu_solve(probs)
    check_parity(probs, res, idx=range(0, 32, 4))


def test_varying_dims_and_edges():
    _need_gpu()
    from tests._util import tiny_problem
    probs = [
        tiny_problem(1100, nx=[1, 3, 5, 2, 4, 1], nu=[1, 2, 1, 3, 1], terminal_rows=1),
        tiny_problem(1101, nx=[6, 2, 6, 2, 6], nu=[1, 5, 1, 5], terminal_rows=0),
        tiny_problem(1102, N=1, n=1, m=1, kinds=[[]], terminal_rows=0),
        tiny_problem(1103, N=2, n=5, m=5, kinds=[["mixed"] * 4, ["state"] * 3], terminal_rows=2),
    ]
    check_parity(probs, gpu_solve(probs))


def test_infeasibility_outcomes():
    _need_gpu()
    from tests._util import tiny_problem
    bad_suffix = tiny_problem(400, N=4, n=3, m=1, kinds=[[], [], [], ["state", "state", "state"]], terminal_rows=3)
    bad_suffix.g[bad_suffix.N] = bad_suffix.g[bad_suffix.N] + 1.0
    bad_init = tiny_problem(401, N=4, n=3, m=2, kinds=[["state"], [], [], []], terminal_rows=0)
    bad_init.g[0] = bad_init.g[0] + 1.0
    nonconvex = tiny_problem(402, N=3, n=2, m=2, kinds=[[]] * 3, terminal_rows=0)
    nonconvex.R[1] = -nonconvex.R[1]
    nan_in = tiny_problem(403, N=3, n=2, m=2, kinds=[[]] * 3, terminal_rows=0)
    nan_in.q[1] = nan_in.q[1].copy()
    nan_in.q[1][0] = np.nan
    good = tiny_problem(404, N=3, n=2, m=2, kinds=[[]] * 3, terminal_rows=0)
    res = gpu_solve([bad_suffix, bad_init, nonconvex, nan_in, good])
    st = res["status"]
    assert st[0] & 1, st
    assert st[1] & 2, st
    assert st[2] & 8, st
    assert st[3] & 16, st
    assert st[4] == 0, st
    assert np.all(np.isnan(np.concatenate(res["x"][0]))) and np.all(np.isfinite(np.concatenate(res["x"][4])))
    check_parity([good], {k: [v[4]] for k, v in res.items() if not k.startswith("_") and k != "status"} |
                 {"status": [0]})


def test_deterministic_bitwise():
    _need_gpu()
    from workloads import config_c1
    probs = config_c1(N=256)
    a = gpu_solve(probs)
    b = gpu_solve(probs)
    for key in ("x", "u", "lam", "mu"):
        assert np.array_equal(np.concatenate(a[key][0]), np.concatenate(b[key][0]))


def test_graph_replay_matches_eager():
    """use_graph: the captured launch sequence, replayed several times with
    eager work in between, reproduces the eager solve bitwise; new values in
    the same buffers are picked up; new buffers re-capture."""
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from workloads import config_c1, config_c3
    for probs in (config_c1(N=200), config_c3(B=5, N_range=(32, 70))):
        eager = ecl.Plan.for_problems(probs)
        graph = ecl.Plan.for_problems(probs, use_graph=1)
        data = ecl.pack(eager, probs)
        ws_e, ws_g = eager.workspace(), graph.workspace()
        ref = ecl.solve(eager, data, ws_e)
        sol = ecl.allocate_solution(graph)
        for rep in range(3):
            ecl.solve(graph, data, ws_g, sol)
            torch.cuda.synchronize()
            for f in ("x", "u", "lam", "mu", "status"):
                assert torch.equal(getattr(sol, f), getattr(ref, f)), (rep, f)
            # eager work between replays
            ecl.solve(eager, data, ws_e, ecl.allocate_solution(eager))
            (data["q"] * 2.0).sum().item()
            torch.cuda.synchronize()
        # new values in the same buffers (linear costs: feasibility unchanged)
        data["q"].mul_(-0.5)
        data["r"].add_(0.25)
        ref2 = ecl.solve(eager, data, ws_e)
        ecl.solve(graph, data, ws_g, sol)
        torch.cuda.synchronize()
        assert int(ref2.status.abs().sum()) == 0
        for f in ("x", "u", "lam", "mu", "status"):
            assert torch.equal(getattr(sol, f), getattr(ref2, f)), ("new values", f)
        # new output buffers: re-capture
        sol2 = ecl.allocate_solution(graph)
        ecl.solve(graph, data, ws_g, sol2)
        torch.cuda.synchronize()
        for f in ("x", "u", "lam", "mu", "status"):
            assert torch.equal(getattr(sol2, f), getattr(ref2, f)), ("new buffers", f)


def test_refine_gate_same_results():
    """refine_gate: the host reads back how many instances still refine after
    the first pass and enqueues the refinement steps only when some does.
    Eager and graph forms (graph replayed with eager work in between) give
    the ungated solve's bits, refinement counts and backward errors, on a
    single instance that takes no step and on batches where some instances
    refine (the steps are then launched)."""
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from workloads import config_c1, config_c2, config_c3
    cases = (("c1 N=200", config_c1(N=200)), ("c3 B=6", config_c3(B=6, N_range=(32, 70))),
             ("c2 N=512", config_c2(N=512)))
    took_step = False
    for name, probs in cases:
        ref_plan = ecl.Plan.for_problems(probs)
        data = ecl.pack(ref_plan, probs)
        ws_r = ref_plan.workspace()
        ref = ecl.solve(ref_plan, data, ws_r)
        torch.cuda.synchronize()
        ref_steps, ref_omega = ref_plan.refine_steps(ws_r), ref_plan.backward_error(ws_r)
        took_step |= bool((ref_steps > 0).any())
        for graph in (0, 1):
            plan = ecl.Plan.for_problems(probs, use_graph=graph)
            ecl.set_tuning(plan, refine_gate=1)
            assert ecl.get_tuning(plan)["refine_gate"] == 1
            ws = plan.workspace()
            sol = ecl.allocate_solution(plan)
            for rep in range(3):
                ecl.solve(plan, data, ws, sol)
                torch.cuda.synchronize()
                for f in ("x", "u", "lam", "mu", "status"):
                    assert torch.equal(getattr(sol, f), getattr(ref, f)), (name, graph, rep, f)
                assert np.array_equal(plan.refine_steps(ws), ref_steps), (name, graph, rep)
                assert np.array_equal(plan.backward_error(ws), ref_omega), (name, graph, rep)
                ecl.solve(ref_plan, data, ws_r, ecl.allocate_solution(ref_plan))
                torch.cuda.synchronize()
    assert took_step, "no case took a refinement step"
    # the other multiplier routes and the overlapped factorizations, gated
    probs = config_c3(B=6, N_range=(32, 70))
    variants = (({}, {"overlap_dual": 1}), ({"reversed_time": 1}, {"multiplier_route": 0, "overlap_dual": 1}),
                ({"reversed_time": 1}, {"multiplier_route": 0, "overlap_dual": 0}), ({"multipliers": 2}, {}),
                ({"multipliers": 3}, {}))
    for opts, tun in variants:
        ref_plan = ecl.Plan.for_problems(probs, **opts)
        ecl.set_tuning(ref_plan, **tun)
        data = ecl.pack(ref_plan, probs)
        ws_r = ref_plan.workspace()
        ref = ecl.solve(ref_plan, data, ws_r)
        torch.cuda.synchronize()
        for graph in (0, 1):
            plan = ecl.Plan.for_problems(probs, use_graph=graph, **opts)
            ecl.set_tuning(plan, refine_gate=1, **tun)
            ws = plan.workspace()
            sol = ecl.allocate_solution(plan)
            for rep in range(2):
                ecl.solve(plan, data, ws, sol)
                torch.cuda.synchronize()
                for f in ("x", "u", "lam", "mu", "status"):
                    assert torch.equal(getattr(sol, f), getattr(ref, f)), (opts, tun, graph, rep, f)
                assert np.array_equal(plan.refine_steps(ws), ref_plan.refine_steps(ws_r)), (opts, tun, graph)


def test_autotune_keeps_results():
    """eclqr_plan_autotune picks a launch configuration by timing; every
    configuration it can choose computes the same solution (bitwise)."""
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from workloads import config_c3
    probs = config_c3(B=8, N_range=(32, 90))
    plan = ecl.Plan.for_problems(probs, reversed_time=1)
    data = ecl.pack(plan, probs)
    ws = plan.workspace()
    ref = ecl.solve(plan, data, ws)
    torch.cuda.synchronize()
    ref = {f: getattr(ref, f).clone() for f in ("x", "u", "lam", "mu", "status")}
    base = ecl.get_tuning(plan)
    tuned = ecl.autotune(plan, data, ws)
    assert tuned["ms_per_solve"] > 0
    for cfg in ({"level_buckets": 0}, {"pool_in_lds": 0}, {"pool_in_lds": 1}, {"pool_in_lds": 2}, {"pool_in_lds": 3},
                {"stage_lds": 0}, {"stage_lds": 2}, {"grid_divisor": 4},
                {"overlap_dual": 1 - base["overlap_dual"]}, {"multiplier_route": 1 - base["multiplier_route"]},
                {"multiplier_route": 1 - base["multiplier_route"], "overlap_dual": 1 - base["overlap_dual"]},
                {"split_combine": 0}, {"fused_scans": 0},
                {"use_graph": 1},
                {"register_compose": 0}, tuned):
        full = dict(base)
        full.update(cfg)
        ecl.set_tuning(plan, **{k: v for k, v in full.items() if k != "ms_per_solve"})
        sol = ecl.solve(plan, data, ws)
        torch.cuda.synchronize()
        for f in ("x", "u", "lam", "mu", "status"):
            same = all(full[k] == base[k] for k in ("register_compose", "overlap_dual", "multiplier_route"))
            if same:
                assert torch.equal(getattr(sol, f), ref[f]), (cfg, f)
            else:
                # the LDS and register compositions differ in rounding only,
                # and so do the multiplier routes and their full and
                # factor-then-replay passes (overlap_dual)
                a, b = getattr(sol, f).double(), ref[f].double()
                err = float((a - b).norm() / max(float(b.norm()), 1e-300))
                assert err <= 1e-8, (cfg, f, err)


def test_domain_shortcut():
    """The domain shortcut of Section VI: instances with no terminal rows whose
    every F_i has full row rank skip the relation scan (every relation slot of
    theirs is left empty); the other instances of the same batch (a state-only
    row, a terminal row, more mixed rows than inputs, a redundant row) run it.
    With the shortcut on and off: oracle parity, and the two agree."""
    _need_gpu()
    from tests._util import rel_err, tiny_problem
    from workloads import config_c4
    probs = config_c4(B=3, N=24) + [
        tiny_problem(1201, N=6, n=4, m=3, kinds=[["mixed", "state"]] * 6, terminal_rows=0),
        tiny_problem(1202, N=6, n=4, m=3, kinds=[["mixed"]] * 6, terminal_rows=1),
        tiny_problem(1203, N=5, n=3, m=2, kinds=[["mixed"] * 3] + [["mixed"]] * 4, terminal_rows=0),
        tiny_problem(1204, N=7, n=3, m=2, kinds=[[]] * 7, terminal_rows=0),
        tiny_problem(1205, N=6, n=4, m=3, kinds=[["mixed", "mixed"]] * 6, terminal_rows=0, redundant=(2,)),
        tiny_problem(1206, N=6, n=4, m=3, kinds=[["mixed", "mixed"]] * 6, terminal_rows=0),
    ]
    vacuous = [True, True, True, False, False, False, True, False, True]
    res = {}
    for sc in (1, 0):
        r = gpu_solve(probs, domain_shortcut=sc)
        check_parity(probs, r)
        plan = r["_plan"]
        rows = plan.scan_rows(r["_ws"])
        inst = plan.slot_info()[0]
        for b, v in enumerate(vacuous):
            sel = inst == b
            if sc and v:
                assert np.all(rows[sel] == 0), (b, rows[sel])
            else:
                assert np.any(rows[sel] > 0), (sc, b)
        res[sc] = r
    for b in range(len(probs)):
        for key in ("x", "u", "lam", "mu"):
            assert rel_err(res[1][key][b], res[0][key][b]) <= 1e-11, (b, key)


def test_theta_route_overlapped_factorization():
    """The theta LQR factored on the second stream once the domains are known
    (matrix pass, then a vector pass at the primal solution): oracle parity on
    the small case, the structural family and a batch; graph replays equal
    the eager solve."""
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from tests._util import problem_family
    from workloads import config_c0, config_c3
    tun = {"overlap_dual": 1, "multiplier_route": 1}
    probs = config_c0()
    res = gpu_solve(probs, tuning=tun)
    assert ecl_tuning(res)["overlap_dual"] == 1
    check_parity(probs, res)
    fam = [p for _, p in problem_family()]
    check_parity(fam, gpu_solve(fam, tuning=tun))
    probs = config_c3(B=8, N_range=(32, 90))
    check_parity(probs, gpu_solve(probs, tuning=tun), block_tol=C3_BLOCK_TOL)
    eager = ecl.Plan.for_problems(probs)
    graph = ecl.Plan.for_problems(probs, use_graph=1)
    for pl in (eager, graph):
        ecl.set_tuning(pl, **tun)
    data = ecl.pack(eager, probs)
    ref = ecl.solve(eager, data, eager.workspace())
    ws_g = graph.workspace()
    sol = ecl.allocate_solution(graph)
    for rep in range(3):
        ecl.solve(graph, data, ws_g, sol)
        torch.cuda.synchronize()
        for f in ("x", "u", "lam", "mu", "status"):
            assert torch.equal(getattr(sol, f), getattr(ref, f)), (rep, f)
        (data["q"] * 2.0).sum().item()
        torch.cuda.synchronize()


def test_indefinite_costs_with_convex_reduction():
    """Convexity is needed only on the feasible set: R_i or Q_i indefinite
    along directions the constraints fix reduce to a strictly convex problem
    and match the oracle (both multiplier routes); a negative direction left
    free is reported as not convex (status bit 8) without touching the other
    instances of the batch."""
    _need_gpu()
    from tests._util import indefinite_cost_problems
    p1, p2, p3 = indefinite_cost_problems()
    check_parity([p1, p2], gpu_solve([p1, p2]))
    check_parity([p1, p2], gpu_solve([p1, p2], tuning={"multiplier_route": 0}, reversed_time=1))
    res = gpu_solve([p1, p3, p2])
    assert res["status"][1] & 8, res["status"]
    check_parity([p1, p2], {k: [v[0], v[2]] for k, v in res.items() if not k.startswith("_")})


def bench_config_solve(probs):
    """A solve in the launch configuration bench.py times: hipGraph replay of
    an autotuned plan (the replay after the capturing solve is returned)."""
    import paper_2407_05433_amd as ecl
    plan = ecl.Plan.for_problems(probs, use_graph=1)
    data = ecl.pack(plan, probs)
    ws = plan.workspace()
    ecl.autotune(plan, data, ws)
    sol = ecl.allocate_solution(plan)
    for _ in range(2):
        ecl.solve(plan, data, ws, sol)
    torch.cuda.synchronize()
    return {
        "status": sol.status.cpu().tolist(),
        "x": ecl.unpack(plan, sol.x, "q", probs), "u": ecl.unpack(plan, sol.u, "r", probs),
        "lam": ecl.unpack(plan, sol.lam, "q", probs), "mu": ecl.unpack(plan, sol.mu, "g", probs),
        "_plan": plan, "_data": data, "_sol": sol, "_ws": ws,
    }


@pytest.mark.parametrize("workload", ["c1", "c2", "c4", "paper"])
def test_full_size_bench_configuration(workload):
    """The full-size workloads in the launch configuration bench.py times
    (autotuned plan, graph replay): every instance through the oracle's KKT
    residual computed on the host from the returned x, u, lambda, mu (initial
    condition, dynamics and normalised equality rows absolute, stationarity
    relative to the largest multiplier); the single instances (N=1024; N=8192
    with n=32; the paper shape at N=8192) against the oracle's solution in
    full, and sampled instances of the batch."""
    _need_gpu()
    from oracle.residual import kkt_residual
    from workloads import config_c1, config_c2, config_c4, config_paper
    probs = {"c1": config_c1, "c2": config_c2, "c4": config_c4, "paper": lambda: config_paper(8192)}[workload]()
    res = bench_config_solve(probs)
    assert np.all(np.array(res["status"]) == 0), np.nonzero(res["status"])
    for b, p in enumerate(probs):
        r = kkt_residual(p, res["x"][b], res["u"][b], res["lam"][b], res["mu"][b])
        scale = max(1.0, max(np.abs(v).max(initial=0.0) for v in res["lam"][b]),
                    max(np.abs(v).max(initial=0.0) for v in res["mu"][b]))
        assert max(r["initial"], r["dynamics"], r["equality"]) < 1e-8, (b, r)
        assert r["stationarity"] <= 1e-7 * scale, (b, r, scale)
    if workload == "c4":
        check_parity(probs, res, idx=range(5, 256, 50))
    else:  # single instances: compared in full at their full size
        check_parity(probs, res)


def test_maximum_dims():
    """Stage dims at the kernels' limit (64): state dim 64 with few inputs,
    input dim 64, and both (the last through the reversed-time multiplier
    route: k_i + n_{i+1} > 64).  Stacked relation systems beyond the device's
    LDS run in the plan's global tiles, so every instance is solved (oracle
    parity), alone and in a batch.  The check also accepts the outcome of a
    relation beyond every tile (ECLQR_CAPACITY, bit 32, possibly with bits
    that follow from the truncated relation, or ECLQR_DUAL_FAILED with the
    capacity bit in bits 8..15 for the reversed-time problem; the outputs are
    then NaN, as the ABI states), so the same check serves plans without
    tiles."""
    _need_gpu()
    from tests._util import tiny_problem
    probs = [
        tiny_problem(1472, N=3, n=64, m=8, kinds=[["mixed", "state", "mixed", "state"]] * 3, terminal_rows=2),
        tiny_problem(1480, N=3, n=16, m=64, kinds=[["mixed"] * 8] * 3, terminal_rows=1),
        tiny_problem(1528, N=2, n=64, m=64, kinds=[["mixed"] * 6 + ["state"] * 2] * 2, terminal_rows=3),
        tiny_problem(1529, N=6, n=4, m=2, terminal_rows=1),
    ]

    def check(res, b, p, i):
        st = res["status"][i]
        if st == 0:
            check_parity([p], {k: [v[i]] for k, v in res.items() if not k.startswith("_")})
        else:
            assert (st & 32) or (st & 64 and (st >> 8) & 32), (b, st)
            for key in ("x", "u", "lam", "mu"):
                assert np.all(np.isnan(np.concatenate([v.ravel() for v in res[key][i]]))), (b, key)
        return st

    outcomes = [check(gpu_solve([p]), b, p, 0) for b, p in enumerate(probs)]
    assert outcomes == [0, 0, 0, 0], outcomes
    res = gpu_solve(probs)
    assert [check(res, b, p, b) for b, p in enumerate(probs)] == outcomes


@pytest.mark.skip(reason="the persistent scan kernels (fused_scans = 1) did not finish on the MI355X: the run "
                         "went silent in the autotune test while they replayed refinement steps; the cause is not "
                         "established (the dependency order is checked on the CPU in test_scan_schedule.py), so "
                         "the path is off by default and stays off the GPU")
def test_persistent_scans_equal_per_level_launches():
    """Refinement steps forced on every instance (accept_tol = 0): the
    vector-only replays with one persistent launch per scan give the same
    bits as one launch per level, on a batch of the 512-instance law and on
    the N=1024 instance, eager and as a replayed graph; no instance reports
    an expired wait (bit 65536)."""
    _need_gpu()
    import paper_2407_05433_amd as ecl
    from workloads import config_c1, config_c3
    for probs in (config_c3(B=16, N_range=(32, 200)), config_c1(N=1024)):
        ref = None
        for fused, graph in ((0, 0), (1, 0), (1, 1)):
            plan = ecl.Plan.for_problems(probs, accept_tol=0.0, use_graph=graph)
            ecl.set_tuning(plan, fused_scans=fused)
            data = ecl.pack(plan, probs)
            ws = plan.workspace()
            sol = ecl.allocate_solution(plan)
            for _ in range(2 if graph else 1):
                ecl.solve(plan, data, ws, sol)
            torch.cuda.synchronize()
            assert int(sol.status.abs().sum()) == 0, sol.status
            assert plan.refine_steps(ws).min() >= 1
            got = {f: getattr(sol, f).clone() for f in ("x", "u", "lam", "mu")}
            if ref is None:
                ref = got
                check_parity(probs, {"status": sol.status.cpu().tolist(),
                                     "x": ecl.unpack(plan, sol.x, "q", probs), "u": ecl.unpack(plan, sol.u, "r", probs),
                                     "lam": ecl.unpack(plan, sol.lam, "q", probs),
                                     "mu": ecl.unpack(plan, sol.mu, "g", probs)},
                             idx=range(0, len(probs), 5), block_tol=C3_BLOCK_TOL)
            else:
                for f in got:
                    assert torch.equal(got[f], ref[f]), (fused, graph, f)
