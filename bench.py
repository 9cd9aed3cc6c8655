"""Benchmark: stages/s of the full solve (primal + multipliers) on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c1|c2|c3|c4|paper]

A step is one solve of the whole hot path (feasible-domain scan, stage
elimination, reduced-LQR scan, recovery, multipliers, and iterative
refinement that each instance stops once its correction is below 1e-8 of its
solution, at most 3 steps) of one batch of synthetic instances already resident in HBM.  Prints one JSON
line; the per-kernel breakdown and the secondary workloads go to stderr and to
the "secondary" object.
"""

from __future__ import annotations

import os

# the CPU baseline (the oracle) runs on one core
for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse  # noqa: E402
import json  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CUs x 128 FP64 flop/clk x 2.4 GHz
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c0": "tiny: 1 instance, N=16, n=4, m=2, 1 mixed row/stage, 2 terminal rows",
    "c1": "single: 1 instance, N=1024, n=12, m=6, k_i in {0..4} (state/mixed, 10% redundant), 3 terminal rows",
    "c2": "dae: 1 instance, N=8192, n=32, m=16, 6 algebraic rows/stage + 4 state rows every 8th stage",
    "c3": "batched: 512 instances, N in [32,512], n in [6,24], m in [3,12], k_i in [0,m-1]",
    "c4": "differentiable: 256 instances, N=128, n=16, m=8, 3 mixed rows/stage",
    "paper": "paper Table I shape: 1 instance, N=8192, n=8, m=4, 2 state rows/stage",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make(workload):
    from workloads import make_config
    if workload == "paper":
        return make_config("paper", N=8192)
    return make_config(workload)


def scan_schedule_name(plan):
    """The scan parenthesization a plan runs: the option, with the default
    hybrid named "doubling" where it reduces to pure doubling (no down-sweep)."""
    opt = int(plan.options.scan_schedule)
    if opt == 1:
        return "balanced"
    sched = plan.schedule()
    if opt == 2 or all(len(lv) == 0 for lv in sched[len(sched) // 2:]):
        return "doubling"
    return "hybrid"


def time_solves(ecl, torch, plan, data, ws, sol, steps, warmup):
    for _ in range(warmup):
        ecl.solve(plan, data, ws, sol)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        ecl.solve(plan, data, ws, sol)
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, e0.elapsed_time(e1) / steps


def kernel_profile(ecl, torch, plan, data, ws, sol, steps):
    plan.set_profiling(True)
    plan.profile(reset=True)
    for _ in range(steps):
        ecl.solve(plan, data, ws, sol)
    torch.cuda.synchronize()
    prof = plan.profile(reset=True)
    plan.set_profiling(False)
    return {k: (ms / steps, n / steps) for k, (ms, n) in prof.items()}


def secondary_batched(ecl, torch, steps):
    """The 512-instance batch solved in one call versus the same instances
    solved one after another, each with its own single-instance plan."""
    problems = make("c3")
    stages = sum(p.N for p in problems)
    plan = ecl.Plan.for_problems(problems)
    data = ecl.pack(plan, problems)
    ws = plan.workspace()
    sol = ecl.allocate_solution(plan)
    batched_ms, _ = time_solves(ecl, torch, plan, data, ws, sol, steps, 1)
    ok_batched = int((sol.status != 0).sum().item()) == 0
    del ws
    singles = []
    for p in problems:
        pl = ecl.Plan.for_problems([p])
        singles.append((pl, ecl.pack(pl, [p]), pl.workspace(), ecl.allocate_solution(pl)))
    for pl, d, w, s in singles:
        ecl.solve(pl, d, w, s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, d, w, s in singles:
        ecl.solve(pl, d, w, s)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3
    ok_single = all(int((s.status != 0).sum().item()) == 0 for _, _, _, s in singles)
    del singles
    return {"workload": "c3: " + WORKLOADS["c3"], "stages": stages,
            "batched_ms": batched_ms, "batched_stages_per_s": stages / (batched_ms * 1e-3),
            "single_loop_ms": loop_ms, "single_loop_stages_per_s": stages / (loop_ms * 1e-3),
            "batched_over_single": loop_ms / batched_ms, "status_ok": ok_batched and ok_single}


def secondary_fast_multipliers(ecl, torch, problems, tuning, steps, warmup, graph, minnorm_ms):
    """The same workload with the factor-reusing multiplier route
    (multipliers = 2) in the launch configuration of the headline run."""
    plan = ecl.Plan.for_problems(problems, multipliers=2, use_graph=graph)
    ecl.set_tuning(plan, **{k: v for k, v in tuning.items() if k not in ("ms_per_solve", "use_graph")})
    data = ecl.pack(plan, problems)
    ws = plan.workspace()
    sol = ecl.allocate_solution(plan)
    wall_ms, ev_ms = time_solves(ecl, torch, plan, data, ws, sol, steps, warmup)
    ok = int((sol.status != 0).sum().item()) == 0
    prof = kernel_profile(ecl, torch, plan, data, ws, sol, max(2, steps // 2))
    stages = sum(p.N for p in problems)
    return {"ms_per_solve": wall_ms, "stages_per_s": stages / (wall_ms * 1e-3),
            "speedup_over_minimum_norm": minnorm_ms / wall_ms, "status_ok": ok,
            "kernel_ms_per_solve": {k: v[0] for k, v in prof.items() if v[1]}}


def secondary_differentiable(ecl, torch, steps):
    """Forward solve + backward (gradients of sum ||x||^2 + ||u||^2 with
    respect to every field) of the 256-instance batch; instance 0 checked
    against the oracle (x, u, lambda, mu at 1e-9) and one central finite
    difference (h = 1e-6, 1e-6 relative)."""
    from paper_2407_05433_amd.autograd import eclqr_layer
    problems = make("c4")
    plan = ecl.Plan.for_problems(problems)
    base = ecl.pack(plan, problems)
    ws = plan.workspace()

    def step():
        leaves = {k: v.detach().clone().requires_grad_(True) for k, v in base.items()}
        x, u, lam, mu, status = eclqr_layer(plan, leaves, ws)
        loss = (x * x).sum() + (u * u).sum()
        loss.backward()
        return leaves, x, u, lam, mu, status

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    leaves, x, u, lam, mu, status = out
    res = {"workload": "c4: " + WORKLOADS["c4"], "fwd_bwd_ms": ms, "status_ok": int((status != 0).sum().item()) == 0}
    try:
        from oracle import solve_with_multipliers
        from oracle.gradients import directional, effective_direction, fd_directional_corrected, random_direction
        p = problems[0]
        o = solve_with_multipliers(p)
        got = {"x": ecl.unpack(plan, x.detach(), "q", problems)[0], "u": ecl.unpack(plan, u.detach(), "r", problems)[0],
               "lam": ecl.unpack(plan, lam, "q", problems)[0], "mu": ecl.unpack(plan, mu, "g", problems)[0]}
        errs = {k: float(np.linalg.norm(np.concatenate([np.ravel(a) for a in got[k]]) -
                                        np.concatenate([np.ravel(a) for a in o[k]])) /
                         max(np.linalg.norm(np.concatenate([np.ravel(a) for a in o[k]])), 1e-300)) for k in got}
        G = {}
        for f in ("Q", "q", "R", "r", "A", "B", "c", "E", "F", "g", "x0"):
            g = leaves[f].grad.detach().cpu().numpy()
            offs, _ = plan.layout(f)
            if f == "x0":
                G[f] = g[offs[0]:offs[0] + p.nx[0]].copy()
            else:
                G[f] = [g[int(offs[i]):int(offs[i]) + a.size].reshape(a.shape) for i, a in enumerate(getattr(p, f))]
        d = random_direction(p, np.random.default_rng(7))
        d.pop("M", None)
        an = directional(G, effective_direction(p, d, 1e-6))
        fd = fd_directional_corrected(p, o, d, 1e-6)
        res["check_instance0"] = {"rel_err": errs, "fd_rel_err": abs(fd - an) / max(abs(fd), abs(an)),
                                  "pass": max(errs.values()) <= 1e-9 and abs(fd - an) / max(abs(fd), abs(an)) <= 1e-6}
    except Exception as ex:  # the check is a report, not part of the timing
        res["check_instance0"] = {"error": repr(ex)}
    return res


def stored_traffic(kernel_class, workload):
    """HBM bytes per launch of `kernel_class` on `workload` from a committed
    rocprofv3 --pmc summary under profiles/ (FETCH_SIZE and WRITE_SIZE runs,
    calibrated against a device copy), or None when there is none or when the
    kernel sources it hashes have changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md"))):
        kv = {}
        with open(path) as fh:
            for ln in fh:
                if ":" in ln and ln[:1].isalpha():
                    k, v = ln.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("traffic_kernel_class") != kernel_class or kv.get("traffic_workload") != workload:
            continue
        h = hashlib.sha256()
        try:
            for f in kv.get("sources", "").split():
                with open(os.path.join(ROOT, f), "rb") as fh:
                    h.update(fh.read())
        except OSError:
            return None
        if h.hexdigest() != kv.get("sources_sha256"):
            return None
        return float(kv["traffic_bytes_per_launch"])
    return None


def cpu_baseline(problems, min_s=10.0, max_s=30.0):
    """The oracle (sequential method + minimum-norm multipliers + one
    refinement step) on a bounded sample of the workload: instances in order,
    cycling, until at least min_s seconds (at most max_s) have passed."""
    from oracle import solve_with_multipliers
    t0 = time.perf_counter()
    stages, solves, i = 0, 0, 0
    while True:
        p = problems[i % len(problems)]
        solve_with_multipliers(p)
        stages += p.N
        solves += 1
        i += 1
        dt = time.perf_counter() - t0
        if dt >= min_s or dt > max_s:
            break
    distinct = min(solves, len(problems))
    return {"value": stages / dt, "unit": "stages/s", "cores": 1, "kind": "oracle",
            "sample": f"{solves} solves of {distinct} of the {len(problems)} instances ({stages} stages), "
                      f"{dt:.1f} s, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--graph", type=int, default=1, help="replay the solve as a captured hipGraph (1) or launch eagerly (0)")
    ap.add_argument("--autotune", type=int, default=1, help="choose the launch configuration by timing first (untimed)")
    ap.add_argument("--scan-schedule", type=int, default=0, choices=(0, 1, 2),
                    help="scan parenthesization: 0 automatic, 1 balanced up/down sweep, 2 recursive doubling")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device once (reference for hardware byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (a batch would split across GPUs "
              "by instances; a long horizon by stage chunks with one small all-gather per scan); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration, "bytes_read": n * 8, "bytes_written": n * 8}))
        return
    import paper_2407_05433_amd as ecl
    from paper_2407_05433_amd import flops as flopmodel

    log(f"[bench] generating {args.workload}")
    problems = make(args.workload)
    plan = ecl.Plan.for_problems(problems, use_graph=args.graph, scan_schedule=args.scan_schedule)
    data = ecl.pack(plan, problems)
    ws = plan.workspace()
    sol = ecl.allocate_solution(plan)
    stages = sum(p.N for p in problems)
    log(f"[bench] {len(problems)} instances, {stages} stages, workspace {plan.workspace_bytes / 2**20:.1f} MiB")
    tuning = ecl.autotune(plan, data, ws, sol) if args.autotune else ecl.get_tuning(plan)
    log(f"[bench] launch configuration {tuning}")
    wall_ms, ev_ms = time_solves(ecl, torch, plan, data, ws, sol, args.steps, args.warmup)
    st = sol.status.cpu().numpy()
    if np.any(st != 0):
        log(f"[bench] WARNING: nonzero status {np.unique(st)}")
    log(f"[bench] {wall_ms:.3f} ms/solve wall, {ev_ms:.3f} ms/solve events")
    prof = kernel_profile(ecl, torch, plan, data, ws, sol, max(3, args.steps // 2))
    for k, (ms, n) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        if n:
            log(f"[bench]   {k:14s} {ms:8.3f} ms/solve  {n:6.1f} launches/solve")
    # roofline of the dominant kernel class (algorithmic FP64 flops / its time)
    rsteps = plan.refine_steps(ws)
    work = flopmodel.solve_flops(plan, problems, ws, steps=rsteps)
    dom = max((k for k in prof if prof[k][1] > 0 and k in work), key=lambda k: prof[k][0])
    dom_ms = prof[dom][0]
    dom_launches = prof[dom][1]
    achieved = work[dom] / (dom_ms * 1e-3) / 1e12
    roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": stored_traffic(dom, args.workload),
            "flops_per_solve": work[dom], "ms_per_solve": dom_ms, "launches_per_solve": dom_launches,
            "avg_launch_us": dom_ms * 1e3 / max(dom_launches, 1)}
    total_flops = sum(work.values())
    log(f"[bench] dominant {dom}: {achieved:.3f} TFLOP/s ({100 * achieved / FP64_VECTOR_PEAK_TFLOPS:.2f}% of FP64 "
        f"vector peak); whole solve {total_flops / (ev_ms * 1e-3) / 1e12:.3f} TFLOP/s")

    line = {
        "metric": "stages/s solved (primal+multipliers)",
        "value": stages / (wall_ms * 1e-3),
        "unit": "stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "instances": len(problems),
                   "stages": stages, "multipliers": True, "launch": tuning,
                   "scan_schedule": scan_schedule_name(plan),
                   "refine": {"max_steps": int(plan.options.refine), "tol": float(plan.options.refine_tol),
                              "steps_taken": {str(int(k)): int(v) for k, v in zip(*np.unique(rsteps, return_counts=True))}}},
        "roofline": roof,
        "kernel_ms_per_solve": {k: v[0] for k, v in prof.items() if v[1]},
    }
    if not args.no_secondary:
        del ws, sol, data
        torch.cuda.empty_cache()
        log("[bench] secondary: the same workload with the factor-reusing multiplier route")
        sec = {"fast_multipliers": secondary_fast_multipliers(ecl, torch, problems, tuning, args.steps, args.warmup,
                                                              args.graph, wall_ms)}
        log(f"[bench]   {sec['fast_multipliers']}")
        torch.cuda.empty_cache()
        log("[bench] secondary: c3 batched vs single-instance loop")
        sec["batched_vs_single"] = secondary_batched(ecl, torch, max(1, min(args.steps, 3)))
        log(f"[bench]   {sec['batched_vs_single']}")
        torch.cuda.empty_cache()
        log("[bench] secondary: c4 forward + backward")
        sec["differentiable"] = secondary_differentiable(ecl, torch, max(1, min(args.steps, 5)))
        log(f"[bench]   {sec['differentiable']}")
        line["secondary"] = sec
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(problems)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
