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


def cpu_baseline(problems, budget_s=20.0):
    """The oracle (sequential method + minimum-norm multipliers + one
    refinement step) on a bounded sample of the workload's instances."""
    from oracle import solve_with_multipliers
    t0 = time.perf_counter()
    stages, used = 0, 0
    for p in problems:
        solve_with_multipliers(p)
        stages += p.N
        used += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": stages / dt, "unit": "stages/s", "cores": 1, "kind": "oracle",
            "sample": f"{used} of {len(problems)} instances ({stages} stages), {dt:.1f} s, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (batches and horizons shard "
              "across GPUs without communication, see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2407_05433_amd as ecl
    from paper_2407_05433_amd import flops as flopmodel

    log(f"[bench] generating {args.workload}")
    problems = make(args.workload)
    plan = ecl.Plan.for_problems(problems)
    data = ecl.pack(plan, problems)
    ws = plan.workspace()
    sol = ecl.allocate_solution(plan)
    stages = sum(p.N for p in problems)
    log(f"[bench] {len(problems)} instances, {stages} stages, workspace {plan.workspace_bytes / 2**20:.1f} MiB")
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
            "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
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
                   "stages": stages, "multipliers": True,
                   "refine": {"max_steps": int(plan.options.refine), "tol": float(plan.options.refine_tol),
                              "steps_taken": {str(int(k)): int(v) for k, v in zip(*np.unique(rsteps, return_counts=True))}}},
        "roofline": roof,
        "kernel_ms_per_solve": {k: v[0] for k, v in prof.items() if v[1]},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(problems)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
