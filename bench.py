"""Benchmark: stages/s of the full solve (primal + multipliers) on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c3|c1|c2|c4|paper]

A step is one solve of the whole hot path (feasible-domain scan, stage
elimination, reduced-LQR scan, recovery, multipliers, and the iterative
refinement an instance takes when its backward error after the first pass
exceeds 1e-10) of one batch of synthetic instances already resident in HBM.
The default workload is the 512-instance batch solved in one call; beside it
the same instances are solved one after another with single-instance plans
(batched vs single), and the single instances (N=1024; N=8192 with n=32) and
the 256-instance differentiable batch (forward, and forward + backward) are
measured as secondaries.  Prints one JSON line; the per-kernel breakdowns go
to stderr and to the "secondary" object.

Roofline: the kernel class that takes the most time per solve, its
algorithmic FP64 flops being the method's work: the kernels' nominal counts at
the actual dims of every stage and of the tasks of the balanced up/down sweep
(two combines per stage and scan, the O(N) scan of the paper's Section IV),
whichever parenthesization ran; vector-only replays by the bytes of the
factors they read.
"""

from __future__ import annotations

import os

# the oracle (CPU baseline) runs one instance per process, one BLAS thread
# each; set before NumPy loads, so no BLAS thread pool exists when the pool's
# workers are forked
for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

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
METRIC = "stages/s solved (primal+multipliers) batched vs single; fwd+bwd ms at 1e-9 acc"

WORKLOADS = {
    "c0": "tiny: 1 instance, N=16, n=4, m=2, 1 mixed row/stage, 2 terminal rows",
    "c1": "single: 1 instance, N=1024, n=12, m=6, k_i in {0..4} (state/mixed, 10% redundant), 3 terminal rows",
    "c2": "dae: 1 instance, N=8192, n=32, m=16, 6 algebraic rows/stage + 4 state rows every 8th stage",
    "c3": "batched: 512 instances, N in [32,512], n in [6,24], m in [3,12], k_i in [0,m-1]",
    "c4": "differentiable: 256 instances, N=128, n=16, m=8, 3 mixed rows/stage",
    "paper": "paper Table I shape: 1 instance, N=8192, n=8, m=4, 2 state rows/stage",
}
MPC_WORKLOAD = ("bounded: 256 instances, N=128, n=16, m=8, 3 mixed rows/stage, inputs boxed at +-0.5 around a "
                "feasible trajectory; Mehrotra predictor-corrector, 25 iterations")
IPM_ITER = 25


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
    t0 = time.perf_counter()
    for _ in range(steps):
        ecl.solve(plan, data, ws, sol)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def kernel_profile(ecl, torch, plan, data, ws, sol, steps):
    """{class: (ms per solve, launches per solve)} from HIP events around
    every launch on the launch stream (eager launches)."""
    plan.set_profiling(True)
    plan.profile(reset=True)
    for _ in range(steps):
        ecl.solve(plan, data, ws, sol)
    torch.cuda.synchronize()
    prof = plan.profile(reset=True)
    plan.set_profiling(False)
    return {k: (ms / steps, n / steps) for k, (ms, n) in prof.items()}


def method_work(ecl, torch, problems, data, multipliers=True):
    """Flops per kernel class of the method's work: the same problem solved
    once (untimed) by a plan with the balanced up/down sweep, its flop model
    evaluated at that solve's dims, plus the bytes of the factor logs a
    vector-only replay pass reads."""
    from paper_2407_05433_amd import flops as flopmodel
    plan = ecl.Plan.for_problems(problems, scan_schedule=1)
    ws = plan.workspace()
    sol = ecl.solve(plan, data, ws)
    torch.cuda.synchronize()
    work = flopmodel.solve_flops(plan, problems, ws, multipliers=multipliers)
    del sol, ws
    torch.cuda.empty_cache()
    return work


def replay_bytes(plan):
    """Bytes of the factors one vector-only pass of the problem and of its
    multiplier route reads (relation and value-function logs, stage arenas)."""
    return float(sum(plan.footprint(w)["factor_bytes"] for w in (0, 2) if plan.has_engine(w)))


def roofline(prof, work, replay_b, passes):
    """The class with the most time per solve among those that do work in it
    (achieved = algorithmic work per solve / its time per solve, which per
    launch is the same ratio).  A class whose launches do no work in this
    solve (replay when no instance refines: its workgroups exit at once) is
    listed under "skipped" with its time and launch count instead."""
    def work_of(k):
        return replay_b * passes if k == "replay" else work.get(k, 0.0)
    live = [k for k in prof if prof[k][1] > 0 and work_of(k) > 0]
    skipped = [{"kernel": k, "ms_per_solve": prof[k][0], "launches_per_solve": prof[k][1],
                "reason": "no modeled work in this solve (launches whose workgroups return at once)"}
               for k in prof if prof[k][1] > 0 and work_of(k) <= 0 and prof[k][0] >= max(v[0] for v in prof.values()) * 0.25]
    dom = max(live, key=lambda k: prof[k][0])
    ms, launches = prof[dom]
    if dom == "replay":
        achieved = replay_b * passes / (ms * 1e-3) / 1e9
        out = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": achieved / HBM_PEAK_GBS, "bytes_per_solve": replay_b * passes, "ms_per_solve": ms,
               "launches_per_solve": launches, "avg_launch_us": ms * 1e3 / max(launches, 1)}
    else:
        achieved = work.get(dom, 0.0) / (ms * 1e-3) / 1e12
        out = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "flops_per_solve": work.get(dom, 0.0), "ms_per_solve": ms,
               "launches_per_solve": launches, "avg_launch_us": ms * 1e3 / max(launches, 1)}
    if skipped:
        out["skipped"] = skipped
    return out


def paper_context(ms):
    """The paper's own number for the same shape (Table I, N = 8192: one
    instance, n = 8, m = 4, two state-only rows per stage, primal and
    multipliers, FP64), quoted with its hardware: context, not a target."""
    return {"source": "Table I, N=8192", "hardware": "NVIDIA Tesla P100 PCIe 16 GiB, CUDA 12.8; CPU: one thread of "
            "a virtualized 2.0 GHz Xeon", "gpu_kernel_ms": 10.518, "gpu_wall_ms": 17.274, "cpu_1thread_ms": 106.424,
            "this_ms_per_solve": ms, "paper_gpu_kernel_ms_over_this": 10.518 / ms}


def measure(ecl, torch, workload, problems, steps, warmup, graph=1, autotune=1, scan_schedule=0, tuning=None):
    """Autotuned solve of one workload: wall ms per solve (graph replay),
    per-class profile, method-work roofline of the dominant class.  With
    autotune = 0, `tuning` (a dict of eclqr_tuning fields) is applied instead."""
    plan = ecl.Plan.for_problems(problems, use_graph=graph, scan_schedule=scan_schedule)
    data = ecl.pack(plan, problems)
    ws = plan.workspace()
    sol = ecl.allocate_solution(plan)
    stages = sum(p.N for p in problems)
    if not autotune and tuning:
        ecl.set_tuning(plan, **tuning)
    tuning = ecl.autotune(plan, data, ws, sol) if autotune else ecl.get_tuning(plan)
    ms = time_solves(ecl, torch, plan, data, ws, sol, steps, warmup)
    status_ok = int((sol.status != 0).sum().item()) == 0
    prof = kernel_profile(ecl, torch, plan, data, ws, sol, max(2, min(steps, 5)))
    rsteps = plan.refine_steps(ws)
    # vector passes per solve: two per refinement step (the problem and its
    # multiplier route; averaged over instances: a finished instance's tasks
    # return at once), plus the multiplier route's pass at the primal point
    # when its factorization was overlapped
    passes = 2.0 * float(np.mean(rsteps)) + (1.0 if tuning.get("overlap_dual") else 0.0)
    rb = replay_bytes(plan)
    sched = scan_schedule_name(plan)
    del ws, sol
    torch.cuda.empty_cache()
    work = method_work(ecl, torch, problems, data)
    roof = roofline(prof, work, rb, passes)
    res = {"workload": f"{workload}: {WORKLOADS[workload]}", "instances": len(problems), "stages": stages,
           "ms_per_solve": ms, "stages_per_s": stages / (ms * 1e-3), "status_ok": status_ok,
           "launch": tuning, "scan_schedule": sched,
           "refine_steps_taken": {str(int(k)): int(v) for k, v in zip(*np.unique(rsteps, return_counts=True))},
           "roofline": roof, "kernel_ms_per_solve": {k: v[0] for k, v in prof.items() if v[1]},
           "launches_per_solve": {k: v[1] for k, v in prof.items() if v[1]},
           "method_flops_per_solve": sum(work.values())}
    log(f"[bench] {workload}: {ms:.3f} ms/solve, {res['stages_per_s']:.0f} stages/s, schedule {sched}, "
        f"dominant {roof['kernel']} {100 * roof['frac']:.3f}% of {roof['peak']} {roof['unit']}")
    for k, (kms, n) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        if n:
            log(f"[bench]   {k:18s} {kms:8.3f} ms/solve  {n:7.1f} launches/solve")
    return res, plan, data


def single_loop(ecl, torch, problems):
    """The same instances solved one after another, each with its own
    single-instance plan (graph replay), wall time of the whole loop."""
    singles = []
    for p in problems:
        pl = ecl.Plan.for_problems([p], use_graph=1)
        singles.append((pl, ecl.pack(pl, [p]), pl.workspace(), ecl.allocate_solution(pl)))
    for _ in range(2):  # capture, then one replay
        for pl, d, w, s in singles:
            ecl.solve(pl, d, w, s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, d, w, s in singles:
        ecl.solve(pl, d, w, s)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    ok = all(int((s.status != 0).sum().item()) == 0 for _, _, _, s in singles)
    del singles
    torch.cuda.empty_cache()
    return ms, ok


def differentiable(ecl, torch, steps):
    """Forward solve + backward (gradients of sum ||x||^2 + ||u||^2 with
    respect to every field) of the 256-instance batch; instance 0 checked
    against the oracle (x, u, lambda, mu at 1e-9) and one central finite
    difference (h = 1e-6, 1e-6 relative) in the same run."""
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
               "lam": ecl.unpack(plan, lam.detach(), "q", problems)[0], "mu": ecl.unpack(plan, mu.detach(), "g", problems)[0]}
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
    del ws
    torch.cuda.empty_cache()
    return res


def interior_point(ecl, torch, steps):
    """The interior-point driver on the bounded batch: one step is a whole
    bound-constrained solve (start solve + IPM_ITER predictor-corrector
    iterations, each a full solve and a factor-replaying solve of the
    256-instance Newton problem), one captured graph per iteration.  Reports
    the converged fraction and the optimality conditions of instance 0
    (evaluated by the oracle's residual function on the device result)."""
    from workloads import config_mpc
    problems = config_mpc()
    bounds = [p.meta["bounds"] for p in problems]
    plan = ecl.Plan.for_problems(problems)
    plan.set_graph(True)
    data = ecl.pack(plan, problems)
    bd = ecl.pack_bounds(plan, problems, bounds)
    ws = ecl.ipm_workspace(plan)
    sol = ecl.ipm_solve(plan, data, bd, ws, iterations=IPM_ITER)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ecl.ipm_solve(plan, data, bd, ws, sol, iterations=IPM_ITER)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    stages = sum(p.N + 1 for p in problems)
    st, it, comp = sol.status.cpu().numpy(), sol.steps.cpu().numpy(), sol.comp.cpu().numpy()
    res = {"workload": "mpc: " + MPC_WORKLOAD, "ms_per_solve": ms, "ms_per_iteration": ms / IPM_ITER,
           "newton_stage_solves_per_s": 2 * IPM_ITER * stages / (ms * 1e-3),
           "converged_fraction": float(np.mean((st == 0) & (comp < 1e-8))),
           "iterations_taken": [int(it.min()), int(it.max())], "status_ok": bool((st == 0).all())}
    plan.set_graph(False)
    plan.set_profiling(True)
    plan.profile(reset=True)
    ecl.ipm_solve(plan, data, bd, ws, sol, iterations=IPM_ITER)
    torch.cuda.synchronize()
    prof = plan.profile(reset=True)
    plan.set_profiling(False)
    res["kernel_ms_per_solve"] = {k: round(v[0], 4) for k, v in prof.items() if v[1] > 0}
    try:
        from oracle.ipm import bound_kkt_residual
        p = problems[0]
        got = {f: ecl.unpack(plan, getattr(sol, f), fl, [p])[0]
               for f, fl in (("x", "q"), ("u", "r"), ("lam", "q"), ("mu", "g"), ("z_ulo", "r"), ("z_uhi", "r"),
                             ("z_xlo", "q"), ("z_xhi", "q"))}
        got["z_u"] = list(zip(got["z_ulo"], got["z_uhi"]))
        got["z_x"] = list(zip(got["z_xlo"], got["z_xhi"]))
        res["kkt_instance0"] = bound_kkt_residual(p, bounds[0], got)
    except Exception as ex:  # a report, not part of the timing
        res["kkt_instance0"] = {"error": repr(ex)}
    del ws, sol
    torch.cuda.empty_cache()
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


def _oracle_task(p):
    from oracle import solve_with_multipliers
    solve_with_multipliers(p)
    return p.N


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(problems, min_s=12.0):
    """The oracle (sequential method + minimum-norm multipliers + one
    refinement step) on a bounded sample of the workload: instances in order,
    one per task, over a process pool of the host cores this job may use (at
    most 16), a new task started whenever one ends until min_s seconds have
    passed; every started task is finished and counted."""
    import concurrent.futures as cf
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    stages = solves = nxt = 0
    with cf.ProcessPoolExecutor(cores, mp_context=mp.get_context("fork")) as ex:
        live = set()
        while True:
            while len(live) < cores and time.perf_counter() - t0 < min_s:
                live.add(ex.submit(_oracle_task, problems[nxt % len(problems)]))
                nxt += 1
            if not live:
                break
            done, live = cf.wait(live, return_when=cf.FIRST_COMPLETED)
            for f in done:
                stages += f.result()
                solves += 1
                if solves % 16 == 0:
                    log(f"[bench]   oracle: {solves} solves, {stages} stages, {time.perf_counter() - t0:.1f} s")
    dt = time.perf_counter() - t0
    distinct = min(solves, len(problems))
    return {"value": stages / dt, "unit": "stages/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{solves} solves of the first {distinct} of the {len(problems)} instances ({stages} stages) "
                      f"in {dt:.1f} s, one instance per process, {cores} processes of one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-single-loop", action="store_true",
                    help="skip the one-by-one solves of the batch (counter runs of the batched solve)")
    ap.add_argument("--graph", type=int, default=1, help="replay the solve as a captured hipGraph (1) or launch eagerly (0)")
    ap.add_argument("--autotune", type=int, default=1, help="choose the launch configuration by timing first (untimed)")
    ap.add_argument("--tuning", default=None, metavar="JSON",
                    help="with --autotune 0: eclqr_tuning fields to set, e.g. the configuration an autotuned run chose")
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

    log(f"[bench] generating {args.workload}")
    problems = make(args.workload)
    cpu = None
    if not args.no_cpu and not args.copy_calibration:
        # before the GPU is touched: the pool's worker processes are forked
        # from a process without a device context
        log("[bench] cpu baseline (oracle, process pool)")
        cpu = cpu_baseline(problems)
        log(f"[bench]   {cpu}")

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

    head, plan, data = measure(ecl, torch, args.workload, problems, args.steps, args.warmup, args.graph,
                               args.autotune, args.scan_schedule, json.loads(args.tuning) if args.tuning else None)
    roof = dict(head["roofline"])
    roof["traffic"] = stored_traffic(roof["kernel"], args.workload)
    del plan, data
    torch.cuda.empty_cache()
    line = {
        "metric": METRIC,
        "value": head["stages_per_s"],
        "unit": "stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "instances": head["instances"], "stages": head["stages"],
                   "multipliers": True, "launch": head["launch"], "scan_schedule": head["scan_schedule"],
                   "refine": {"accept_backward_error": 1e-10, "steps_taken": head["refine_steps_taken"]}},
        "roofline": roof,
        "kernel_ms_per_solve": head["kernel_ms_per_solve"],
        "launches_per_solve": head["launches_per_solve"],
    }
    if args.workload == "c3" and not args.no_single_loop:
        log("[bench] the same 512 instances one after another (single-instance plans)")
        loop_ms, ok = single_loop(ecl, torch, problems)
        line["batched_vs_single"] = {"batched_ms": head["ms_per_solve"], "batched_stages_per_s": head["stages_per_s"],
                                     "single_loop_ms": loop_ms,
                                     "single_loop_stages_per_s": head["stages"] / (loop_ms * 1e-3),
                                     "batched_over_single": loop_ms / head["ms_per_solve"], "status_ok": ok}
        log(f"[bench]   {line['batched_vs_single']}")
    if not args.no_secondary:
        sec = {}
        for w in ("c1", "c2", "c4", "paper"):
            if w == args.workload:
                continue
            log(f"[bench] secondary: {w}")
            r, pl, dt = measure(ecl, torch, w, make(w), max(3, min(args.steps, 10)), 2)
            del pl, dt
            torch.cuda.empty_cache()
            if w == "paper":
                r["paper_context"] = paper_context(r["ms_per_solve"])
            sec[w] = r
        log("[bench] secondary: c4 forward + backward")
        sec["c4_fwd_bwd"] = differentiable(ecl, torch, max(2, min(args.steps, 5)))
        log(f"[bench]   {sec['c4_fwd_bwd']}")
        log("[bench] secondary: bounded batch, interior-point driver")
        sec["mpc_ipm"] = interior_point(ecl, torch, max(2, min(args.steps, 5)))
        log(f"[bench]   {sec['mpc_ipm']}")
        line["secondary"] = sec
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
