"""Python binding of the solver: plans, packing into flat device tensors, and
the solve / backward / residual calls of the C ABI.  PyTorch provides device
memory and the current HIP stream; every computation runs in the HIP kernels."""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import FIELDS, FIELD_INDEX, check, lib


def default_options(**kw) -> _lib.Options:
    o = _lib.Options()
    lib().eclqr_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Plan:
    """Host-side plan for a batch of instances with given per-stage dims.

    ``dims`` is a list of (nx, nu, nc) per instance: nx has N+1 entries, nu N,
    nc N+1 (the last = terminal rows)."""

    def __init__(self, dims: Sequence, **options):
        nx, nu, nc, hor = [], [], [], []
        for (x, u, c) in dims:
            N = len(u)
            if len(x) != N + 1 or len(c) != N + 1:
                raise ValueError("nx and nc need N+1 entries, nu N")
            hor.append(N)
            nx += list(x)
            nu += list(u)
            nc += list(c)
        self.horizons = hor
        self.batch = len(hor)
        self._nx = np.asarray(nx, dtype=np.int32)
        self._nu = np.asarray(nu, dtype=np.int32)
        self._nc = np.asarray(nc, dtype=np.int32)
        d = _lib.Dims(self.batch, self._arr(hor), self._arr(nx), self._arr(nu), self._arr(nc))
        self.options = default_options(**options)
        h = C.c_void_p()
        check(lib().eclqr_plan_create(C.byref(h), C.byref(d), C.byref(self.options)), "eclqr_plan_create")
        self._h = h
        sz = C.c_size_t()
        check(lib().eclqr_plan_workspace_size(h, C.byref(sz)), "eclqr_plan_workspace_size")
        self.workspace_bytes = int(sz.value)
        self._layout: Dict[str, tuple] = {}

    @staticmethod
    def _arr(v):
        a = (C.c_int32 * max(1, len(v)))()
        for i, x in enumerate(v):
            a[i] = int(x)
        return a

    @classmethod
    def for_problems(cls, problems, **options) -> "Plan":
        return cls([(p.nx, p.nu, p.nc) for p in problems], **options)

    def layout(self, field: str):
        """(per-stage offsets as int64 numpy array, total elements)."""
        if field not in self._layout:
            ptr = C.POINTER(C.c_int64)()
            cnt, tot = C.c_int64(), C.c_int64()
            check(lib().eclqr_plan_layout(self._h, FIELD_INDEX[field], C.byref(ptr), C.byref(cnt), C.byref(tot)),
                  "eclqr_plan_layout")
            offs = np.ctypeslib.as_array(ptr, shape=(cnt.value,)).copy() if cnt.value else np.zeros(0, np.int64)
            self._layout[field] = (offs, int(tot.value))
        return self._layout[field]

    def schedule(self, dual: bool = False) -> List[np.ndarray]:
        lev = C.c_int32()
        check(lib().eclqr_plan_schedule(self._h, int(dual), C.byref(lev), -1, None, None), "eclqr_plan_schedule")
        out = []
        for level in range(lev.value):
            ptr = C.POINTER(C.c_int32)()
            nt = C.c_int32()
            check(lib().eclqr_plan_schedule(self._h, int(dual), None, level, C.byref(ptr), C.byref(nt)),
                  "eclqr_plan_schedule")
            out.append(np.ctypeslib.as_array(ptr, shape=(nt.value * 3,)).reshape(-1, 3).copy()
                       if nt.value else np.zeros((0, 3), np.int32))
        return out

    def set_graph(self, on: bool) -> None:
        """Capture the solve's launch sequence as a hipGraph and replay it."""
        check(lib().eclqr_plan_set_graph(self._h, int(on)), "eclqr_plan_set_graph")

    def set_profiling(self, on: bool) -> None:
        check(lib().eclqr_plan_set_profiling(self._h, int(on)), "eclqr_plan_set_profiling")

    def profile(self, reset: bool = True) -> Dict[str, tuple]:
        """{kernel class: (total ms, launches)} of the launches recorded since the last reset."""
        n = _lib.NUM_KERNEL_CLASSES
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        check(lib().eclqr_plan_profile(self._h, ms, cnt, int(reset)), "eclqr_plan_profile")
        return {lib().eclqr_kernel_class_name(k).decode(): (ms[k], cnt[k]) for k in range(n)}

    def reduced_dims(self, ws: torch.Tensor, dual: bool = False, which: Optional[int] = None):
        """(n-bar, m-bar) per stage from the last solve in ``ws`` (synchronises);
        which = 2: (r, f) of the theta LQR of the minimum-norm route."""
        w = int(dual) if which is None else int(which)
        S = int(sum(h + 2 for h in self.horizons)) if w == 1 else len(self._nx)
        nb = (C.c_int32 * S)()
        mb = (C.c_int32 * S)()
        wptr, _ = _aligned_ws(ws)
        check(lib().eclqr_plan_reduced_dims(self._h, C.c_void_p(wptr), w, nb, mb), "eclqr_plan_reduced_dims")
        return np.frombuffer(nb, dtype=np.int32).copy(), np.frombuffer(mb, dtype=np.int32).copy()

    def refine_steps(self, ws: torch.Tensor) -> np.ndarray:
        """Refinement steps each instance took in the last solve in ``ws`` (synchronises)."""
        out = (C.c_int32 * max(1, self.batch))()
        wptr, _ = _aligned_ws(ws)
        check(lib().eclqr_plan_refine_steps(self._h, C.c_void_p(wptr), out), "eclqr_plan_refine_steps")
        return np.frombuffer(out, dtype=np.int32)[:self.batch].copy()

    def backward_error(self, ws: torch.Tensor) -> np.ndarray:
        """Componentwise KKT backward error of each instance at the point the last solve returned (0 with
        refine = 0; synchronises)."""
        out = (C.c_double * max(1, self.batch))()
        wptr, _ = _aligned_ws(ws)
        check(lib().eclqr_plan_backward_error(self._h, C.c_void_p(wptr), out), "eclqr_plan_backward_error")
        return np.frombuffer(out, dtype=np.float64)[:self.batch].copy()

    def scan_rows(self, ws: Optional[torch.Tensor], dual: bool = False) -> np.ndarray:
        """Rows of every feasible-domain-scan slot after the last solve (synchronises)."""
        n = C.c_int32()
        check(lib().eclqr_plan_scan_rows(self._h, None, int(dual), None, C.byref(n)), "eclqr_plan_scan_rows")
        rows = (C.c_int32 * max(1, n.value))()
        wptr, _ = _aligned_ws(ws)
        check(lib().eclqr_plan_scan_rows(self._h, C.c_void_p(wptr), int(dual), rows, C.byref(n)),
              "eclqr_plan_scan_rows")
        return np.frombuffer(rows, dtype=np.int32)[:n.value].copy()

    def combine_forms(self, ws: torch.Tensor, dual: bool = False) -> np.ndarray:
        """Form of the value-function combine of every scan slot in the last solve:
        0 none, 1 Cholesky-factored, 2 LU (synchronises)."""
        n = C.c_int32()
        check(lib().eclqr_plan_combine_forms(self._h, None, int(dual), None, C.byref(n)), "eclqr_plan_combine_forms")
        forms = (C.c_int32 * max(1, n.value))()
        wptr, _ = _aligned_ws(ws)
        check(lib().eclqr_plan_combine_forms(self._h, C.c_void_p(wptr), int(dual), forms, C.byref(n)),
              "eclqr_plan_combine_forms")
        return np.frombuffer(forms, dtype=np.int32)[:n.value].copy()

    def slot_info(self, dual: bool = False):
        """(instance, first leaf, end leaf) of every scan slot."""
        n = C.c_int32()
        check(lib().eclqr_plan_slot_info(self._h, int(dual), None, None, None, C.byref(n)), "eclqr_plan_slot_info")
        a, b, c = ((C.c_int32 * max(1, n.value))() for _ in range(3))
        check(lib().eclqr_plan_slot_info(self._h, int(dual), a, b, c, C.byref(n)), "eclqr_plan_slot_info")
        return tuple(np.frombuffer(x, dtype=np.int32)[:n.value].copy() for x in (a, b, c))

    def has_engine(self, which: int) -> bool:
        """Whether the plan lays out engine `which` (0 problem, 1 reversed-time
        problem, 2 theta LQR)."""
        out = (C.c_int64 * 4)()
        return lib().eclqr_plan_footprint(self._h, int(which), out) == 0

    def footprint(self, which: int = 0) -> Dict[str, int]:
        """Device bytes of one engine's workspace parts (eclqr_plan_footprint)."""
        out = (C.c_int64 * 4)()
        check(lib().eclqr_plan_footprint(self._h, int(which), out), "eclqr_plan_footprint")
        arena, rel, ric, slots = (int(v) for v in out)
        return {"arena_bytes": arena, "rel_log_bytes": rel, "ric_log_bytes": ric, "slot_bytes": slots,
                "factor_bytes": arena + rel + ric}

    def stage_dims(self, dual: bool = False):
        """(n, n', m, k) per stage of the problem or of the reversed-time problem."""
        nx, nu, nc = self._nx, self._nu, self._nc
        out = []
        s = u = 0
        for N in self.horizons:
            xs, us, cs = nx[s:s + N + 1], nu[u:u + N], nc[s:s + N + 1]
            if dual:
                dxs = [0] + [int(xs[N - j + 1]) for j in range(1, N + 2)]
                dus = [int(cs[N])] + [int(cs[N - j]) for j in range(1, N + 1)]
                dcs = [0] + [int(us[N - j]) for j in range(1, N + 1)] + [0]
                xs, us, cs, NN = dxs, dus, dcs, N + 1
            else:
                NN = N
            for i in range(NN + 1):
                out.append((int(xs[i]), int(xs[i + 1]) if i < NN else 0, int(us[i]) if i < NN else 0, int(cs[i])))
            s += N + 1
            u += N
        return out

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().eclqr_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h


def pack(plan: Plan, problems, device="cuda", with_M: Optional[bool] = None) -> Dict[str, torch.Tensor]:
    """Flat FP64 device tensors of every field, in the plan's layout (blocks in
    stage order, instance after instance)."""
    if with_M is None:
        with_M = any(np.any(Mi) for p in problems for Mi in p.M)
    out: Dict[str, torch.Tensor] = {}
    for f in FIELDS:
        if f == "M" and not with_M:
            continue
        if f == "x0":
            parts = [np.asarray(p.x0, dtype=np.float64).ravel() for p in problems]
        else:
            parts = [np.asarray(a, dtype=np.float64).ravel() for p in problems for a in getattr(p, f)]
        flat = np.concatenate(parts) if parts else np.zeros(0)
        offs, tot = plan.layout(f)
        if flat.size != tot:
            raise ValueError(f"field {f}: {flat.size} elements, layout expects {tot}")
        out[f] = torch.from_numpy(np.ascontiguousarray(flat)).to(device)
    return out


@dataclass
class Solution:
    x: torch.Tensor
    u: torch.Tensor
    lam: Optional[torch.Tensor]
    mu: Optional[torch.Tensor]
    status: torch.Tensor
    info: Optional[torch.Tensor] = None  # per instance: stage of the first failure in Algorithm 1's order, -1 none

    def ptrs(self) -> _lib.SolutionPtrs:
        return _lib.SolutionPtrs(self.x.data_ptr(), self.u.data_ptr(),
                                 self.lam.data_ptr() if self.lam is not None else None,
                                 self.mu.data_ptr() if self.mu is not None else None, self.status.data_ptr(),
                                 self.info.data_ptr() if self.info is not None else None)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if t.dtype == torch.float64 or t.dtype == torch.int32 or t.dtype == torch.uint8:
        return C.c_void_p(t.data_ptr()) if t.numel() else C.c_void_p(t.data_ptr() or 0)
    raise TypeError(t.dtype)


def _problem_ptrs(data: Dict[str, torch.Tensor]) -> _lib.ProblemPtrs:
    pp = _lib.ProblemPtrs()
    for f in FIELDS:
        t = data.get(f)
        setattr(pp, f, t.data_ptr() if (t is not None and t.numel()) else (t.data_ptr() if t is not None else None))
    return pp


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _aligned_ws(ws: torch.Tensor):
    base = ws.data_ptr()
    off = (-base) % 256
    return base + off, ws.numel() - off


def allocate_solution(plan: Plan, device="cuda", multipliers: bool = True) -> Solution:
    _, nq = plan.layout("q")
    _, nr = plan.layout("r")
    _, ng = plan.layout("g")
    mk = lambda n: torch.empty(max(1, n), dtype=torch.float64, device=device)  # noqa: E731
    return Solution(mk(nq), mk(nr), mk(nq) if multipliers else None, mk(ng) if multipliers else None,
                    torch.empty(plan.batch, dtype=torch.int32, device=device),
                    torch.empty(plan.batch, dtype=torch.int32, device=device))


def solve(plan: Plan, data: Dict[str, torch.Tensor], ws: Optional[torch.Tensor] = None,
          out: Optional[Solution] = None) -> Solution:
    """eclqr_solve on the current stream (asynchronous)."""
    device = data["Q"].device
    if ws is None:
        ws = plan.workspace(device)
    if out is None:
        out = allocate_solution(plan, device, bool(plan.options.multipliers))
    sp = out.ptrs()
    pp = _problem_ptrs(data)
    wptr, wbytes = _aligned_ws(ws)
    check(lib().eclqr_solve(plan.handle, C.byref(pp), C.byref(sp), C.c_void_p(wptr), C.c_size_t(wbytes), _stream()),
          "eclqr_solve")
    out._ws = ws  # keep the workspace alive with the solution (backward reuses it)
    return out


def solve_noalloc(plan: Plan, data: Dict[str, torch.Tensor], out: Solution) -> Solution:
    """eclqr_solve_noalloc on the current stream: the solve with the library's
    static per-GPU scratch as its workspace (no allocation by the library;
    the caller provides the solution buffers)."""
    pp = _problem_ptrs(data)
    sp = out.ptrs()
    check(lib().eclqr_solve_noalloc(plan.handle, C.byref(pp), C.byref(sp), _stream()), "eclqr_solve_noalloc")
    return out


@dataclass
class IpmSolution:
    """Last iterate of the interior-point driver (layouts of q, r, q, g; bound
    multipliers of the inputs in the layout of r, of the states in that of q)."""
    x: torch.Tensor
    u: torch.Tensor
    lam: torch.Tensor
    mu: torch.Tensor
    z_ulo: torch.Tensor
    z_uhi: torch.Tensor
    z_xlo: torch.Tensor
    z_xhi: torch.Tensor
    comp: torch.Tensor
    steps: torch.Tensor
    status: torch.Tensor

    def ptrs(self) -> _lib.IpmSolutionPtrs:
        return _lib.IpmSolutionPtrs(*(getattr(self, f).data_ptr() for f, _ in _lib.IpmSolutionPtrs._fields_))


def pack_bounds(plan: Plan, problems, bounds, device="cuda") -> Dict[str, Optional[torch.Tensor]]:
    """Device arrays of box bounds in the plan's layouts: bounds[b] is a dict
    with any of u_lo, u_hi (one array per stage i < N), x_lo, x_hi (one per
    stage i <= N; the block of x_0 is ignored).  A key no instance has is None
    (no bound); a missing block is infinite."""
    out: Dict[str, Optional[torch.Tensor]] = {}
    for key, field in (("u_lo", "r"), ("u_hi", "r"), ("x_lo", "q"), ("x_hi", "q")):
        if all(b.get(key) is None for b in bounds):
            out[key] = None
            continue
        inf = -np.inf if key.endswith("lo") else np.inf
        parts = []
        for p, b in zip(problems, bounds):
            dims = p.nu if field == "r" else p.nx
            blocks = b.get(key)
            if blocks is None:
                blocks = [np.full(d, inf) for d in dims]
            if len(blocks) != len(dims):
                raise ValueError(f"bound {key}: {len(blocks)} blocks, the instance has {len(dims)}")
            parts += [np.asarray(v, dtype=np.float64).ravel() for v in blocks]
        flat = np.concatenate(parts) if parts else np.zeros(0)
        if flat.size != plan.layout(field)[1]:
            raise ValueError(f"bound {key}: {flat.size} elements, layout of {field} expects {plan.layout(field)[1]}")
        out[key] = torch.from_numpy(np.ascontiguousarray(flat)).to(device)
    return out


def ipm_default_params() -> Dict[str, float]:
    prm = _lib.IpmParams()
    lib().eclqr_ipm_default_params(C.byref(prm))
    return {f: getattr(prm, f) for f, _ in _lib.IpmParams._fields_}


def ipm_workspace(plan: Plan, device="cuda") -> torch.Tensor:
    n = C.c_size_t()
    check(lib().eclqr_ipm_workspace_size(plan.handle, C.byref(n)), "eclqr_ipm_workspace_size")
    return torch.empty(n.value + 256, dtype=torch.uint8, device=device)


def ipm_solve(plan: Plan, data: Dict[str, torch.Tensor], bounds: Dict[str, Optional[torch.Tensor]],
              ws: Optional[torch.Tensor] = None, out: Optional[IpmSolution] = None, **params) -> IpmSolution:
    """eclqr_ipm_solve on the current stream (asynchronous).  bounds: device
    tensors u_lo, u_hi (layout of r), x_lo, x_hi (layout of q), any of them
    absent or None; params override eclqr_ipm_default_params."""
    device = data["Q"].device
    if ws is None:
        ws = ipm_workspace(plan, device)
    prm = _lib.IpmParams()
    lib().eclqr_ipm_default_params(C.byref(prm))
    for k, v in params.items():
        if k not in dict(_lib.IpmParams._fields_):
            raise TypeError(f"unknown interior-point parameter {k}")
        setattr(prm, k, v)
    if out is None:
        _, nq = plan.layout("q")
        _, nr = plan.layout("r")
        _, ng = plan.layout("g")
        mk = lambda n: torch.empty(max(1, n), dtype=torch.float64, device=device)  # noqa: E731
        out = IpmSolution(mk(nq), mk(nr), mk(nq), mk(ng), mk(nr), mk(nr), mk(nq), mk(nq),
                          torch.empty(plan.batch, dtype=torch.float64, device=device),
                          torch.empty(plan.batch, dtype=torch.int32, device=device),
                          torch.empty(plan.batch, dtype=torch.int32, device=device))
    bp = _lib.BoundPtrs()
    for f in ("u_lo", "u_hi", "x_lo", "x_hi"):
        t = bounds.get(f)
        if t is not None and t.dtype != torch.float64:
            raise TypeError(f"bound {f} must be float64")
        setattr(bp, f, t.data_ptr() if t is not None else None)
    pp = _problem_ptrs(data)
    sp = out.ptrs()
    wptr, wbytes = _aligned_ws(ws)
    check(lib().eclqr_ipm_solve(plan.handle, C.byref(pp), C.byref(bp), C.byref(prm), C.byref(sp), C.c_void_p(wptr),
                                C.c_size_t(wbytes), _stream()), "eclqr_ipm_solve")
    out._ws = ws
    return out


def backward(plan: Plan, data: Dict[str, torch.Tensor], sol: Solution, dx: torch.Tensor, du: torch.Tensor,
             ws: torch.Tensor, dlam: Optional[torch.Tensor] = None,
             dmu: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
    """eclqr_backward: gradients of a loss L(x, u, lam, mu) given dL/dx, dL/du
    and optionally dL/dlam, dL/dmu.  ``grads["status"]`` holds the per-instance
    outcome (ECLQR_NOT_DIFFERENTIABLE where the constraint rows are dependent;
    the gradients of a flagged instance are NaN)."""
    device = dx.device
    grads = {f: torch.empty(max(1, plan.layout(f)[1]), dtype=torch.float64, device=device)
             for f in FIELDS if f != "M" or "M" in data}
    grads["status"] = torch.empty(plan.batch, dtype=torch.int32, device=device)
    gp = _lib.GradPtrs()
    for f in FIELDS + ("status",):
        setattr(gp, f, grads[f].data_ptr() if f in grads else None)
    sp = sol.ptrs()
    ct = _lib.CotangentPtrs(dx.data_ptr(), du.data_ptr(), dlam.data_ptr() if dlam is not None else None,
                            dmu.data_ptr() if dmu is not None else None)
    pp = _problem_ptrs(data)
    wptr, wbytes = _aligned_ws(ws)
    check(lib().eclqr_backward(plan.handle, C.byref(pp), C.byref(sp), C.byref(ct), C.byref(gp), C.c_void_p(wptr),
                               C.c_size_t(wbytes), _stream()), "eclqr_backward")
    return grads


def kkt_residual(plan: Plan, data: Dict[str, torch.Tensor], sol: Solution, ws: torch.Tensor) -> torch.Tensor:
    out = torch.empty(4 * plan.batch, dtype=torch.float64, device=sol.x.device)
    sp = sol.ptrs()
    pp = _problem_ptrs(data)
    wptr, wbytes = _aligned_ws(ws)
    check(lib().eclqr_kkt_residual(plan.handle, C.byref(pp), C.byref(sp), C.c_void_p(out.data_ptr()),
                                   C.c_void_p(wptr), C.c_size_t(wbytes), _stream()), "eclqr_kkt_residual")
    return out.view(plan.batch, 4)


def unpack(plan: Plan, flat: torch.Tensor, field: str, problems) -> List[List[np.ndarray]]:
    """Split a flat output (layout of ``field``: 'q' for x/lam, 'r' for u, 'g' for mu)
    into per-instance lists of per-stage vectors."""
    arr = flat.detach().cpu().numpy()
    offs, _ = plan.layout(field)
    out, s = [], 0
    for p in problems:
        sizes = {"q": p.nx, "r": p.nu, "g": p.nc}[field]
        blocks = []
        for i, n in enumerate(sizes):
            o = int(offs[s + i])
            blocks.append(arr[o:o + n].copy())
        out.append(blocks)
        s += p.N + 1
    return out


def _tuning_dict(t: _lib.Tuning) -> Dict[str, float]:
    return {"use_graph": int(t.use_graph), "level_buckets": int(t.level_buckets), "pool_in_lds": int(t.pool_in_lds),
            "grid_divisor": int(t.grid_divisor), "register_compose": int(t.register_compose),
            "stage_lds": int(t.stage_lds), "overlap_dual": int(t.overlap_dual), "multiplier_route": int(t.multiplier_route),
            "split_combine": int(t.split_combine), "fused_scans": int(t.fused_scans),
            "refine_gate": int(t.refine_gate),
            "ms_per_solve": float(t.ms_per_solve)}


def autotune(plan: Plan, data: Dict[str, torch.Tensor], ws: torch.Tensor, out: Optional[Solution] = None) -> Dict:
    """eclqr_plan_autotune on the current stream (synchronous): times the
    problem under alternative launch configurations and keeps the fastest."""
    if out is None:
        out = allocate_solution(plan, data["Q"].device, bool(plan.options.multipliers))
    sp = out.ptrs()
    pp = _problem_ptrs(data)
    wptr, wbytes = _aligned_ws(ws)
    t = _lib.Tuning()
    check(lib().eclqr_plan_autotune(plan.handle, C.byref(pp), C.byref(sp), C.c_void_p(wptr), C.c_size_t(wbytes),
                                    _stream(), C.byref(t)), "eclqr_plan_autotune")
    return _tuning_dict(t)


def get_tuning(plan: Plan) -> Dict:
    t = _lib.Tuning()
    check(lib().eclqr_plan_get_tuning(plan.handle, C.byref(t)), "eclqr_plan_get_tuning")
    return _tuning_dict(t)


def set_tuning(plan: Plan, **kw) -> None:
    t = _lib.Tuning()
    check(lib().eclqr_plan_get_tuning(plan.handle, C.byref(t)), "eclqr_plan_get_tuning")
    for k, v in kw.items():
        if not hasattr(t, k):
            raise KeyError(k)
        setattr(t, k, v)
    check(lib().eclqr_plan_set_tuning(plan.handle, C.byref(t)), "eclqr_plan_set_tuning")
