"""CPU checks of the C ABI library: it loads, exports every function that
include/eclqr.h declares, validates arguments, lays out the caller's fields in
stage order, and its associative-scan schedule computes the right suffix
relations (replayed here with the oracle's composition on the CPU)."""

from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2407_05433_amd as ecl
from paper_2407_05433_amd import _lib
from workloads import config_c0, config_c3
from tests._util import tiny_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eclqr.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eclqr_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert L.eclqr_abi_version() == 3


def test_status_strings_and_defaults():
    L = _lib.lib()
    assert L.eclqr_status_string(0) == b"ok"
    assert L.eclqr_status_string(2) == b"infeasible_initial"
    o = ecl.default_options()
    assert o.rank_tol == 1e-10 and o.cons_tol == 1e-8 and o.multipliers == 1 and o.refine == 2 and o.refine_tol == 1e-8
    assert o.domain_shortcut == 1 and o.reversed_time == 0 and o.scan_schedule == 0


def test_plan_rejects_bad_options():
    dims = [([3, 3, 3], [2, 2], [1, 1, 0])]
    for bad in ({"domain_shortcut": 2}, {"domain_shortcut": -1}, {"multipliers": 4}, {"refine": 5},
                {"scan_schedule": 3}):
        with pytest.raises(ecl.EclqrError):
            ecl.Plan(dims, **bad)
    for ok in ({"domain_shortcut": 0}, {"domain_shortcut": 1}):
        ecl.Plan(dims, **ok)


def test_plan_rejects_bad_dims():
    with pytest.raises(ecl.EclqrError):
        ecl.Plan([([3], [], [0])])  # N = 0
    with pytest.raises(ecl.EclqrError):
        ecl.Plan([([3, 65], [2], [0, 0])])  # dimension above the kernel limit
    with pytest.raises(ValueError):
        ecl.Plan([([3, 3, 3], [2], [0, 0])])


def test_layout_is_stage_order_concatenation():
    probs = [tiny_problem(700 + s, nx=[2, 3, 4, 3], nu=[1, 2, 3], terminal_rows=1) for s in range(3)]
    plan = ecl.Plan.for_problems(probs)
    for f in ("Q", "q", "R", "r", "A", "B", "c", "E", "F", "g"):
        offs, tot = plan.layout(f)
        sizes = [a.size for p in probs for a in getattr(p, f)]
        assert tot == sum(sizes)
        # offsets of the present blocks are the running sums
        run, k = 0, 0
        for p in probs:
            n_blocks = len(getattr(p, f))
            for i in range(p.N + 1):
                if i < n_blocks:
                    assert offs[k + i] == run
                    run += getattr(p, f)[i].size
            k += p.N + 1
    offs, tot = plan.layout("x0")
    assert list(offs) == [0, 2, 4] and tot == 6
    assert plan.workspace_bytes > 0


def _replay_schedule(plan, problem):
    """Run the plan's task list with the oracle's composition; return the
    suffix relation of every leaf."""
    from oracle.relations import base_relation, compose, terminal_relation
    N = problem.N
    rel = {}
    for i in range(N):
        rel[i] = base_relation(problem.A[i], problem.B[i], problem.c[i], problem.E[i], problem.F[i], problem.g[i])
    rel[N] = terminal_relation(problem.E[N], problem.g[N])
    levels = plan.schedule()
    D = len(levels) // 2
    for lv in levels:
        for a, b, o in lv:
            rel[int(o)] = compose(rel[int(a)], rel[int(b)])
    return rel, levels, D


@pytest.mark.parametrize("schedule", [1, 2])
@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 13, 16])
def test_schedule_reproduces_sequential_suffixes(N, schedule):
    """Both parenthesizations (balanced up/down sweep, recursive doubling)
    compose the oracle's base relations into the sequential suffixes
    (Proposition 1)."""
    from oracle import solve_sequential
    from oracle.relations import same_set
    p = tiny_problem(800 + N, N=N, n=3, m=1, kinds=[["state"]] * N, terminal_rows=2)
    plan = ecl.Plan.for_problems([p], scan_schedule=schedule)
    rel, levels, D = _replay_schedule(plan, p)
    assert D == max(1, int(np.ceil(np.log2(N + 1))))
    seq = solve_sequential(p, keep_relations=True)
    # every leaf's suffix slot must hold S_i; locate it through the stage table
    # (slots are leaves 0..N, then internal / suffix slots in allocation order)
    leaf_suffix = _leaf_suffix_slots(plan, N) if schedule == 1 else _doubling_suffix_slots(plan, N)
    for i in range(N + 1):
        assert same_set(rel[leaf_suffix[i]], seq.suffix[i], tol=1e-9), i
    if schedule == 2:
        L = N + 1
        assert all(len(lv) == 0 for lv in levels[D:])  # no down-sweep
        assert [len(lv) for lv in levels[:D]] == [L - 2 ** l for l in range(D)]


def _doubling_suffix_slots(plan, N):
    """Recursive doubling: the last output whose left operand starts at leaf
    i covers [i, L); the terminal leaf is its own suffix."""
    levels = plan.schedule()
    start = {i: i for i in range(N + 1)}
    suf = {i: i for i in range(N + 1)}
    for lv in levels:
        for a, b, o in lv:
            start[int(o)] = start[int(a)]
            suf[start[int(a)]] = int(o)
    return suf


def _leaf_suffix_slots(plan, N):
    """Recover suffix slot ids by re-deriving the down-sweep from the task lists:
    the output of a down task is the suffix of the leaf its left operand starts at."""
    levels = plan.schedule()
    D = len(levels) // 2
    start = {i: i for i in range(N + 1)}  # slot -> first leaf
    for lv in levels[:D]:
        for a, b, o in lv:
            start[int(o)] = start[int(a)]
    suf = {}
    # root: the last up task's output covers leaf 0
    root = int(levels[D - 1][-1][2]) if D else 0
    suf[0] = root
    for lv in levels[D:]:
        for a, b, o in lv:
            suf[start[int(a)]] = int(o)
    # leaves whose suffix aliases a node containing the terminal: their node is
    # the right child of a spine node, i.e. an up-sweep operand whose start is i
    for i in range(1, N + 1):
        if i not in suf:
            cands = [int(b) for lv in levels[:D] for a, b, o in lv if start[int(b)] == i]
            cands += [i] if i == N else []
            # the largest node starting at i that reaches the end
            suf[i] = max(cands) if cands else i
    return suf


def test_batched_schedule_levels_merge_instances():
    probs = [tiny_problem(900 + s, N=N, n=2, m=1, kinds=[[]] * N, terminal_rows=0) for s, N in
             enumerate([3, 17, 1, 64])]
    plan = ecl.Plan.for_problems(probs, scan_schedule=1, reversed_time=1)
    levels = plan.schedule()
    D = len(levels) // 2
    assert D == 7  # ceil(log2(65))
    total_up = sum(len(lv) for lv in levels[:D])
    assert total_up == sum(p.N for p in probs)  # L - 1 combines per instance
    # the reversed-time problem has one more stage per instance
    dlev = plan.schedule(dual=True)
    assert sum(len(lv) for lv in dlev[:len(dlev) // 2]) == sum(p.N + 1 for p in probs)


def test_c3_plan_builds_quickly():
    import time
    probs = config_c3(B=64)
    t = time.time()
    plan = ecl.Plan.for_problems(probs)
    assert time.time() - t < 5.0
    assert plan.batch == 64


def test_hybrid_schedule_reproduces_sequential_suffixes():
    """The automatic schedule on a batch of 2440 leaves: one balanced level,
    recursive doubling over the 1240 nodes left, one balanced down level; every
    leaf's suffix slot (the one slot covering [i, L) of its instance) holds the
    oracle's sequential suffix S_i."""
    from oracle import solve_sequential
    from oracle.relations import base_relation, compose, same_set, terminal_relation
    probs = [tiny_problem(1500 + s, N=60, n=3, m=1, kinds=[["state"]] * 60, terminal_rows=2) for s in range(40)]
    plan = ecl.Plan.for_problems(probs)
    inst, first, last = plan.slot_info()
    levels = plan.schedule()
    D = len(levels) // 2
    # one balanced level (1200 tasks), ceil(log2 31) = 5 doubling levels over the
    # 31 nodes per instance, one balanced down level
    assert [len(lv) for lv in levels] == [1200, 1200, 1160, 1080, 920, 600, 0, 0, 0, 0, 0, 1200]
    rel = {}
    leaf0 = {}
    for q in range(len(inst)):
        b, i, e = int(inst[q]), int(first[q]), int(last[q])
        if e == i + 1:
            p = probs[b]
            rel[q] = (base_relation(p.A[i], p.B[i], p.c[i], p.E[i], p.F[i], p.g[i]) if i < p.N
                      else terminal_relation(p.E[p.N], p.g[p.N]))
    for lv in levels:
        for a, bb, o in lv:
            rel[int(o)] = compose(rel[int(a)], rel[int(bb)])
    for b in (0, 17, 39):
        p = probs[b]
        seq = solve_sequential(p, keep_relations=True)
        for i in range(p.N + 1):
            q = [q for q in range(len(inst)) if inst[q] == b and first[q] == i and last[q] == p.N + 1]
            assert len(q) == 1, (b, i, q)
            assert same_set(rel[q[0]], seq.suffix[i], tol=1e-9), (b, i)


def test_route_decided_at_plan_creation_from_the_lds_bound():
    """Minimum-norm local systems whose tile exceeds 160 KiB of LDS (n = 64,
    m = 64, no rows) get the reversed-time route when the plan is made; a
    plan whose tiles fit keeps the theta route."""
    big = [([64] * 4, [64] * 3, [0] * 4)]
    assert ecl.get_tuning(ecl.Plan(big))["multiplier_route"] == 0
    small = [([12] * 4, [6] * 3, [2, 2, 2, 1])]
    assert ecl.get_tuning(ecl.Plan(small))["multiplier_route"] == 1


def test_tuning_defaults_and_ranges():
    """Launch configuration of a new plan (staged-operand combines, LDS work
    arrays for eliminations and gains) and the accepted range of each
    multi-valued field: pool_in_lds 0..3, stage_lds 0..2 (2: gains only)."""
    plan = ecl.Plan([([6] * 5, [3] * 4, [1] * 5)])
    t = ecl.get_tuning(plan)
    assert t["pool_in_lds"] == 3 and t["stage_lds"] == 1 and t["grid_divisor"] == 1 and t["refine_gate"] == 0
    for k, v in (("pool_in_lds", 0), ("pool_in_lds", 2), ("stage_lds", 2), ("stage_lds", 0), ("refine_gate", 1)):
        ecl.set_tuning(plan, **{k: v})
        assert ecl.get_tuning(plan)[k] == v
    for k, v in (("pool_in_lds", 4), ("pool_in_lds", -1), ("stage_lds", 3), ("grid_divisor", 0)):
        with pytest.raises(RuntimeError):
            ecl.set_tuning(plan, **{k: v})


def test_ctypes_structs_follow_the_header():
    """The ctypes mirrors of eclqr_solution, eclqr_cotangent and eclqr_grads
    list the header's fields in the header's order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)

    def fields(tag):
        body = re.search(r"typedef struct \{([^}]*)\}\s*" + tag + ";", text).group(1)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            names = decl.split(None, 1)[1] if not decl.startswith("const") else decl.split(None, 2)[2]
            out += [n.strip().lstrip("*") for n in names.split(",")]
        return out

    assert [f for f, _ in _lib.SolutionPtrs._fields_] == fields("eclqr_solution")
    assert [f for f, _ in _lib.CotangentPtrs._fields_] == fields("eclqr_cotangent")
    assert [f for f, _ in _lib.GradPtrs._fields_] == fields("eclqr_grads")


def test_contraction_expansion_option():
    """multipliers = 3 (the contraction-expansion route) is accepted and
    lays out its engine; 4 is refused."""
    dims = [([3, 3, 3, 3], [2, 2, 2], [1, 0, 1, 1])]
    p3 = ecl.Plan(dims, multipliers=3)
    p1 = ecl.Plan(dims, multipliers=1)
    assert p3.workspace_bytes > p1.workspace_bytes
    with pytest.raises(ecl.EclqrError):
        ecl.Plan(dims, multipliers=4)


def test_ipm_structs_defaults_and_argument_errors():
    """The interior-point entry points: ctypes mirrors in the header's order,
    the documented defaults, a workspace larger than the solve's, and the
    argument errors that are decided before any device work (a plan without
    multipliers, parameters out of range, missing outputs)."""
    import ctypes as C
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)

    def fields(tag):
        body = re.search(r"typedef struct \{([^}]*)\}\s*" + tag + ";", text).group(1)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if decl:
                names = decl.split(None, 1)[1] if not decl.startswith("const") else decl.split(None, 2)[2]
                out += [n.strip().lstrip("*") for n in names.split(",")]
        return out

    assert [f for f, _ in _lib.BoundPtrs._fields_] == fields("eclqr_bounds")
    assert [f for f, _ in _lib.IpmParams._fields_] == fields("eclqr_ipm_params")
    assert [f for f, _ in _lib.IpmSolutionPtrs._fields_] == fields("eclqr_ipm_solution")
    d = ecl.ipm_default_params()
    assert d == {"iterations": 30, "mu_stop": 1e-8, "tau": 0.995, "mu0": 100.0, "interior": 0.25, "corrector_replay": 1,
                 "newton_refine": 2}
    L = _lib.lib()
    dims = [([3, 3, 3, 3], [2, 2, 2], [1, 0, 1, 0])]
    plan = ecl.Plan(dims)
    n = C.c_size_t()
    assert L.eclqr_ipm_workspace_size(plan.handle, C.byref(n)) == 0
    assert n.value > plan.workspace_bytes
    fake_ws, big = C.c_void_p(1 << 20), C.c_size_t(1 << 40)  # never dereferenced: every case fails first
    pp, bp, sp = _lib.ProblemPtrs(), _lib.BoundPtrs(), _lib.IpmSolutionPtrs()

    def call(pl, **kw):
        prm = _lib.IpmParams()
        L.eclqr_ipm_default_params(C.byref(prm))
        for k, v in kw.items():
            setattr(prm, k, v)
        return L.eclqr_ipm_solve(pl.handle, C.byref(pp), C.byref(bp), C.byref(prm), C.byref(sp), fake_ws, big, None)

    assert call(ecl.Plan(dims, multipliers=0)) == 1
    assert b"multipliers" in L.eclqr_last_error()
    for bad in ({"tau": 1.0}, {"tau": 0.0}, {"mu0": 0.0}, {"interior": 0.5}, {"iterations": -1}, {"mu_stop": -1.0},
                {"newton_refine": 5}):
        assert call(plan, **bad) == 1, bad
    assert call(plan) == 1 and b"NULL output" in L.eclqr_last_error()
    assert L.eclqr_ipm_solve(plan.handle, C.byref(pp), C.byref(bp), None, C.byref(sp), fake_ws, big, None) == 1
    assert L.eclqr_ipm_solve(plan.handle, C.byref(pp), C.byref(bp), C.byref(_lib.IpmParams()), C.byref(sp), fake_ws,
                             C.c_size_t(16), None) == 2


def test_pack_bounds_layout():
    """Bounds land in the plan's layouts of r (inputs) and q (states), missing
    blocks and instances are infinite with the right sign, and a key no
    instance has is absent (None)."""
    import numpy as np
    from tests._util import tiny_problem
    probs = [tiny_problem(5, N=3, n=3, m=2, kinds=[["mixed"]] * 3, terminal_rows=0),
             tiny_problem(6, N=2, n=2, m=1, kinds=[[]] * 2, terminal_rows=1)]
    plan = ecl.Plan.for_problems(probs)
    b0 = {"u_lo": [np.full(2, -1.0 - i) for i in range(3)], "x_hi": [np.full(3, 10.0 + i) for i in range(4)]}
    out = ecl.pack_bounds(plan, probs, [b0, {}], device="cpu")
    assert out["u_hi"] is None and out["x_lo"] is None
    ulo, xhi = out["u_lo"].numpy(), out["x_hi"].numpy()
    offs, tot = plan.layout("r")
    assert ulo.size == tot
    for i in range(3):
        assert np.all(ulo[offs[i]:offs[i] + 2] == -1.0 - i)
    assert np.all(np.isneginf(ulo[offs[4]:offs[4] + 1])) and np.all(np.isneginf(ulo[offs[5]:offs[5] + 1]))
    offs, tot = plan.layout("q")
    assert xhi.size == tot
    for i in range(4):
        assert np.all(xhi[offs[i]:offs[i] + 3] == 10.0 + i)
    assert np.all(np.isposinf(xhi[offs[4]:]))
    with pytest.raises(ValueError):
        ecl.pack_bounds(plan, probs, [{"u_lo": [np.zeros(2)] * 2}, {}], device="cpu")
