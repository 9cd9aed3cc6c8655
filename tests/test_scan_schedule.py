"""CPU checks of the dependency order the persistent scan kernels rely on.

The persistent kernels take a scan's tasks in task-list order and let a task
start once every level before its own is complete.  That is correct and free
of deadlock when (1) the levels are contiguous, ordered ranges of the task
list, and (2) every operand slot of a task is a leaf (written before the scan
starts) or the output of a task in an earlier level.  Both are checked here on
the schedules of every parenthesization, single and batched, and the
scheduler itself is simulated with workgroups that take tasks in order and
finish them in random order.
"""

from __future__ import annotations

import functools

import numpy as np
import pytest

import paper_2407_05433_amd as ecl
from tests._util import problem_family, tiny_problem
from workloads import config_c1, config_c3


@functools.lru_cache(maxsize=1)
def _plans():
    fam = [p for _, p in problem_family()]
    out = []
    for sched in (0, 1, 2):
        out.append(("family", ecl.Plan.for_problems(fam, scan_schedule=sched)))
        out.append(("c1-300", ecl.Plan.for_problems(config_c1(N=300), scan_schedule=sched)))
        out.append(("c3-24", ecl.Plan.for_problems(config_c3(B=24, N_range=(32, 300)), scan_schedule=sched)))
        out.append(("N1", ecl.Plan.for_problems([tiny_problem(5, N=1, n=2, m=1, kinds=[[]], terminal_rows=0)],
                                                scan_schedule=sched)))
    return out


def _levels(plan):
    lv = [np.asarray(l) for l in plan.schedule()]
    return [l for l in lv if len(l)]


@pytest.mark.parametrize("idx", range(12))
def test_operands_come_from_earlier_levels(idx):
    name, plan = _plans()[idx]
    levels = _levels(plan)
    inst, first, last = plan.slot_info()
    produced_at = {}
    for k, lv in enumerate(levels):
        for a, b, o in lv:
            assert int(o) not in produced_at, (name, "slot written twice")
            produced_at[int(o)] = k
    outputs = set(produced_at)
    for k, lv in enumerate(levels):
        for a, b, o in lv:
            for operand in (int(a), int(b)):
                if operand in outputs:
                    assert produced_at[operand] < k, (name, k, operand)
                else:  # a leaf: one stage's own element, written before the scan
                    assert last[operand] - first[operand] <= 1 or last[operand] == first[operand] + 1, \
                        (name, operand)


def _simulate(levels, workgroups, rng):
    """Workgroups take tasks in list order; a taken task may finish only once
    every task of the earlier levels has finished.  Returns the number of
    finished tasks (all of them unless the scheme deadlocks)."""
    counts = [len(l) for l in levels]
    level_of = np.repeat(np.arange(len(levels)), counts)
    total = int(sum(counts))
    done = [0] * len(levels)
    nxt = 0
    held = []  # tasks taken and not finished
    finished = 0
    while finished < total:
        while len(held) < workgroups and nxt < total:
            held.append(nxt)
            nxt += 1
        ready = [t for t in held if all(done[j] == counts[j] for j in range(level_of[t]))]
        if not ready:
            return finished  # deadlock
        t = ready[int(rng.integers(len(ready)))]
        held.remove(t)
        done[level_of[t]] += 1
        finished += 1
    return finished


@pytest.mark.parametrize("workgroups", [1, 2, 7, 64])
def test_scheduler_simulation_never_deadlocks(workgroups):
    rng = np.random.default_rng(workgroups)
    for name, plan in _plans():
        levels = _levels(plan)
        total = sum(len(l) for l in levels)
        assert _simulate(levels, workgroups, rng) == total, name


def test_levels_are_contiguous_ranges():
    """Level l + 1's tasks start where level l's end in the plan's task list
    (the addresses eclqr_plan_schedule hands out)."""
    import ctypes as C
    from paper_2407_05433_amd._lib import lib
    for name, plan in _plans():
        nlev = C.c_int32()
        assert lib().eclqr_plan_schedule(plan.handle, 0, C.byref(nlev), -1, None, None) == 0
        assert nlev.value <= 64, name
        prev_end = None
        for level in range(nlev.value):
            ptr = C.POINTER(C.c_int32)()
            nt = C.c_int32()
            assert lib().eclqr_plan_schedule(plan.handle, 0, None, level, C.byref(ptr), C.byref(nt)) == 0
            addr = C.cast(ptr, C.c_void_p).value or 0
            if prev_end is not None and nt.value:
                assert addr == prev_end, (name, level)
            if nt.value:
                prev_end = addr + 3 * 4 * nt.value
