"""ctypes declarations of the C ABI in ``include/eclqr.h`` (argument
marshalling only).  Loading fails loudly when ``libeclqr.so`` is missing:
there is no fallback path."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeclqr.so")

NUM_FIELDS = 12
FIELDS = ("Q", "q", "R", "r", "M", "A", "B", "c", "E", "F", "g", "x0")
FIELD_INDEX = {f: i for i, f in enumerate(FIELDS)}

NUM_KERNEL_CLASSES = 17

STATUS_BITS = {
    1: "infeasible_suffix",
    2: "infeasible_initial",
    4: "rank_inconsistent",
    8: "not_convex",
    16: "invalid_input",
    32: "capacity",
    64: "dual_failed",
    128: "not_differentiable",
    1 << 16: "timeout",
    1 << 17: "no_minimizer",
    1 << 18: "not_unique",
}


class Dims(C.Structure):
    _fields_ = [("batch", C.c_int32), ("horizon", C.POINTER(C.c_int32)), ("nx", C.POINTER(C.c_int32)),
                ("nu", C.POINTER(C.c_int32)), ("nc", C.POINTER(C.c_int32))]


class Options(C.Structure):
    _fields_ = [("rank_tol", C.c_double), ("cons_tol", C.c_double), ("dual_cons_tol", C.c_double),
                ("refine_tol", C.c_double), ("accept_tol", C.c_double), ("multipliers", C.c_int32), ("refine", C.c_int32), ("use_graph", C.c_int32),
                ("scan_schedule", C.c_int32), ("reversed_time", C.c_int32), ("domain_shortcut", C.c_int32),
                ("reserved", C.c_int32 * 2)]


class Tuning(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("level_buckets", C.c_int32), ("pool_in_lds", C.c_int32),
                ("grid_divisor", C.c_int32), ("ms_per_solve", C.c_double), ("register_compose", C.c_int32),
                ("stage_lds", C.c_int32), ("overlap_dual", C.c_int32), ("multiplier_route", C.c_int32),
                ("split_combine", C.c_int32), ("fused_scans", C.c_int32), ("refine_gate", C.c_int32)]


class ProblemPtrs(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in FIELDS]


class SolutionPtrs(C.Structure):
    _fields_ = [("x", C.c_void_p), ("u", C.c_void_p), ("lam", C.c_void_p), ("mu", C.c_void_p),
                ("status", C.c_void_p), ("info", C.c_void_p)]


class CotangentPtrs(C.Structure):
    _fields_ = [("dx", C.c_void_p), ("du", C.c_void_p), ("dlam", C.c_void_p), ("dmu", C.c_void_p)]


class GradPtrs(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in FIELDS] + [("status", C.c_void_p)]


class BoundPtrs(C.Structure):
    _fields_ = [("u_lo", C.c_void_p), ("u_hi", C.c_void_p), ("x_lo", C.c_void_p), ("x_hi", C.c_void_p)]


class IpmParams(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("mu_stop", C.c_double), ("tau", C.c_double), ("mu0", C.c_double),
                ("interior", C.c_double), ("corrector_replay", C.c_int32), ("newton_refine", C.c_int32)]


class IpmSolutionPtrs(C.Structure):
    _fields_ = [("x", C.c_void_p), ("u", C.c_void_p), ("lam", C.c_void_p), ("mu", C.c_void_p),
                ("z_ulo", C.c_void_p), ("z_uhi", C.c_void_p), ("z_xlo", C.c_void_p), ("z_xhi", C.c_void_p),
                ("comp", C.c_void_p), ("steps", C.c_void_p), ("status", C.c_void_p)]


_lib = None


def lib():
    """The loaded ``libeclqr.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2407_05433_amd.build`")
    L = C.CDLL(LIB_PATH)
    L.eclqr_abi_version.restype = C.c_int
    L.eclqr_default_options.argtypes = [C.POINTER(Options)]
    L.eclqr_status_string.restype = C.c_char_p
    L.eclqr_status_string.argtypes = [C.c_int32]
    L.eclqr_last_error.restype = C.c_char_p
    L.eclqr_plan_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(Dims), C.POINTER(Options)]
    L.eclqr_plan_destroy.argtypes = [C.c_void_p]
    L.eclqr_plan_destroy.restype = None
    L.eclqr_plan_layout.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.POINTER(C.c_int64)), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)]
    L.eclqr_plan_workspace_size.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
    L.eclqr_plan_schedule.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                      C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.c_int32)]
    L.eclqr_solve.argtypes = [C.c_void_p, C.POINTER(ProblemPtrs), C.POINTER(SolutionPtrs), C.c_void_p, C.c_size_t,
                              C.c_void_p]
    L.eclqr_solve_noalloc.argtypes = [C.c_void_p, C.POINTER(ProblemPtrs), C.POINTER(SolutionPtrs), C.c_void_p]
    L.eclqr_solve_noalloc.restype = C.c_int
    L.eclqr_backward.argtypes = [C.c_void_p, C.POINTER(ProblemPtrs), C.POINTER(SolutionPtrs),
                                 C.POINTER(CotangentPtrs), C.POINTER(GradPtrs), C.c_void_p, C.c_size_t, C.c_void_p]
    L.eclqr_kkt_residual.argtypes = [C.c_void_p, C.POINTER(ProblemPtrs), C.POINTER(SolutionPtrs), C.c_void_p,
                                     C.c_void_p, C.c_size_t, C.c_void_p]
    L.eclqr_plan_set_profiling.argtypes = [C.c_void_p, C.c_int32]
    L.eclqr_plan_set_graph.argtypes = [C.c_void_p, C.c_int32]
    L.eclqr_plan_autotune.argtypes = [C.c_void_p, C.POINTER(ProblemPtrs), C.POINTER(SolutionPtrs), C.c_void_p,
                                      C.c_size_t, C.c_void_p, C.POINTER(Tuning)]
    L.eclqr_plan_get_tuning.argtypes = [C.c_void_p, C.POINTER(Tuning)]
    L.eclqr_plan_set_tuning.argtypes = [C.c_void_p, C.POINTER(Tuning)]
    for fn in ("eclqr_plan_autotune", "eclqr_plan_get_tuning", "eclqr_plan_set_tuning"):
        getattr(L, fn).restype = C.c_int
    L.eclqr_plan_set_graph.restype = C.c_int
    L.eclqr_plan_profile.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
    L.eclqr_kernel_class_name.restype = C.c_char_p
    L.eclqr_kernel_class_name.argtypes = [C.c_int32]
    L.eclqr_plan_reduced_dims.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32)]
    L.eclqr_plan_combine_forms.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32)]
    L.eclqr_plan_combine_forms.restype = C.c_int
    L.eclqr_plan_scan_rows.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]
    L.eclqr_plan_refine_steps.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]
    L.eclqr_plan_refine_steps.restype = C.c_int
    L.eclqr_plan_backward_error.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
    L.eclqr_plan_backward_error.restype = C.c_int
    L.eclqr_plan_scan_rows.restype = C.c_int
    L.eclqr_plan_slot_info.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.eclqr_plan_slot_info.restype = C.c_int
    L.eclqr_plan_footprint.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]
    L.eclqr_plan_footprint.restype = C.c_int
    L.eclqr_ipm_default_params.argtypes = [C.POINTER(IpmParams)]
    L.eclqr_ipm_default_params.restype = None
    L.eclqr_ipm_workspace_size.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
    L.eclqr_ipm_workspace_size.restype = C.c_int
    L.eclqr_ipm_solve.argtypes = [C.c_void_p, C.POINTER(ProblemPtrs), C.POINTER(BoundPtrs), C.POINTER(IpmParams),
                                  C.POINTER(IpmSolutionPtrs), C.c_void_p, C.c_size_t, C.c_void_p]
    L.eclqr_ipm_solve.restype = C.c_int
    for fn in ("eclqr_plan_create", "eclqr_plan_layout", "eclqr_plan_workspace_size", "eclqr_plan_schedule",
               "eclqr_solve", "eclqr_backward", "eclqr_kkt_residual", "eclqr_plan_set_profiling",
               "eclqr_plan_profile", "eclqr_plan_reduced_dims"):
        getattr(L, fn).restype = C.c_int
    _lib = L
    return L


class EclqrError(RuntimeError):
    pass


def check(code: int, what: str) -> None:
    if code != 0:
        msg = lib().eclqr_last_error().decode()
        raise EclqrError(f"{what} failed (status {code}): {msg}")


def status_names(code: int):
    if code == 0:
        return ["ok"]
    out = [name for bit, name in STATUS_BITS.items() if code & bit]
    out += ["dual:" + name for bit, name in STATUS_BITS.items() if bit < 256 and (code >> 8) & bit]
    return out
