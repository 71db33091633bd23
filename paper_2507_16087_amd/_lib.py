"""ctypes declarations of the C ABI in include/cbs.h.

Loads the in-tree ``libcbs.so``; there is no fallback: if the library is
missing or does not load, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcbs.so")

CBS_OK = 0
CBS_NOT_CONVERGED = 1
CBS_E_INVALID = -1
CBS_E_UNSUPPORTED = -2
CBS_E_NOMEM = -3
CBS_E_DEVICE = -4
CBS_E_DIVERGED = -5
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "E_INVALID", -2: "E_UNSUPPORTED", -3: "E_NOMEM",
                -4: "E_DEVICE", -5: "E_DIVERGED"}

CBS_FP64 = 0
CBS_FP32_REFINED = 1
CBS_PTR_HOST = 0
CBS_PTR_DEVICE = 1
CBS_RHS_PHYSICAL = 0
CBS_RHS_EQUATION = 1
CBS_STOP_UPDATE = 0
CBS_STOP_RESIDUAL = 1
CBS_NOALLOC_SCRATCH_BYTES = 64 << 20

# every entry point declared in include/cbs.h
EXPORTS = [
    "cbs_create_medium", "cbs_destroy_medium", "cbs_medium_scalars", "cbs_plan_scalars", "cbs_set_scalars",
    "cbs_workspace_bytes", "cbs_solve", "cbs_solve_adjoint", "cbs_residual", "cbs_gradient",
    "cbs_pass_config", "cbs_pass_timing", "cbs_pass_timing_slots", "cbs_pass_timing_read",
    "cbs_batch_workspace_bytes", "cbs_batch_create", "cbs_batch_destroy", "cbs_batch_submit",
    "cbs_batch_step", "cbs_batch_retire", "cbs_residual_noalloc", "cbs_split_workspace_bytes",
    "cbs_solve_split", "cbs_stream_probe",
]


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int64 * 3), ("dx", C.c_double),
                ("omega", C.c_double), ("pml_cells", C.c_int32), ("pml_gamma_max", C.c_double),
                ("beta", C.c_double), ("nu", C.c_double), ("shift_rule", C.c_int32),
                ("collocated", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("prec", C.c_int32),
                ("check_every", C.c_int32), ("inner_tol", C.c_double), ("rhs_kind", C.c_int32),
                ("ptr_kind", C.c_int32), ("stop_rule", C.c_int32), ("max_outer", C.c_int32),
                ("max_inner", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("outer", C.c_int32), ("status", C.c_int32),
                ("rel_update", C.c_double), ("rel_residual", C.c_double),
                ("seconds", C.c_double), ("residual_evals", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2507_16087_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
    L.cbs_create_medium.argtypes = [C.POINTER(Grid), vp, vp, vp, i32, vp, C.POINTER(vp)]
    L.cbs_destroy_medium.argtypes = [vp]
    L.cbs_medium_scalars.argtypes = [vp, dp]
    L.cbs_plan_scalars.argtypes = [C.POINTER(Grid), vp, vp, vp, dp]
    L.cbs_set_scalars.argtypes = [vp, dp]
    L.cbs_workspace_bytes.argtypes = [vp, i32, i32, C.POINTER(C.c_size_t)]
    solve_args = [vp, vp, vp, C.POINTER(SolveOpts), vp, vp, vp, C.c_size_t, C.POINTER(SolveInfo), vp]
    L.cbs_solve.argtypes = solve_args
    L.cbs_solve_adjoint.argtypes = solve_args
    L.cbs_residual.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, dp, vp, vp, vp, C.c_size_t, vp]
    L.cbs_split_workspace_bytes.argtypes = [vp, i32, i32, C.POINTER(C.c_size_t)]
    L.cbs_solve_split.argtypes = [vp, i32, vp, vp, C.POINTER(SolveOpts), vp, vp, vp, C.c_size_t,
                                  C.POINTER(SolveInfo), vp]
    L.cbs_residual_noalloc.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, dp, vp, vp, vp]
    L.cbs_gradient.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp]
    L.cbs_pass_config.argtypes = [vp, i32, C.POINTER(C.c_int32)]
    L.cbs_pass_timing.argtypes = [vp, i32]
    L.cbs_pass_timing_slots.argtypes = [vp, i32]
    L.cbs_pass_timing_read.argtypes = [vp, dp, C.POINTER(C.c_int64)]
    L.cbs_stream_probe.argtypes = [vp, vp, C.c_size_t, i32, dp, vp]
    L.cbs_batch_workspace_bytes.argtypes = [C.POINTER(Grid), i32, i32, C.POINTER(C.c_size_t)]
    L.cbs_batch_create.argtypes = [C.POINTER(Grid), i32, i32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.cbs_batch_destroy.argtypes = [vp]
    L.cbs_batch_submit.argtypes = [vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(i32)]
    L.cbs_batch_step.argtypes = [vp, i32, C.POINTER(C.c_uint8)]
    L.cbs_batch_retire.argtypes = [vp, i32, vp, vp, i32, C.POINTER(SolveInfo)]
    for name in EXPORTS:
        getattr(L, name).restype = C.c_int
    _LIB = L
    return L


class CbsError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")
        self.status = status


def check(status: int, what: str, allow=(CBS_OK,)) -> int:
    if status not in allow:
        raise CbsError(status, what)
    return status
