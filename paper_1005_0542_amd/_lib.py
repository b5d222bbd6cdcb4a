"""ctypes declarations of the C ABI in ``include/laguerre.h``.

Loading fails loudly (``RuntimeError``) when ``liblaguerre.so`` has not been
built: there is no CPU fallback anywhere in the package.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblaguerre.so")

LG_OK = 0
LG_ERR_INVALID_ARG = 1
LG_ERR_NOT_CONVERGED = 2
LG_ERR_BREAKDOWN = 3
LG_ERR_NONFINITE = 4
LG_ERR_HIP = 5
LG_ERR_OOM = 6
LG_ERR_UNSUPPORTED = 7

LG_FP64, LG_MIXED = 0, 1
LG_ACOUSTIC, LG_ELASTIC = 0, 1
LG_TOP_DIRICHLET, LG_TOP_FREE = 0, 1
LG_CARTESIAN, LG_CYLINDRICAL = 0, 1
LG_RICKER, LG_GAUSS_SINE = 0, 1
LG_SYNTH_BATCH_MAX = 8
LG_TRACE_SCRATCH_MAX = 1 << 21


class Grid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("nz", c_int32), ("dx", c_double), ("dz", c_double),
                ("top_bc", c_int32), ("geometry", c_int32), ("order", c_int32), ("reserved", c_int32)]


class Laguerre(ctypes.Structure):
    _fields_ = [("alpha", c_int32), ("h", c_double), ("n", c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("max_iter", c_int32), ("restart", c_int32), ("x0_given", c_int32),
                ("reserved", c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("status", c_int32), ("relres", c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("segments", c_int32), ("graph_iters", c_int32), ("op_shots", c_int32),
                ("seg_per_wave", c_int32), ("op_fusion", c_int32), ("x_ring", c_int32),
                ("reserved", c_int32 * 2)]


_PLAN = c_void_p
_SIGNATURES = {
    "lg_plan_create": [POINTER(c_void_p), c_int32, POINTER(Grid), POINTER(Laguerre), c_int32, c_int32,
                       POINTER(c_double), POINTER(Tuning), c_void_p],
    "lg_plan_destroy": [_PLAN],
    "lg_plan_set_stream": [_PLAN, c_void_p],
    "lg_plan_set_sources": [_PLAN, POINTER(c_int32)],
    "lg_plan_layout": [_PLAN, POINTER(c_int32), POINTER(c_int32)],
    "lg_plan_x_ring": [_PLAN, POINTER(c_int32)],
    "lg_source_coeffs": [c_int32, c_double, c_double, c_double, POINTER(Laguerre), POINTER(c_double)],
    "lg_laguerre_weights": [POINTER(Laguerre), POINTER(c_double), c_int32, POINTER(c_double)],
    "lg_status_string": [c_int32],
    "lg_last_error": [],
    "lg_laguerre_rhs": [_PLAN, c_int32, c_void_p, c_void_p, c_void_p, POINTER(c_double), c_void_p],
    "lg_stencil_apply": [_PLAN, c_void_p, c_void_p],
    "lg_precond_dst": [_PLAN, c_int32, c_void_p, c_void_p],
    "lg_precond_dichotomy_tdma": [_PLAN, c_int32, c_void_p, c_void_p],
    "lg_precond_apply": [_PLAN, c_void_p, c_void_p],
    "lg_pcg_solve": [_PLAN, c_void_p, c_void_p, POINTER(SolveOpts), POINTER(SolveInfo)],
    "lg_gmres_solve": [_PLAN, c_void_p, c_void_p, POINTER(SolveOpts), POINTER(SolveInfo)],
    "lg_laguerre_synthesize": [_PLAN, c_int32, c_void_p, POINTER(c_double), c_int32, c_void_p, c_int32,
                               c_void_p],
    "lg_laguerre_synthesize_batch": [_PLAN, c_int32, c_int32, POINTER(c_void_p), POINTER(c_double), c_int32,
                                     c_void_p, c_int32, c_void_p],
    "lg_trace_synthesize": [_PLAN, c_void_p, POINTER(c_double), c_int32, c_void_p],
    "lg_trace_synthesize_noalloc": [_PLAN, c_void_p, POINTER(c_double), c_int32, c_void_p],
    "lg_pcg_profile": [_PLAN, c_void_p, c_void_p, c_int32, POINTER(ctypes.c_float)],
}

_lib = None


def load() -> ctypes.CDLL:
    """Load ``liblaguerre.so`` (once) and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1005_0542_amd.build` "
            "(the HIP library is the only implementation; there is no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_char_p if name in ("lg_status_string", "lg_last_error") else c_int32
    _lib = lib
    return lib


class LgError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        self.status = status
        msg = lib.lg_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib.lg_status_string(status).decode()} ({status}): {msg}")


def check(status: int, where: str, allowed=(LG_OK,)) -> int:
    if status not in allowed:
        raise LgError(status, where)
    return status
