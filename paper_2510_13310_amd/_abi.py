"""ctypes view of the C ABI in include/ba.h (structures, prototypes, status codes).

Only argument marshalling lives here; every step of the computation runs in the HIP library.
Loading fails loudly if ``libinstantba.so`` has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char, c_char_p, c_double, c_int32, c_int64,
                    c_uint8, c_void_p)

LIB_NAME = "libinstantba.so"
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), LIB_NAME)

BA_OK = 0
BA_EMPTY = 1
BA_NOT_CONVERGED = 2
BA_ERR_ARG = -1
BA_ERR_STATE = -2
BA_ERR_OOM = -3
BA_ERR_DEVICE = -4
BA_ERR_NUMERIC = -5
STATUS_NAMES = {0: "BA_OK", 1: "BA_EMPTY", 2: "BA_NOT_CONVERGED", -1: "BA_ERR_ARG",
                -2: "BA_ERR_STATE", -3: "BA_ERR_OOM", -4: "BA_ERR_DEVICE", -5: "BA_ERR_NUMERIC"}

BA_PRECISION_FP64 = 0
BA_PRECISION_MIXED = 1
BA_ACTIVITY_ROWS = 0
BA_ACTIVITY_LITERAL = 1
BA_ADJOINT_FULL = 0
BA_ADJOINT_GAUSS_NEWTON = 1


class BaOptions(Structure):
    _fields_ = [
        ("precision", c_int32), ("img_w", c_int32), ("img_h", c_int32),
        ("activity_rule", c_int32), ("min_depth", c_double), ("huber_px", c_double),
        ("filter_px", c_double), ("lambda_init", c_double), ("lambda_min", c_double),
        ("lambda_max", c_double), ("diag_min", c_double), ("diag_max", c_double),
        ("accept_ratio", c_double), ("pcg_max_iters", c_int32), ("pcg_check_every", c_int32),
        ("pcg_rel_tol", c_double), ("cost_rel_tol", c_double), ("grad_tol", c_double),
        ("max_lm_iters", c_int32), ("timing", c_int32), ("adjoint_max_iters", c_int32),
        ("solver", c_int32), ("refine_focal", c_int32), ("adjoint_hessian", c_int32),
        ("adjoint_rel_tol", c_double), ("adjoint_damping", c_double), ("gp_huber", c_double),
        ("hip_stream", c_void_p),
    ]


class BaStepReport(Structure):
    _fields_ = [
        ("status", c_int32), ("accepted", c_int32), ("relinearized", c_int32),
        ("fixpoint_rounds", c_int32), ("pcg_iters", c_int32), ("pcg_breakdown", c_int32),
        ("n_cams_active", c_int32), ("n_points_active", c_int32), ("n_obs_active", c_int64),
        ("cost_before", c_double), ("cost_after", c_double), ("model_decrease", c_double),
        ("gain_ratio", c_double), ("lambda_", c_double), ("pcg_rel_residual", c_double),
        ("rms_px", c_double), ("grad_inf", c_double), ("ms_extract", c_double),
        ("ms_linearize", c_double), ("ms_setup", c_double), ("ms_pcg", c_double),
        ("ms_candidate", c_double), ("ms_total", c_double), ("pcg_true_residual", c_double),
    ]


class BaSolveReport(Structure):
    _fields_ = [
        ("iterations", c_int32), ("accepted", c_int32), ("stop_reason", c_int32),
        ("total_pcg_iters", c_int64), ("initial_cost", c_double), ("final_cost", c_double),
        ("initial_rms_px", c_double), ("final_rms_px", c_double), ("lambda_", c_double),
        ("ms_total", c_double),
    ]


class BaKernelStat(Structure):
    _fields_ = [("name", c_char * 32), ("launches", c_int64), ("total_ms", c_double),
                ("total_bytes", c_double)]


def struct_to_dict(s: Structure) -> dict:
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        out[name.rstrip("_")] = v.decode() if isinstance(v, bytes) else v
    return out


EXPORTS = {
    "ba_default_options": (None, [POINTER(BaOptions)]),
    "ba_create": (c_int32, [POINTER(BaOptions), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                            POINTER(c_void_p)]),
    "ba_set_observations": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "ba_set_depth_priors": (c_int32, [c_void_p, c_void_p, c_void_p, c_double]),
    "ba_set_fixed_cameras": (c_int32, [c_void_p, c_int32, c_void_p]),
    "ba_lm_step": (c_int32, [c_void_p, POINTER(BaStepReport)]),
    "ba_lm_step_noalloc": (c_int32, [c_void_p, POINTER(BaStepReport)]),
    "ba_solve": (c_int32, [c_void_p, POINTER(BaSolveReport)]),
    "ba_get_params": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ba_set_params": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ba_get_intrinsics": (c_int32, [c_void_p, c_void_p]),
    "ba_gp_step": (c_int32, [c_void_p, POINTER(BaStepReport)]),
    "ba_gp_solve": (c_int32, [c_void_p, POINTER(BaSolveReport)]),
    "ba_gp_get_scales": (c_int32, [c_void_p, c_void_p]),
    "ba_gp_reset": (c_int32, [c_void_p]),
    "ba_get_active": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ba_get_last_step": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ba_get_normal_blocks": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ba_get_preconditioner": (c_int32, [c_void_p, c_void_p]),
    "ba_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ba_kernel_stats": (c_int32, [c_void_p, POINTER(BaKernelStat), c_int32, POINTER(c_int32)]),
    "ba_reset_kernel_stats": (c_int32, [c_void_p]),
    "ba_device_bytes": (c_int64, [c_void_p]),
    "ba_last_error": (c_char_p, [c_void_p]),
    "ba_destroy": (None, [c_void_p]),
}

_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the HIP library once; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(
            f"{p} not found: the gfx950 HIP library must be built first "
            "(python -m paper_2510_13310_amd.build, or __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class BAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
