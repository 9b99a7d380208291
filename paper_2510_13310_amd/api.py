"""Python binding of the C ABI: functions with the ABI's names plus a small owning class.

Arrays may be NumPy arrays (host) or torch tensors (host or ``cuda:0``); their pointers are
passed straight through (the library accepts host or device memory). Torch supplies device
memory and the stream; it computes nothing here.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_int32, c_void_p

import numpy as np

from . import _abi
from ._abi import (BaOptions, BaStepReport, BaSolveReport, BaKernelStat, BAError,
                   struct_to_dict, BA_OK, BA_EMPTY)

try:  # torch is optional for the binding itself
    import torch
except Exception:  # pragma: no cover - torch is present in this image
    torch = None


def _ptr(a, dtype=None):
    """Raw pointer of a contiguous NumPy array / torch tensor (plus a keep-alive object)."""
    if a is None:
        return None, None
    if torch is not None and isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor arguments must be contiguous")
        if dtype is not None and a.dtype != dtype[1]:
            raise TypeError(f"expected {dtype[1]}, got {a.dtype}")
        return a.data_ptr(), a
    arr = np.ascontiguousarray(a, dtype=None if dtype is None else dtype[0])
    return arr.ctypes.data, arr


F64 = (np.float64, getattr(torch, "float64", None))
F32 = (np.float32, getattr(torch, "float32", None))
I32 = (np.int32, getattr(torch, "int32", None))
U8 = (np.uint8, getattr(torch, "uint8", None))


def _check(lib, ctx, status: int) -> int:
    if status < 0:
        msg = lib.ba_last_error(ctx)
        raise BAError(status, msg.decode() if msg else "")
    return status


# ---------------------------------------------------------------- ABI-named functions
def ba_default_options() -> BaOptions:
    o = BaOptions()
    _abi.load().ba_default_options(byref(o))
    return o


def ba_create(opts: BaOptions, n_cams: int, n_points: int, cams, intr, points) -> int:
    lib = _abi.load()
    pc, kc = _ptr(cams, F64)
    pi, ki = _ptr(intr, F64)
    pp, kp = _ptr(points, F64)
    h = c_void_p()
    st = lib.ba_create(byref(opts), n_cams, n_points, pc, pi, pp, byref(h))
    _check(lib, None, st)
    return h.value


def ba_set_observations(ctx: int, cam_idx, pt_idx, xy) -> int:
    lib = _abi.load()
    pc, kc = _ptr(cam_idx, I32)
    pp, kp = _ptr(pt_idx, I32)
    px, kx = _ptr(xy, F32)
    n = int(kc.shape[0])
    return _check(lib, ctx, lib.ba_set_observations(ctx, n, pc, pp, px))


def ba_set_depth_priors(ctx: int, depth, valid, lambda_d: float) -> int:
    lib = _abi.load()
    pd, kd = _ptr(depth, F32)
    pv, kv = _ptr(valid, U8)
    return _check(lib, ctx, lib.ba_set_depth_priors(ctx, pd, pv, float(lambda_d)))


def ba_set_fixed_cameras(ctx: int, cam_ids) -> int:
    lib = _abi.load()
    p, k = _ptr(cam_ids, I32)
    n = 0 if k is None else int(k.shape[0])
    return _check(lib, ctx, lib.ba_set_fixed_cameras(ctx, n, p))


def ba_lm_step(ctx: int) -> dict:
    lib = _abi.load()
    rep = BaStepReport()
    st = _check(lib, ctx, lib.ba_lm_step(ctx, byref(rep)))
    d = struct_to_dict(rep)
    d["status"] = st
    return d


def ba_lm_step_noalloc(ctx: int) -> dict:
    lib = _abi.load()
    rep = BaStepReport()
    st = _check(lib, ctx, lib.ba_lm_step_noalloc(ctx, byref(rep)))
    d = struct_to_dict(rep)
    d["status"] = st
    return d


def ba_solve(ctx: int) -> dict:
    lib = _abi.load()
    rep = BaSolveReport()
    st = _check(lib, ctx, lib.ba_solve(ctx, byref(rep)))
    d = struct_to_dict(rep)
    d["status"] = st
    return d


def ba_gp_step(ctx: int) -> dict:
    lib = _abi.load()
    rep = BaStepReport()
    st = _check(lib, ctx, lib.ba_gp_step(ctx, byref(rep)))
    d = struct_to_dict(rep)
    d["status"] = st
    return d


def ba_gp_solve(ctx: int) -> dict:
    lib = _abi.load()
    rep = BaSolveReport()
    st = _check(lib, ctx, lib.ba_gp_solve(ctx, byref(rep)))
    d = struct_to_dict(rep)
    d["status"] = st
    return d


def ba_gp_get_scales(ctx: int, scales_out) -> int:
    lib = _abi.load()
    ps, _ = _ptr(scales_out, F64)
    return _check(lib, ctx, lib.ba_gp_get_scales(ctx, ps))


def ba_gp_reset(ctx: int) -> int:
    lib = _abi.load()
    return _check(lib, ctx, lib.ba_gp_reset(ctx))


def ba_get_params(ctx: int, cams_out, points_out) -> int:
    lib = _abi.load()
    pc, _ = _ptr(cams_out, F64)
    pp, _ = _ptr(points_out, F64)
    return _check(lib, ctx, lib.ba_get_params(ctx, pc, pp))


def ba_get_intrinsics(ctx: int, intr_out) -> int:
    lib = _abi.load()
    pi, _ = _ptr(intr_out, F64)
    return _check(lib, ctx, lib.ba_get_intrinsics(ctx, pi))


def ba_set_params(ctx: int, cams, points) -> int:
    lib = _abi.load()
    pc, kc = _ptr(cams, F64)
    pp, kp = _ptr(points, F64)
    return _check(lib, ctx, lib.ba_set_params(ctx, pc, pp))


def ba_get_active(ctx: int, cams_out, points_out, obs_out) -> int:
    lib = _abi.load()
    a, _ = _ptr(cams_out, U8)
    b, _ = _ptr(points_out, U8)
    c, _ = _ptr(obs_out, U8)
    return _check(lib, ctx, lib.ba_get_active(ctx, a, b, c))


def ba_get_last_step(ctx: int, dcams_out, dpoints_out) -> int:
    lib = _abi.load()
    a, _ = _ptr(dcams_out, F64)
    b, _ = _ptr(dpoints_out, F64)
    return _check(lib, ctx, lib.ba_get_last_step(ctx, a, b))


def ba_get_normal_blocks(ctx: int, U_out, gc_out, V_out, gp_out) -> int:
    lib = _abi.load()
    ptrs = [_ptr(a, F64)[0] for a in (U_out, gc_out, V_out, gp_out)]
    return _check(lib, ctx, lib.ba_get_normal_blocks(ctx, *ptrs))


def ba_get_preconditioner(ctx: int, Minv_out) -> int:
    lib = _abi.load()
    p, _ = _ptr(Minv_out, F64)
    return _check(lib, ctx, lib.ba_get_preconditioner(ctx, p))


def ba_adjoint(ctx: int, grad_cams, grad_points, grad_xy_out, grad_depth_out) -> int:
    """Returns BA_OK, or BA_NOT_CONVERGED (with a warning) when the adjoint PCG stopped at its
    iteration cap above its tolerance; errors raise BAError."""
    lib = _abi.load()
    a, ka = _ptr(grad_cams, F64)
    b, kb = _ptr(grad_points, F64)
    c, _ = _ptr(grad_xy_out, F32)
    d, _ = _ptr(grad_depth_out, F32)
    st = _check(lib, ctx, lib.ba_adjoint(ctx, a, b, c, d))
    if st == _abi.BA_NOT_CONVERGED:
        import warnings
        warnings.warn("ba_adjoint: " + ba_last_error(ctx), RuntimeWarning, stacklevel=2)
    return st


def ba_kernel_stats(ctx: int, max_entries: int = 64) -> list:
    lib = _abi.load()
    arr = (BaKernelStat * max_entries)()
    n = c_int32(0)
    _check(lib, ctx, lib.ba_kernel_stats(ctx, arr, max_entries, byref(n)))
    return [struct_to_dict(arr[i]) for i in range(n.value)]


def ba_reset_kernel_stats(ctx: int) -> int:
    lib = _abi.load()
    return _check(lib, ctx, lib.ba_reset_kernel_stats(ctx))


def ba_device_bytes(ctx: int) -> int:
    return int(_abi.load().ba_device_bytes(ctx))


def ba_last_error(ctx: int | None) -> str:
    msg = _abi.load().ba_last_error(ctx)
    return msg.decode() if msg else ""


def ba_destroy(ctx: int) -> None:
    _abi.load().ba_destroy(ctx)


# ---------------------------------------------------------------- owning wrapper
_PRECISION = {"fp64": 0, "mixed": 1}
_RULE = {"rows": 0, "literal": 1}
_SOLVER = {"implicit": 0, "explicit": 1}
_ADJ_HESSIAN = {"full": 0, "gauss_newton": 1}


def make_options(precision="mixed", **kw) -> BaOptions:
    o = ba_default_options()
    o.precision = _PRECISION[precision] if isinstance(precision, str) else int(precision)
    if "activity_rule" in kw and isinstance(kw["activity_rule"], str):
        kw["activity_rule"] = _RULE[kw["activity_rule"]]
    if "solver" in kw and isinstance(kw["solver"], str):
        kw["solver"] = _SOLVER[kw["solver"]]
    if "adjoint_hessian" in kw and isinstance(kw["adjoint_hessian"], str):
        kw["adjoint_hessian"] = _ADJ_HESSIAN[kw["adjoint_hessian"]]
    if "stream" in kw:
        kw["hip_stream"] = kw.pop("stream")
    names = {f for f, _ in BaOptions._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown option {k!r}")
        setattr(o, k, v)
    return o


def current_torch_stream():
    """Handle of torch's current HIP stream (None when no GPU is usable)."""
    if torch is not None and torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


class BundleAdjuster:
    """Owns one ``ba_ctx``. Parameters follow include/ba.h: cams C x 7
    ``[qw, qx, qy, qz, cx, cy, cz]``, intr C x 3 ``[f, cx, cy]``, points P x 3."""

    def __init__(self, cams, intr, points, precision="mixed", use_torch_stream=True, **opts):
        if use_torch_stream and "stream" not in opts:
            opts["stream"] = current_torch_stream()
        self.opts = make_options(precision, **opts)
        self.n_cams = int(cams.shape[0])
        self.n_points = int(points.shape[0])
        self.cam_dim = 7 if self.opts.refine_focal else 6
        self.n_obs = 0
        self.ctx = ba_create(self.opts, self.n_cams, self.n_points, cams, intr, points)

    # lifetime
    def close(self):
        if getattr(self, "ctx", None):
            ba_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # inputs
    def set_observations(self, cam_idx, pt_idx, xy):
        self.n_obs = int(cam_idx.shape[0])
        return ba_set_observations(self.ctx, cam_idx, pt_idx, xy)

    def set_depth_priors(self, depth, valid=None, lambda_d=1.0):
        return ba_set_depth_priors(self.ctx, depth, valid, lambda_d)

    def set_fixed_cameras(self, cam_ids):
        return ba_set_fixed_cameras(self.ctx, cam_ids)

    # solve
    def lm_step(self) -> dict:
        return ba_lm_step(self.ctx)

    def lm_step_noalloc(self) -> dict:
        return ba_lm_step_noalloc(self.ctx)

    def solve(self) -> dict:
        return ba_solve(self.ctx)

    # depth-constrained global positioning
    def gp_step(self) -> dict:
        return ba_gp_step(self.ctx)

    def gp_solve(self) -> dict:
        return ba_gp_solve(self.ctx)

    def gp_scales(self):
        out = np.empty(self.n_obs)
        ba_gp_get_scales(self.ctx, out)
        return out

    def gp_reset(self):
        return ba_gp_reset(self.ctx)

    # outputs
    def get_params(self):
        cams = np.empty((self.n_cams, 7))
        pts = np.empty((self.n_points, 3))
        ba_get_params(self.ctx, cams, pts)
        return cams, pts

    def get_params_into(self, cams_out, points_out):
        ba_get_params(self.ctx, cams_out, points_out)

    def set_params(self, cams=None, points=None):
        return ba_set_params(self.ctx, cams, points)

    def get_intrinsics(self):
        intr = np.empty((self.n_cams, 3))
        ba_get_intrinsics(self.ctx, intr)
        return intr

    def get_active(self):
        c = np.empty(self.n_cams, np.uint8)
        p = np.empty(self.n_points, np.uint8)
        o = np.empty(self.n_obs, np.uint8)
        ba_get_active(self.ctx, c, p, o)
        return c.astype(bool), p.astype(bool), o.astype(bool)

    def get_last_step(self):
        dc = np.empty((self.n_cams, self.cam_dim))
        dp = np.empty((self.n_points, 3))
        ba_get_last_step(self.ctx, dc, dp)
        return dc, dp

    def get_normal_blocks(self):
        d = self.cam_dim
        U = np.empty((self.n_cams, d, d))
        gc = np.empty((self.n_cams, d))
        V = np.empty((self.n_points, 3, 3))
        gp = np.empty((self.n_points, 3))
        ba_get_normal_blocks(self.ctx, U, gc, V, gp)
        return U, gc, V, gp

    def get_preconditioner(self):
        d = self.cam_dim
        M = np.empty((self.n_cams, d, d))
        ba_get_preconditioner(self.ctx, M)
        return M

    def adjoint(self, grad_cams, grad_points, grad_xy_out=None, grad_depth_out=None):
        if grad_xy_out is None:
            grad_xy_out = np.empty((self.n_obs, 2), np.float32)
        if grad_depth_out is None:
            grad_depth_out = np.empty(self.n_obs, np.float32)
        self.last_adjoint_status = ba_adjoint(self.ctx, grad_cams, grad_points, grad_xy_out,
                                              grad_depth_out)
        return grad_xy_out, grad_depth_out

    def kernel_stats(self):
        return ba_kernel_stats(self.ctx)

    def reset_kernel_stats(self):
        return ba_reset_kernel_stats(self.ctx)

    def device_bytes(self) -> int:
        return ba_device_bytes(self.ctx)
