"""``torch.autograd.Function`` around the solve and its implicit adjoint.

Forward runs ``ba_solve`` to convergence; backward calls ``ba_adjoint``, which solves
``H v = dL/dtheta`` with the same Schur-PCG kernels and maps ``v`` to gradients of the 2-D
observations and depth priors (implicit function theorem at the converged solution). The
initial parameters get no gradient: at a strict local minimum the solution does not depend
on where the solve started.
"""
from __future__ import annotations

import numpy as np
import torch

from .api import BundleAdjuster


def _as_tensor(a, like: torch.Tensor, dtype):
    if isinstance(a, torch.Tensor):
        return a.to(device=like.device, dtype=dtype).contiguous()
    return torch.as_tensor(np.asarray(a), dtype=dtype, device=like.device).contiguous()


class BASolve(torch.autograd.Function):
    """cams, points = BASolve.apply(xy, depth, cams0, points0, problem)

    ``problem`` is a dict with ``cam_idx`` (N int32), ``pt_idx`` (N int32), ``intr`` (C x 3),
    optional ``depth_valid`` (N uint8), ``lambda_d``, ``fixed`` (camera ids) and ``options``
    (keyword options of :class:`BundleAdjuster`). ``depth`` may be None (no depth rows).
    """

    @staticmethod
    def forward(ctx, xy, depth, cams0, points0, problem):
        dev = xy
        opts = dict(problem.get("options", {}))
        ba = BundleAdjuster(_as_tensor(cams0.detach(), dev, torch.float64),
                            _as_tensor(problem["intr"], dev, torch.float64),
                            _as_tensor(points0.detach(), dev, torch.float64), **opts)
        ba.set_observations(_as_tensor(problem["cam_idx"], dev, torch.int32),
                            _as_tensor(problem["pt_idx"], dev, torch.int32),
                            xy.detach().to(torch.float32).contiguous())
        if depth is not None:
            valid = problem.get("depth_valid")
            ba.set_depth_priors(depth.detach().to(torch.float32).contiguous(),
                                None if valid is None else _as_tensor(valid, dev, torch.uint8),
                                float(problem.get("lambda_d", 1.0)))
        fixed = problem.get("fixed")
        if fixed is not None and len(fixed):
            ba.set_fixed_cameras(_as_tensor(fixed, dev, torch.int32))
        ctx.report = ba.solve()
        cams = torch.empty((ba.n_cams, 7), dtype=torch.float64, device=dev.device)
        pts = torch.empty((ba.n_points, 3), dtype=torch.float64, device=dev.device)
        ba.get_params_into(cams, pts)
        ctx.ba = ba
        ctx.has_depth = depth is not None
        return cams, pts

    @staticmethod
    def backward(ctx, grad_cams, grad_points):
        ba = ctx.ba
        dev = grad_cams.device if grad_cams is not None else grad_points.device
        if grad_cams is None:
            grad_cams = torch.zeros((ba.n_cams, 7), dtype=torch.float64, device=dev)
        if grad_points is None:
            grad_points = torch.zeros((ba.n_points, 3), dtype=torch.float64, device=dev)
        gxy = torch.empty((ba.n_obs, 2), dtype=torch.float32, device=dev)
        gd = torch.empty(ba.n_obs, dtype=torch.float32, device=dev)
        ba.adjoint(grad_cams.to(torch.float64).contiguous(),
                   grad_points.to(torch.float64).contiguous(), gxy, gd)
        return gxy, (gd if ctx.has_depth else None), None, None, None
