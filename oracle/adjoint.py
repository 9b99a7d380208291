"""Implicit adjoint of the converged BA solution, dense/direct reference (FP64).

Test infrastructure only (see the package docstring).

At a converged solution the gradient ``g(theta*; x, d_hat)`` of the BA cost over the free
parameters (active, not fixed) vanishes. By the implicit function theorem
``d theta*/d y = -H^-1 dg/dy`` for an input y, so for a scalar loss L(theta*)

    v = H^-1 dL/dtheta,      dL/dy = -(dg/dy)^T v.

H is the robust-corrected Gauss-Newton Hessian ``sum_k J_k^T M_k J_k`` with
``M_k = rho'_k I + 2 rho''_k e_k e_k^T`` (the second-derivative term of the residuals is
dropped). For observation k with ``t_k = J_k v``:

    dL/dx_k     = (M_k t_k)[0:2]                 (e_k depends on x_k through -I),
    dL/dd_hat_k = -(M_k t_k)[2] * lambda_d m_k / d_hat_k^2.

Tangent mapping of a camera gradient (left perturbation xi = (rho, phi)):
``dc/drho = -R^T``, ``dc/dphi = 0`` and ``dq/dphi = 1/2 [-q_v^T ; q_w I - [q_v]x]``.
H is solved directly over all free parameters (no Schur reduction).

``full_hessian`` keeps what the Gauss-Newton H drops: it differentiates the exact gradient
``g = J^T rho' e`` of the cost by central differences along every free tangent coordinate
(the active set and the Huber regimes of the base point held), so that its adjoint carries
the second-order residual term ``sum rho' e . d^2 e``. It is the check of how much of an
adjoint's gap to finite differences of re-solves that term explains.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .geometry import quat_normalize, quat_to_rot
from .lm import (candidate, damped, extract, linearize, metric_blocks, normal_equations,
                 Options, State)
from .model import Problem


def tangent_gradient(st: State, cams: np.ndarray, grad_cams: np.ndarray) -> np.ndarray:
    """Map dL/d[q, c] (k x 7) of the listed cameras to dL/dxi (k x 6)."""
    q = quat_normalize(st.q[cams])
    R = quat_to_rot(q)
    gq, gc = grad_cams[cams, :4], grad_cams[cams, 4:7]
    g_rho = -np.einsum("nij,nj->ni", R, gc)
    qw, qv = q[:, :1], q[:, 1:]
    gw, gv = gq[:, :1], gq[:, 1:]
    g_phi = 0.5 * (-gw * qv + qw * gv + np.cross(qv, gv))
    return np.concatenate([g_rho, g_phi], axis=1)


def full_hessian(prob: Problem, st: State, opts: Options, h: float = 1e-6) -> np.ndarray:
    """Dense Hessian of F over the free compact parameters (cameras in the left-perturbation
    tangent space, then points): column j is the central difference of the exact gradient
    along coordinate j, over the active set of ``st``. At a converged point (g = 0) this is
    the Hessian of the cost itself; it is symmetrised."""
    ex = extract(prob, st, opts)
    n = 6 * ex.cams.size + 3 * ex.pts.size
    H = np.zeros((n, n))
    for j in range(n):
        cols = []
        for sgn in (1.0, -1.0):
            d = np.zeros(n)
            d[j] = sgn * h
            lin = linearize(prob, candidate(st, ex, d), ex, opts.huber_px)
            cols.append(normal_equations(lin)[1])
        H[:, j] = (cols[0] - cols[1]) / (2 * h)
    return 0.5 * (H + H.T)


def adjoint(prob: Problem, st: State, opts: Options, grad_cams: np.ndarray,
            grad_points: np.ndarray, damping: float = 0.0, hessian: str = "gauss_newton"):
    """Returns (grad_xy N x 2, grad_depth N, v) for the loss gradient at state ``st``.

    ``damping`` > 0 solves (H + damping D) v = dL/dtheta with Marquardt's D = diag(H) clamped
    like the LM damping: a Tikhonov-regularised derivative for systems where H is singular
    (parity unpinned for damping > 0 beyond its damping -> 0 limit).
    ``hessian = "full"`` solves with ``full_hessian`` instead of the robust-corrected
    Gauss-Newton H (dense; small problems only).
    """
    if prob.fixed.size == 0:
        raise ValueError("the adjoint needs a fixed gauge (at least one fixed camera)")
    if opts.refine_focal:
        raise ValueError("the adjoint covers poses and points only (focal lengths fixed)")
    ex = extract(prob, st, opts)
    lin = linearize(prob, st, ex, opts.huber_px)
    gbar = np.concatenate([tangent_gradient(st, ex.cams, grad_cams).ravel(),
                           np.asarray(grad_points, np.float64)[ex.pts].ravel()])
    if hessian == "full":
        v = np.linalg.solve(full_hessian(prob, st, opts), gbar)
    else:
        H, _ = normal_equations(lin, robust_correction=True)
        if damping > 0:
            H = damped(H, damping, opts)
        v = spla.spsolve(H.tocsc(), gbar)
    M = metric_blocks(lin, robust_correction=True)
    u = (M @ (lin.J @ v)).reshape(lin.e.shape)
    gxy = np.zeros((prob.n_obs, 2))
    gd = np.zeros(prob.n_obs)
    gxy[lin.obs] = u[:, :2]
    if prob.lambda_d > 0:
        gd[lin.obs] = -u[:, 2] * prob.lambda_d * prob.dinv[lin.obs] ** 2
    return gxy, gd, v
