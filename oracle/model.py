"""Residual model of the oracle: reprojection, inverse-depth prior, Huber (FP64, NumPy).

Test infrastructure only (see the package docstring).

* Reprojection residual, Eq. (2): ``r = Pi(zeta_i, X_j, K_i) - x_ij`` with a pinhole
  ``Pi = (f x/z + cx, f y/z + cy)`` on camera coordinates ``(x, y, z) = R_i (X_j - c_i)``.
* Depth residual, Eq. (6): ``r^d = 1/Depth - 1/d_hat`` with Depth the camera-frame z.
* Masked reference inverse depth, Eq. (9): ``d~^-1 = m * d_hat^-1``; an invalid prior keeps
  its row with target 0 (the weak far-depth prior of Sec. IV-A).
* Depth-weighted objective, Eq. (7): the residual of one observation is the stacked vector
  ``e = [r ; lambda_d r^d]`` and one robustifier is applied to ``|e|^2``.
* Huber (Sec. III-A names it): ``rho(s) = s`` for ``s <= delta^2`` and
  ``2 delta sqrt(s) - delta^2`` above; the cost is ``F = 1/2 sum rho(|e|^2)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

from .geometry import quat_to_rot, hat


@dataclass
class Problem:
    """Observations and fixed data of one BA problem (float64 copies of the inputs)."""
    n_cams: int
    n_points: int
    intr: np.ndarray            # C x 3 [f, cx, cy]
    cam_idx: np.ndarray         # N int64
    pt_idx: np.ndarray          # N int64
    xy: np.ndarray              # N x 2 float64 (exact copies of the float32 inputs)
    dinv: np.ndarray            # N float64: m / d_hat (0 where the prior is invalid)
    prior_mask: np.ndarray      # N bool: m
    lambda_d: float             # 0 disables the depth rows
    img_w: int
    img_h: int
    fixed: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))

    @property
    def n_obs(self) -> int:
        return int(self.cam_idx.shape[0])

    @property
    def rows_per_obs(self) -> int:
        return 3 if self.lambda_d > 0 else 2

    @classmethod
    def from_scene(cls, sc, use_depth=None, lambda_d=None) -> "Problem":
        use_depth = sc.use_depth if use_depth is None else use_depth
        lam = (sc.lambda_d if lambda_d is None else lambda_d) if use_depth else 0.0
        d = sc.depth.astype(np.float64)
        m = (sc.depth_valid != 0) & np.isfinite(d) & (d > 0) & use_depth
        dinv = np.where(m, 1.0 / np.where(m, d, 1.0), 0.0)
        return cls(n_cams=sc.n_cams, n_points=sc.n_points, intr=sc.intr.astype(np.float64),
                   cam_idx=sc.cam_idx.astype(np.int64), pt_idx=sc.pt_idx.astype(np.int64),
                   xy=sc.xy.astype(np.float64), dinv=dinv, prior_mask=m, lambda_d=float(lam),
                   img_w=sc.img_w, img_h=sc.img_h, fixed=sc.fixed.astype(np.int64))


def huber(s: np.ndarray, delta: float):
    """rho(s), rho'(s), rho''(s) of the Huber function on the squared norm s (delta<=0: L2)."""
    s = np.asarray(s, dtype=np.float64)
    if delta <= 0:
        return s.copy(), np.ones_like(s), np.zeros_like(s)
    big = s > delta * delta
    rs = np.sqrt(np.where(big, s, 1.0))
    rho = np.where(big, 2 * delta * rs - delta * delta, s)
    d1 = np.where(big, delta / rs, 1.0)
    d2 = np.where(big, -0.5 * delta / (rs * rs * rs), 0.0)
    return rho, d1, d2


def camera_points(q, c, X, cam, pt):
    """Camera-frame coordinates X_c = R (X - c) and R for observations (cam, pt)."""
    R = quat_to_rot(q)[cam]
    Xc = np.einsum("nij,nj->ni", R, X[pt] - c[cam])
    return Xc, R


def residuals(prob: Problem, q, c, X, obs=None):
    """Stacked residuals e (n x 2 or n x 3), camera coordinates X_c and R of observations."""
    obs = np.arange(prob.n_obs) if obs is None else obs
    cam, pt = prob.cam_idx[obs], prob.pt_idx[obs]
    Xc, R = camera_points(q, c, X, cam, pt)
    f, cx, cy = prob.intr[cam, 0], prob.intr[cam, 1], prob.intr[cam, 2]
    iz = 1.0 / Xc[:, 2]
    u = f * Xc[:, 0] * iz + cx
    v = f * Xc[:, 1] * iz + cy
    cols = [u - prob.xy[obs, 0], v - prob.xy[obs, 1]]
    if prob.lambda_d > 0:
        cols.append(prob.lambda_d * (iz - prob.dinv[obs]))
    return np.stack(cols, axis=1), Xc, R


def jacobians(prob: Problem, Xc, R, cam):
    """Analytic blocks de/dxi (n x r x 6) and de/dX (n x r x 3).

    de/dX_c of the pinhole is (f/z)[[1, 0, -x/z], [0, 1, -y/z]]; of lambda_d/z it is
    [0, 0, -lambda_d/z^2]. dX_c/dxi = [I | -[X_c]x] for the left perturbation and
    dX_c/dX = R.
    """
    n = Xc.shape[0]
    f = prob.intr[cam, 0]
    iz = 1.0 / Xc[:, 2]
    r = prob.rows_per_obs
    A = np.zeros((n, r, 3))
    A[:, 0, 0] = f * iz
    A[:, 0, 2] = -f * Xc[:, 0] * iz * iz
    A[:, 1, 1] = f * iz
    A[:, 1, 2] = -f * Xc[:, 1] * iz * iz
    if r == 3:
        A[:, 2, 2] = -prob.lambda_d * iz * iz
    B = np.concatenate([np.broadcast_to(np.eye(3), (n, 3, 3)), -hat(Xc)], axis=2)
    return A @ B, A @ R


def cost(prob: Problem, q, c, X, obs, delta: float) -> float:
    e, _, _ = residuals(prob, q, c, X, obs)
    rho, _, _ = huber(np.sum(e * e, axis=1), delta)
    return 0.5 * float(np.sum(rho))
