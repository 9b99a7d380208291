"""Dynamic parameter extraction of the oracle (Sec. IV-B, Eqs. (10)-(15)).

Test infrastructure only (see the package docstring).

Step 1, validity (Eq. (10) and the frustum test of Sec. IV-B): an observation is valid when
its camera-frame depth exceeds ``min_depth`` (0.1), its projection falls in
``[0, W) x [0, H)`` and, when a filter threshold is set, its 2-D reprojection error is at
most ``filter_px``.

Step 2, active sets (Eqs. (11)-(12)). Reading of "under-constrained": each valid
observation contributes 2 rows, plus 1 when it carries a valid depth prior (depth rows
enabled). A point is active when it has at least 3 rows, a camera when it has at least 6
rows and is not held fixed; observations of inactive points or of inactive free cameras are
dropped, and this is repeated until nothing changes (the greatest fixpoint).
``rule="literal"`` uses the paper's literal sets instead: any entity with one valid
observation is active.

Step 3, rank remap (Eqs. (13)-(15)): active entities are numbered in ascending original
index, the order ``torch.unique`` returns.
"""
from __future__ import annotations

import numpy as np

from .model import Problem, residuals


def geometric_validity(prob: Problem, q, c, X, min_depth: float, filter_px: float):
    e, Xc, _ = residuals(prob, q, c, X)
    z = Xc[:, 2]
    ok = z > min_depth
    zs = np.where(ok, z, 1.0)
    f, cx, cy = prob.intr[prob.cam_idx].T
    u = f * Xc[:, 0] / zs + cx
    v = f * Xc[:, 1] / zs + cy
    ok &= (u >= 0) & (u < prob.img_w) & (v >= 0) & (v < prob.img_h)
    if filter_px > 0:
        ok &= (e[:, 0] ** 2 + e[:, 1] ** 2) <= filter_px * filter_px
    return ok


def observation_rows(prob: Problem) -> np.ndarray:
    rows = np.full(prob.n_obs, 2, np.int64)
    if prob.lambda_d > 0:
        rows += prob.prior_mask.astype(np.int64)
    return rows


def activity_fixpoint(prob: Problem, valid: np.ndarray, rule: str = "rows", cam_dim: int = 6):
    """Greatest fixpoint of the pruning rule (a camera needs cam_dim rows). Returns
    (obs_active, cam_active, pt_active, rounds)."""
    fixed = np.zeros(prob.n_cams, bool)
    fixed[prob.fixed] = True
    rows = observation_rows(prob)
    need_p, need_c = (3, cam_dim) if rule == "rows" else (1, 1)
    act = valid.copy()
    rounds = 0
    while True:
        rounds += 1
        rp = np.bincount(prob.pt_idx[act], weights=rows[act], minlength=prob.n_points)
        rc = np.bincount(prob.cam_idx[act], weights=rows[act], minlength=prob.n_cams)
        pt_ok = rp >= need_p
        cam_ok = (rc >= need_c) & ~fixed
        keep = act & pt_ok[prob.pt_idx] & (cam_ok | fixed)[prob.cam_idx]
        if np.array_equal(keep, act):
            return act, cam_ok, pt_ok, rounds
        act = keep


def ranks(active: np.ndarray):
    """rank[i] = position of i among the active entities (ascending), -1 if inactive;
    also the list of active original indices."""
    members = np.nonzero(active)[0]
    rank = np.full(active.shape[0], -1, np.int64)
    rank[members] = np.arange(members.size)
    return rank, members
