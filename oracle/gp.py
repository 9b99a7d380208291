"""Depth-constrained global positioning (GP) of the oracle (FP64, NumPy/SciPy).

Test infrastructure only (see the package docstring).

The objective of Eq. (1) with the depth constraint of Eqs. (4)-(5) and the pinned/free scale
partition of Eq. (8) (Sec. III-A, Sec. IV-A):

* camera rotations are fixed (they come from rotation averaging); the unknowns are the camera
  centres c_i, the points X_j and one scale s_ij per observation whose depth prior is invalid;
* the ray of an observation is the unit world direction ``v = R^T a / |a|`` with
  ``a = K^-1 [x, y, 1]`` (R maps world to camera);
* residual ``u = v - s (X - c)``; an observation with a valid prior is pinned at
  ``s = 1 / (d_hat |a|)``: the prior is a camera-frame z-depth and the scale of a unit ray is
  the inverse distance along it, which is ``z |a|`` (a reading: the paper states the pinned
  scale as the inverse of the measured depth for a unit-normalised ray);
* Huber on ``|u|^2`` (threshold ``huber``, ray units); ``F = 1/2 sum rho``;
* Jacobians ``du/dc = s I``, ``du/dX = -s I``, ``du/ds = -(X - c)`` (free scales only; the
  columns of pinned scales are not in J, Eq. (8));
* extraction: every observation with finite data is valid (no frustum test: GP starts from
  estimates far from the truth and has no reprojection); an observation brings 3 rows, less
  its own free scale, so 3 rows when pinned and 2 when free; a point needs 3, a camera 3 and
  must not be fixed; the greatest fixpoint of that pruning as in BA;
* LM exactly as in ``lm.py`` (Marquardt diagonal floored, Nielsen update, gain ratio on the
  per-observation actual reduction); the damped system is solved directly: the scale block is
  diagonal (each scale has one observation), so it is eliminated exactly, then the points
  (3x3 blocks) by the dense camera Schur complement and Cholesky of ``lm.schur_solve``; a
  candidate with a free scale <= 0 is rejected (a scale is an inverse distance);
* free scales start at the inverse distance of the current estimate, ``1 / |X - c|``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.sparse as sp

from .geometry import quat_to_rot
from .model import Problem, huber
from .extract import activity_fixpoint, ranks
from .lm import schur_solve, nielsen_update


@dataclass
class GpOptions:
    huber: float = 0.1
    lambda_init: float = 1e-3
    lambda_min: float = 1e-12
    lambda_max: float = 1e12
    diag_min: float = 1e-6
    diag_max: float = 1e32
    accept_ratio: float = 1e-3
    cost_rel_tol: float = 1e-10
    grad_tol: float = 1e-10
    max_iters: int = 100


def rays(prob: Problem, q: np.ndarray):
    """Unit world ray directions (n x 3) and |K^-1 [x, y, 1]| of every observation."""
    cam = prob.cam_idx
    f, cx, cy = prob.intr[cam, 0], prob.intr[cam, 1], prob.intr[cam, 2]
    a = np.stack([(prob.xy[:, 0] - cx) / f, (prob.xy[:, 1] - cy) / f, np.ones(prob.n_obs)], 1)
    na = np.linalg.norm(a, axis=1)
    R = quat_to_rot(q)[cam]
    v = np.einsum("nji,nj->ni", R, a) / na[:, None]   # R^T a / |a|
    return v, na


def pinned(prob: Problem) -> np.ndarray:
    """Eq. (8): S_pin = observations with a valid depth prior."""
    return prob.prior_mask.copy()


def pinned_scales(prob: Problem, na: np.ndarray) -> np.ndarray:
    """s = 1 / (d_hat |a|) on pinned observations, 0 elsewhere."""
    return np.where(prob.prior_mask, prob.dinv / na, 0.0)


@dataclass
class GpState:
    c: np.ndarray            # C x 3 camera centres
    X: np.ndarray            # P x 3 points
    s: np.ndarray            # N scales (pinned entries hold their fixed value)
    lam: float = 1e-3
    nu: float = 2.0

    @classmethod
    def initial(cls, prob: Problem, q, cams, points, opts: GpOptions) -> "GpState":
        c = np.asarray(cams, np.float64)[:, 4:7].copy()
        X = np.asarray(points, np.float64).copy()
        _, na = rays(prob, q)
        dist = np.linalg.norm(X[prob.pt_idx] - c[prob.cam_idx], axis=1)
        s = np.where(prob.prior_mask, pinned_scales(prob, na), 1.0 / np.maximum(dist, 1e-12))
        return cls(c=c, X=X, s=s, lam=opts.lambda_init)

    def copy(self) -> "GpState":
        return GpState(self.c.copy(), self.X.copy(), self.s.copy(), self.lam, self.nu)


@dataclass
class GpExtraction:
    obs_active: np.ndarray
    cam_active: np.ndarray
    pt_active: np.ndarray
    rounds: int
    obs: np.ndarray          # active observations, ascending
    cam_rank: np.ndarray
    cams: np.ndarray
    pt_rank: np.ndarray
    pts: np.ndarray
    free: np.ndarray         # active observations with a free scale, ascending
    free_rank: np.ndarray    # N: column of the free scale among them, -1 otherwise


def gp_valid(prob: Problem) -> np.ndarray:
    return np.isfinite(prob.xy).all(axis=1)


def gp_extract(prob: Problem) -> GpExtraction:
    """Active sets of GP. The row count of an observation (3 pinned, 2 free) is the BA row
    count with the prior mask as the pinned set and depth rows on, so the BA fixpoint with
    3-row cameras computes it."""
    rows_prob = Problem(n_cams=prob.n_cams, n_points=prob.n_points, intr=prob.intr,
                        cam_idx=prob.cam_idx, pt_idx=prob.pt_idx, xy=prob.xy,
                        dinv=prob.dinv, prior_mask=pinned(prob), lambda_d=1.0,
                        img_w=prob.img_w, img_h=prob.img_h, fixed=prob.fixed)
    oa, ca, pa, rounds = activity_fixpoint(rows_prob, gp_valid(prob), "rows", cam_dim=3)
    cam_rank, cams = ranks(ca)
    pt_rank, pts = ranks(pa)
    obs = np.nonzero(oa)[0]
    free = obs[~prob.prior_mask[obs]]
    free_rank = np.full(prob.n_obs, -1, np.int64)
    free_rank[free] = np.arange(free.size)
    return GpExtraction(oa, ca, pa, rounds, obs, cam_rank, cams, pt_rank, pts, free, free_rank)


@dataclass
class GpLinearization:
    obs: np.ndarray
    u: np.ndarray            # n x 3
    rho: np.ndarray
    w: np.ndarray
    J: sp.csr_matrix         # 3n x (3 Ca + 3 Pa + n_free)
    ncol_cam: int
    ncol_pt: int


def gp_residuals(prob: Problem, q, st: GpState, obs):
    v, _ = rays(prob, q)
    cam, pt = prob.cam_idx[obs], prob.pt_idx[obs]
    d = st.X[pt] - st.c[cam]
    return v[obs] - st.s[obs, None] * d, d


def gp_linearize(prob: Problem, q, st: GpState, ex: GpExtraction, delta: float):
    obs = ex.obs
    u, d = gp_residuals(prob, q, st, obs)
    rho, w, _ = huber(np.sum(u * u, axis=1), delta)
    n = obs.size
    s = st.s[obs]
    cam, pt = prob.cam_idx[obs], prob.pt_idx[obs]
    nc = 3 * ex.cams.size
    npt = 3 * ex.pts.size
    rows = np.arange(3 * n).reshape(n, 3)
    ri, ci, vi = [], [], []
    crank = ex.cam_rank[cam]
    has_cam = crank >= 0                     # fixed cameras have no columns
    eye = np.arange(3)
    # du/dc = s I
    rr = rows[has_cam]
    ri.append(rr.ravel())
    ci.append((3 * crank[has_cam][:, None] + eye).ravel())
    vi.append(np.repeat(s[has_cam], 3))
    # du/dX = -s I
    ri.append(rows.ravel())
    ci.append((nc + 3 * ex.pt_rank[pt][:, None] + eye).ravel())
    vi.append(np.repeat(-s, 3))
    # du/ds = -(X - c), free scales only
    fr = ex.free_rank[obs]
    isf = fr >= 0
    ri.append(rows[isf].ravel())
    ci.append(np.repeat(nc + npt + fr[isf], 3))
    vi.append((-d[isf]).ravel())
    J = sp.csr_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))),
                      shape=(3 * n, nc + npt + ex.free.size))
    return GpLinearization(obs, u, rho, w, J, nc, npt)


def gp_normal_equations(lin: GpLinearization):
    Wd = sp.diags(np.repeat(lin.w, 3))
    H = (lin.J.T @ Wd @ lin.J).tocsr()
    g = lin.J.T @ (np.repeat(lin.w, 3) * lin.u.ravel())
    return H, g


def gp_damped(H: sp.spmatrix, lam: float, opts: GpOptions) -> sp.csr_matrix:
    D = np.clip(H.diagonal(), opts.diag_min, opts.diag_max)
    return (H + sp.diags(lam * D)).tocsr()


def gp_solve_system(Hd: sp.spmatrix, rhs: np.ndarray, nc: int, npt: int) -> np.ndarray:
    """Solve the damped GP system: eliminate the diagonal scale block, then the points and
    cameras with the dense Schur complement + Cholesky."""
    Hd = Hd.tocsr()
    m = nc + npt
    Hss = Hd[m:, m:]
    hs = Hss.diagonal()
    assert (Hss - sp.diags(hs)).count_nonzero() == 0, "scale block must be diagonal"
    B = Hd[:m, m:]
    Hr = Hd[:m, :m] - B @ sp.diags(1.0 / hs) @ B.T
    rr = rhs[:m] - B @ (rhs[m:] / hs)
    xcp = schur_solve(Hr, rr, nc)
    xs = (rhs[m:] - B.T @ xcp) / hs
    return np.concatenate([xcp, xs])


@dataclass
class GpStepReport:
    status: str = "ok"
    accepted: bool = False
    cost_before: float = 0.0
    cost_after: float = 0.0
    model_decrease: float = 0.0
    gain_ratio: float = 0.0
    lam: float = 0.0
    n_obs: int = 0
    n_free: int = 0
    grad_inf: float = 0.0
    rms: float = 0.0
    delta: np.ndarray | None = None
    extraction: GpExtraction | None = None
    extra: dict = field(default_factory=dict)


def gp_candidate(st: GpState, ex: GpExtraction, delta: np.ndarray) -> GpState:
    nc, npt = 3 * ex.cams.size, 3 * ex.pts.size
    new = st.copy()
    new.c[ex.cams] = st.c[ex.cams] + delta[:nc].reshape(-1, 3)
    new.X[ex.pts] = st.X[ex.pts] + delta[nc:nc + npt].reshape(-1, 3)
    new.s[ex.free] = st.s[ex.free] + delta[nc + npt:]
    return new


def gp_step(prob: Problem, q, st: GpState, opts: GpOptions):
    """One LM iteration of GP. Returns (new_state, GpStepReport)."""
    ex = gp_extract(prob)
    rep = GpStepReport(lam=st.lam, n_obs=int(ex.obs.size), n_free=int(ex.free.size),
                       extraction=ex)
    if ex.obs.size == 0:
        rep.status = "empty"
        return st.copy(), rep
    lin = gp_linearize(prob, q, st, ex, opts.huber)
    H, g = gp_normal_equations(lin)
    F = 0.5 * float(np.sum(lin.rho))
    rep.cost_before = F
    rep.rms = float(np.sqrt(np.mean(np.sum(lin.u * lin.u, axis=1))))
    rep.grad_inf = float(np.max(np.abs(g))) if g.size else 0.0
    delta = gp_solve_system(gp_damped(H, st.lam, opts), -g, lin.ncol_cam, lin.ncol_pt)
    rep.delta = delta
    Jd = (lin.J @ delta).reshape(lin.u.shape)
    model = -(float(g @ delta) + 0.5 * float(np.sum(lin.w[:, None] * Jd * Jd)))
    rep.model_decrease = model
    cand = gp_candidate(st, ex, delta)
    if np.any(cand.s[ex.free] <= 0):
        F2, dF = np.inf, -np.inf
    else:
        u2, _ = gp_residuals(prob, q, cand, ex.obs)
        rho2 = huber(np.sum(u2 * u2, axis=1), opts.huber)[0]
        F2 = 0.5 * float(np.sum(rho2))
        dF = 0.5 * float(np.sum(lin.rho - rho2))
    rep.cost_after = F - dF if np.isfinite(F2) else np.inf
    ratio = dF / model if (model > 0 and np.isfinite(F2)) else -np.inf
    rep.gain_ratio = ratio
    rep.extra["actual_decrease"] = dF
    rep.accepted = bool(np.isfinite(F2) and dF > 0 and ratio > opts.accept_ratio)
    out = cand if rep.accepted else st.copy()
    out.lam, out.nu = nielsen_update(st.lam, st.nu, rep.accepted, ratio, opts.lambda_min,
                                     opts.lambda_max)
    return out, rep


def gp_solve(prob: Problem, q, st: GpState, opts: GpOptions, max_iters: int | None = None):
    reps = []
    for _ in range(opts.max_iters if max_iters is None else max_iters):
        st, rep = gp_step(prob, q, st, opts)
        reps.append(rep)
        if rep.status == "empty" or rep.grad_inf <= opts.grad_tol:
            break
        if rep.accepted and rep.extra["actual_decrease"] <= opts.cost_rel_tol * rep.cost_before:
            break
        if not rep.accepted and rep.lam >= opts.lambda_max:
            break
    return st, reps
