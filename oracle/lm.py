"""Levenberg-Marquardt bundle adjustment of the oracle (FP64, NumPy/SciPy).

Test infrastructure only (see the package docstring).

One LM iteration, following Sec. III-C and Sec. IV-B:

1. extraction at the current parameters (validity, active sets, ranks; ``extract.py``);
2. residuals and Jacobian blocks of the active observations (``model.py``), robust weights
   ``w = rho'(|e|^2)``; the Jacobian is assembled as one sparse matrix over the compact
   columns ``[6 per active camera | 3 per active point]`` (Eq. (15) ranks);
3. the LM system of Eq. (3), ``(H + lambda D) delta = -g`` with ``H = J^T W J``,
   ``g = J^T W e`` and Marquardt's ``D = diag(H)`` floored to ``[1e-6, 1e32]``;
4. the camera block is obtained from the Schur complement ``S = U* - W V*^-1 W^T`` formed as
   a dense matrix and factorised by Cholesky (LAPACK through SciPy); the point block by
   back-substitution;
5. the candidate ``theta (+) delta`` (left SE(3) update for cameras, additive for points),
   its cost over the same active observations (+inf if one of them has z <= min_depth),
   the gain ratio of the actual reduction (summed per observation) against the model
   decrease ``-(g^T delta + 1/2 |W^(1/2) J delta|^2)``;
6. accept when the cost drops and the ratio exceeds 1e-3, then scatter the compact update
   into the full arrays (inactive entries untouched); lambda follows Nielsen's rule
   (accept: lambda *= max(1/3, 1 - (2 rho - 1)^3), nu = 2; reject: lambda *= nu, nu *= 2).

With ``refine_focal`` the per-camera focal length of the intrinsics (Sec. III-B lists K among
the BA parameters) becomes a seventh camera parameter: the camera block is 7 x 7, de/df =
[x/z, y/z, 0], the update is additive, and a camera needs 7 residual rows to be active.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .geometry import retract_cameras
from .model import Problem, residuals, jacobians, huber
from .extract import geometric_validity, activity_fixpoint, ranks


@dataclass
class Options:
    min_depth: float = 0.1
    huber_px: float = 0.0
    filter_px: float = 0.0
    rule: str = "rows"            # "rows" (row-count rule) or "literal" (>= 1 observation)
    lambda_init: float = 1e-3
    lambda_min: float = 1e-12
    lambda_max: float = 1e12
    diag_min: float = 1e-6
    diag_max: float = 1e32
    accept_ratio: float = 1e-3
    cost_rel_tol: float = 1e-10
    grad_tol: float = 1e-10
    max_iters: int = 100
    refine_focal: bool = False

    @property
    def cam_dim(self) -> int:
        return 7 if self.refine_focal else 6


@dataclass
class State:
    q: np.ndarray
    c: np.ndarray
    X: np.ndarray
    lam: float
    nu: float = 2.0
    f: np.ndarray | None = None   # per-camera focal length when it is refined

    @classmethod
    def initial(cls, cams: np.ndarray, points: np.ndarray, opts: Options,
                focal: np.ndarray | None = None) -> "State":
        cams = np.asarray(cams, np.float64)
        f = np.asarray(focal, np.float64).copy() if opts.refine_focal else None
        return cls(q=cams[:, :4].copy(), c=cams[:, 4:7].copy(),
                   X=np.asarray(points, np.float64).copy(), lam=opts.lambda_init, f=f)

    def cams(self) -> np.ndarray:
        return np.concatenate([self.q, self.c], axis=1)

    def copy(self) -> "State":
        return State(self.q.copy(), self.c.copy(), self.X.copy(), self.lam, self.nu,
                     None if self.f is None else self.f.copy())


def problem_at(prob: Problem, st: State) -> Problem:
    """The problem with the state's focal lengths in its intrinsics (when refined)."""
    if st.f is None:
        return prob
    intr = prob.intr.copy()
    intr[:, 0] = st.f
    return replace(prob, intr=intr)


@dataclass
class Extraction:
    valid: np.ndarray
    obs_active: np.ndarray
    cam_active: np.ndarray
    pt_active: np.ndarray
    rounds: int
    obs: np.ndarray
    cam_rank: np.ndarray
    cams: np.ndarray
    pt_rank: np.ndarray
    pts: np.ndarray


def extract(prob: Problem, st: State, opts: Options) -> Extraction:
    prob = problem_at(prob, st)
    valid = geometric_validity(prob, st.q, st.c, st.X, opts.min_depth, opts.filter_px)
    oa, ca, pa, rounds = activity_fixpoint(prob, valid, opts.rule, opts.cam_dim)
    cr, cams = ranks(ca)
    pr, pts = ranks(pa)
    return Extraction(valid, oa, ca, pa, rounds, np.nonzero(oa)[0], cr, cams, pr, pts)


@dataclass
class Linearization:
    obs: np.ndarray
    e: np.ndarray          # n x r
    Jc: np.ndarray         # n x r x d (d = 6, or 7 with the focal length)
    Jp: np.ndarray         # n x r x 3
    rho: np.ndarray        # n
    w: np.ndarray          # n   rho'
    d2: np.ndarray         # n   rho''
    J: sp.csr_matrix       # (n r) x (d Ca + 3 Pa)
    ncol_cam: int


def linearize(prob: Problem, st: State, ex: Extraction, delta: float) -> Linearization:
    prob = problem_at(prob, st)
    obs = ex.obs
    e, Xc, R = residuals(prob, st.q, st.c, st.X, obs)
    cam, pt = prob.cam_idx[obs], prob.pt_idx[obs]
    Jc, Jp = jacobians(prob, Xc, R, cam)
    if st.f is not None:
        # de/df of the pinhole rows: (x/z, y/z); the inverse-depth row does not depend on f
        Jf = np.zeros(e.shape + (1,))
        Jf[:, 0, 0] = Xc[:, 0] / Xc[:, 2]
        Jf[:, 1, 0] = Xc[:, 1] / Xc[:, 2]
        Jc = np.concatenate([Jc, Jf], axis=2)
    d = Jc.shape[2]
    rho, w, d2 = huber(np.sum(e * e, axis=1), delta)
    n, r = e.shape
    nc = d * ex.cams.size
    ncols = nc + 3 * ex.pts.size
    rows = np.arange(n * r).reshape(n, r)
    crank = ex.cam_rank[cam]
    has_cam = crank >= 0                   # observations of fixed cameras have no camera block
    ri, ci, vi = [], [], []
    rr = np.broadcast_to(rows[:, :, None], (n, r, d))[has_cam]
    cc = np.broadcast_to((d * crank)[:, None, None] + np.arange(d), (n, r, d))[has_cam]
    ri.append(rr.ravel()); ci.append(cc.ravel()); vi.append(Jc[has_cam].ravel())
    rr = np.broadcast_to(rows[:, :, None], (n, r, 3))
    cc = np.broadcast_to((nc + 3 * ex.pt_rank[pt])[:, None, None] + np.arange(3), (n, r, 3))
    ri.append(rr.ravel()); ci.append(cc.ravel()); vi.append(Jp.ravel())
    J = sp.csr_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))),
                      shape=(n * r, ncols))
    return Linearization(obs, e, Jc, Jp, rho, w, d2, J, nc)


def metric_blocks(lin: Linearization, robust_correction: bool) -> sp.csr_matrix:
    """Per-observation metric M_k as a sparse block-diagonal matrix.

    IRLS (the LM step): ``M_k = rho'_k I``. Robust-corrected Gauss-Newton (the adjoint):
    ``M_k = rho'_k I + 2 rho''_k e_k e_k^T``.
    """
    n, r = lin.e.shape
    M = lin.w[:, None, None] * np.broadcast_to(np.eye(r), (n, r, r))
    if robust_correction:
        M = M + 2 * lin.d2[:, None, None] * lin.e[:, :, None] * lin.e[:, None, :]
    base = (np.arange(n) * r)[:, None, None]
    ri = np.broadcast_to(base + np.arange(r)[None, :, None], (n, r, r))
    ci = np.broadcast_to(base + np.arange(r)[None, None, :], (n, r, r))
    return sp.csr_matrix((M.ravel(), (ri.ravel(), ci.ravel())), shape=(n * r, n * r))


def normal_equations(lin: Linearization, robust_correction: bool = False):
    M = metric_blocks(lin, robust_correction)
    MJ = M @ lin.J
    H = (lin.J.T @ MJ).tocsr()
    g = lin.J.T @ (M @ lin.e.ravel())
    return H, g


def _point_block_inverse(Hpp: sp.spmatrix) -> sp.csr_matrix:
    coo = Hpp.tocoo()
    n = Hpp.shape[0] // 3
    same = coo.row // 3 == coo.col // 3
    blocks = np.zeros((n, 3, 3))
    np.add.at(blocks, (coo.row[same] // 3, coo.row[same] % 3, coo.col[same] % 3),
              coo.data[same])
    inv = np.linalg.inv(blocks)
    base = (np.arange(n) * 3)[:, None, None]
    ri = np.broadcast_to(base + np.arange(3)[None, :, None], (n, 3, 3))
    ci = np.broadcast_to(base + np.arange(3)[None, None, :], (n, 3, 3))
    return sp.csr_matrix((inv.ravel(), (ri.ravel(), ci.ravel())), shape=(3 * n, 3 * n))


def reduced_camera_system(H: sp.spmatrix, rhs: np.ndarray, nc: int):
    """The camera Schur complement of Eq. (3)'s system after eliminating the 3x3 point blocks:
    ``S = U - W V^-1 W^T`` as a dense matrix and ``b = rhs_c - W V^-1 rhs_p``. Returns
    ``(S, b, Vinv, W)``."""
    H = H.tocsr()
    Vinv = _point_block_inverse(H[nc:, nc:])
    U = H[:nc, :nc]
    W = H[:nc, nc:]
    S = (U - W @ Vinv @ W.T).toarray()
    b = rhs[:nc] - W @ (Vinv @ rhs[nc:])
    return S, b, Vinv, W


def schur_solve(H: sp.spmatrix, rhs: np.ndarray, nc: int) -> np.ndarray:
    """Solve H x = rhs by eliminating the 3x3 point blocks: a dense Schur complement on the
    camera columns, Cholesky, and back-substitution. Raises LinAlgError if S is not SPD."""
    H = H.tocsr()
    rp = rhs[nc:]
    if nc == 0:
        return _point_block_inverse(H) @ rp
    S, b, Vinv, W = reduced_camera_system(H, rhs, nc)
    xc = sla.cho_solve(sla.cho_factor(S, lower=True), b)
    xp = Vinv @ (rp - W.T @ xc)
    return np.concatenate([xc, xp])


def nielsen_update(lam: float, nu: float, accepted: bool, ratio: float, lambda_min: float,
                   lambda_max: float):
    """Damping schedule of Nielsen (1999), as given by Madsen, Nielsen and Tingleff (2004):
    after an accepted step with gain ratio ``ratio`` the damping is scaled by
    ``max(1/3, 1 - (2 ratio - 1)^3)`` and ``nu`` resets to 2; after a rejection it is scaled
    by ``nu`` and ``nu`` doubles. The damping is clamped to ``[lambda_min, lambda_max]``.
    Returns ``(lam, nu)``."""
    if accepted:
        f = max(1.0 / 3.0, 1.0 - (2.0 * ratio - 1.0) ** 3)
        return max(lambda_min, min(lambda_max, lam * f)), 2.0
    return min(lam * nu, lambda_max), nu * 2.0


def damped(H: sp.spmatrix, lam: float, opts: Options) -> sp.csr_matrix:
    D = np.clip(H.diagonal(), opts.diag_min, opts.diag_max)
    return (H + sp.diags(lam * D)).tocsr()


@dataclass
class StepReport:
    status: str = "ok"            # "ok", "empty", "singular"
    accepted: bool = False
    cost_before: float = 0.0
    cost_after: float = 0.0
    model_decrease: float = 0.0
    gain_ratio: float = 0.0
    lam: float = 0.0
    n_obs: int = 0
    n_cams: int = 0
    n_points: int = 0
    rms_px: float = 0.0
    grad_inf: float = 0.0
    rounds: int = 0
    delta: np.ndarray | None = None
    extraction: Extraction | None = None
    extra: dict = field(default_factory=dict)


def candidate(st: State, ex: Extraction, delta: np.ndarray) -> State:
    d = 6 if st.f is None else 7
    nc = d * ex.cams.size
    new = st.copy()
    if ex.cams.size:
        xi = delta[:nc].reshape(-1, d)
        new.q[ex.cams], new.c[ex.cams] = retract_cameras(st.q[ex.cams], st.c[ex.cams],
                                                         xi[:, :6])
        if st.f is not None:
            new.f[ex.cams] = st.f[ex.cams] + xi[:, 6]
    new.X[ex.pts] = st.X[ex.pts] + delta[nc:].reshape(-1, 3)
    return new


def lm_step(prob: Problem, st: State, opts: Options):
    """One LM iteration. Returns (new_state, StepReport)."""
    ex = extract(prob, st, opts)
    rep = StepReport(lam=st.lam, n_obs=int(ex.obs.size), n_cams=int(ex.cams.size),
                     n_points=int(ex.pts.size), rounds=ex.rounds, extraction=ex)
    if ex.obs.size == 0:
        rep.status = "empty"
        return st.copy(), rep
    lin = linearize(prob, st, ex, opts.huber_px)
    H, g = normal_equations(lin)
    F = 0.5 * float(np.sum(lin.rho))
    rep.cost_before = F
    rep.rms_px = float(np.sqrt(np.mean(np.sum(lin.e[:, :2] ** 2, axis=1))))
    rep.grad_inf = float(np.max(np.abs(g))) if g.size else 0.0
    new = st.copy()
    try:
        delta = schur_solve(damped(H, st.lam, opts), -g, lin.ncol_cam)
    except np.linalg.LinAlgError:
        rep.status = "singular"
        new.lam, new.nu = nielsen_update(st.lam, st.nu, False, 0.0, opts.lambda_min,
                                         opts.lambda_max)
        return new, rep
    rep.delta = delta
    Jd = (lin.J @ delta).reshape(lin.e.shape)
    model = -(float(g @ delta) + 0.5 * float(np.sum(lin.w[:, None] * Jd * Jd)))
    rep.model_decrease = model
    cand = candidate(st, ex, delta)
    e2, Xc2, _ = residuals(problem_at(prob, cand), cand.q, cand.c, cand.X, ex.obs)
    if np.any(Xc2[:, 2] <= opts.min_depth):
        F2, dF = np.inf, -np.inf
    else:
        rho2 = huber(np.sum(e2 * e2, axis=1), opts.huber_px)[0]
        F2 = 0.5 * float(np.sum(rho2))
        # actual reduction F(theta) - F(theta (+) delta), summed per observation so that its
        # rounding error scales with the changes rather than with F
        dF = 0.5 * float(np.sum(lin.rho - rho2))
    # reported as F - (per-observation reduction), consistent with the acceptance test
    rep.cost_after = F - dF if np.isfinite(F2) else np.inf
    ratio = dF / model if (model > 0 and np.isfinite(F2)) else -np.inf
    rep.gain_ratio = ratio
    rep.extra["actual_decrease"] = dF
    rep.accepted = bool(np.isfinite(F2) and dF > 0 and ratio > opts.accept_ratio)
    out = cand if rep.accepted else new
    out.lam, out.nu = nielsen_update(st.lam, st.nu, rep.accepted, ratio, opts.lambda_min,
                                     opts.lambda_max)
    return out, rep


def solve(prob: Problem, st: State, opts: Options, max_iters: int | None = None):
    """Iterate LM steps until a stopping rule fires. Returns (state, [StepReport])."""
    reps = []
    for _ in range(opts.max_iters if max_iters is None else max_iters):
        st, rep = lm_step(prob, st, opts)
        reps.append(rep)
        if rep.status == "empty" or rep.grad_inf <= opts.grad_tol:
            break
        if rep.accepted and rep.extra["actual_decrease"] <= opts.cost_rel_tol * rep.cost_before:
            break
        if not rep.accepted and rep.lam >= opts.lambda_max:
            break
    return st, reps
