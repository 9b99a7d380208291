"""Pins of the oracle's implicit adjoint: tangent mapping by finite differences and the
adjoint by central differences of converged re-solves on noise-free scenes (where the
dropped second-order residual term vanishes)."""
import numpy as np

from oracle.adjoint import adjoint, tangent_gradient
from oracle.geometry import retract_cameras
from oracle.model import Problem
from oracle.lm import Options, State, solve
from scenes import make_scene

rng = np.random.default_rng(11)


def test_tangent_gradient_matches_finite_differences():
    q = rng.normal(size=(5, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    c = rng.normal(size=(5, 3))
    A = rng.normal(size=(5, 7))
    B = rng.normal(size=(5, 7))

    def L(qq, cc):
        z = np.concatenate([qq, cc], axis=1)
        return float(np.sum(A * z) + 0.5 * np.sum(B * z * z))

    gq = A[:, :4] + B[:, :4] * q
    gc = A[:, 4:] + B[:, 4:] * c
    st = State(q=q, c=c, X=np.zeros((1, 3)), lam=0.0)
    gt = tangent_gradient(st, np.arange(5), np.concatenate([gq, gc], axis=1))
    h = 1e-6
    for i in range(5):
        for j in range(6):
            d = np.zeros((1, 6))
            d[0, j] = h
            vals = []
            for s in (1, -1):
                qq, cc = q.copy(), c.copy()
                qq[i:i + 1], cc[i:i + 1] = retract_cameras(q[i:i + 1], c[i:i + 1], s * d)
                vals.append(L(qq, cc))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - gt[i, j]) < 1e-7 * max(1, abs(fd)), (i, j, fd, gt[i, j])


def _adjoint_scene():
    sc = make_scene("tiny", n_points=60, noise_px=0.0, prior_frac=1.0, depth_sigma=0.0,
                    use_depth=True, lambda_d=50.0, exact=True)
    sc.fixed = np.array([0], np.int32)
    return sc


def test_adjoint_matches_central_differences_noise_free():
    sc = _adjoint_scene()
    opts = Options(lambda_init=1e-4, cost_rel_tol=0.0, grad_tol=1e-13, max_iters=60)
    prob = Problem.from_scene(sc)
    st, _ = solve(prob, State.initial(sc.cams0, sc.points0, opts), opts)
    gt_c = sc.cams_gt[:, 4:]
    W = rng.normal(size=sc.points_gt.shape)

    def loss(s):
        return float(np.sum((s.c - gt_c) ** 2) + np.sum(W * s.X))

    grad_cams = np.zeros((sc.n_cams, 7))
    grad_cams[:, 4:] = 2 * (st.c - gt_c)
    gxy, gd, _ = adjoint(prob, st, opts, grad_cams, W)
    # central differences: 1e-3 px for pixels, 1e-4 relative for depths. The re-solves
    # reach the float32 rounding floor of the inputs (gradient noise ~1e-9), which bounds
    # how small the step can be.
    picks = rng.choice(prob.n_obs, size=6, replace=False)
    fds, refs = [], []
    for k in picks:
        for j in range(3):
            h = 1e-3 if j < 2 else 1e-4 / prob.dinv[k]
            vals = []
            for s in (1, -1):
                p2 = Problem.from_scene(sc)
                if j < 2:
                    p2.xy[k, j] += s * h
                else:
                    p2.dinv[k] = 1.0 / (1.0 / prob.dinv[k] + s * h)
                warm = st.copy()
                warm.lam, warm.nu = opts.lambda_init, 2.0     # warm start, fresh damping
                s2, _ = solve(p2, warm, opts)
                vals.append(loss(s2))
            fds.append((vals[0] - vals[1]) / (2 * h))
            refs.append(gxy[k, j] if j < 2 else gd[k])
    fds, refs = np.array(fds), np.array(refs)
    assert np.max(np.abs(fds - refs)) <= 1e-5 * np.max(np.abs(refs)), np.c_[fds, refs]


def test_robust_corrected_metric_is_needed_with_huber():
    """A noisy scene with Huber delta = 1 px (about half the observations in the linear
    regime): central differences of converged re-solves agree with the robust-corrected
    adjoint (rho' I + 2 rho'' e e^T) within a few percent -- the dropped second-order
    residual term -- and much better than with the IRLS metric rho' I alone."""
    import sys
    from dataclasses import replace
    from oracle.lm import extract
    from oracle.model import residuals
    A = sys.modules["oracle.adjoint"]
    rng_l = np.random.default_rng(5)
    sc = make_scene("tiny", n_points=80, noise_px=1.0, prior_frac=1.0, use_depth=True,
                    lambda_d=50.0, exact=True)
    sc = replace(sc, fixed=np.array([0], np.int32), huber_px=1.0)
    opts = Options(huber_px=1.0, lambda_init=1e-4, cost_rel_tol=0.0, grad_tol=0.0,
                   max_iters=400)
    prob = Problem.from_scene(sc)
    st, _ = solve(prob, State.initial(sc.cams0, sc.points0, opts), opts)
    ex = extract(prob, st, opts)
    e, _, _ = residuals(prob, st.q, st.c, st.X, ex.obs)
    s = np.sqrt(np.sum(e * e, axis=1))
    assert np.mean(s > 1.0) > 0.3
    gt_c = sc.cams_gt[:, 4:]
    gcam = np.zeros((sc.n_cams, 7))
    gcam[:, 4:] = 2 * (st.c - gt_c)
    gxy, gd, _ = adjoint(prob, st, opts, gcam, np.zeros_like(st.X))
    # the same solve with the IRLS metric only
    ne, mb = A.normal_equations, A.metric_blocks
    A.normal_equations = lambda lin, robust_correction=False: ne(lin, False)
    A.metric_blocks = lambda lin, robust_correction=False: mb(lin, False)
    try:
        gxy0, gd0, _ = adjoint(prob, st, opts, gcam, np.zeros_like(st.X))
    finally:
        A.normal_equations, A.metric_blocks = ne, mb
    obs = ex.obs[np.abs(s - 1.0) > 0.05]
    e_corr, e_irls = [], []
    for k in rng_l.choice(obs, 4, replace=False):
        for j in (0, 2):
            h = 1e-4 if j < 2 else 1e-5 / prob.dinv[k]
            vals = []
            for sg in (1, -1):
                p2 = Problem.from_scene(sc)
                if j < 2:
                    p2.xy[k, j] += sg * h
                else:
                    p2.dinv[k] = 1.0 / (1.0 / prob.dinv[k] + sg * h)
                warm = st.copy()
                warm.lam, warm.nu = 1e-4, 2.0
                s2, _ = solve(p2, warm, opts)
                vals.append(float(np.sum((s2.c - gt_c) ** 2)))
            fd = (vals[0] - vals[1]) / (2 * h)
            ref = gxy[k, j] if j < 2 else gd[k]
            ref0 = gxy0[k, j] if j < 2 else gd0[k]
            e_corr.append(abs(fd - ref) / abs(fd))
            e_irls.append(abs(fd - ref0) / abs(fd))
    assert np.median(e_corr) < 0.05 and max(e_corr) < 0.15, e_corr
    assert np.median(e_corr) < 0.3 * np.median(e_irls), (e_corr, e_irls)


def test_damped_adjoint_limit_and_effect():
    """The Tikhonov-damped adjoint tends to the exact one as the damping goes to 0 (pinned
    above by central differences), and a finite damping changes it."""
    sc = _adjoint_scene()
    opts = Options(lambda_init=1e-4, cost_rel_tol=0.0, grad_tol=1e-13, max_iters=60)
    prob = Problem.from_scene(sc)
    st, _ = solve(prob, State.initial(sc.cams0, sc.points0, opts), opts)
    grad_cams = np.zeros((sc.n_cams, 7))
    grad_cams[:, 4:] = 2 * (st.c - sc.cams_gt[:, 4:])
    W = rng.normal(size=sc.points_gt.shape)
    ref = adjoint(prob, st, opts, grad_cams, W)[0]
    scale = np.max(np.abs(ref))
    d10 = np.max(np.abs(adjoint(prob, st, opts, grad_cams, W, damping=1e-10)[0] - ref))
    d11 = np.max(np.abs(adjoint(prob, st, opts, grad_cams, W, damping=1e-11)[0] - ref))
    big = adjoint(prob, st, opts, grad_cams, W, damping=1e-1)[0]
    # first-order in the damping: ten times smaller damping, ten times smaller change
    assert d10 <= 1e-6 * scale and 5.0 < d10 / d11 < 20.0, (d10, d11)
    assert np.max(np.abs(big - ref)) >= 1e-3 * scale


# ---------------------------------------------------------------- full Hessian
def _newton_polish(prob, st, opts, iters=2):
    """Newton's method on the exact gradient with the full Hessian: from a point near a
    solution it converges quadratically (two iterations take |g| from ~1e-4 to ~1e-9), where
    LM under IRLS converges only linearly. Used to make re-solves exact for differencing."""
    from oracle.adjoint import full_hessian
    from oracle.lm import candidate, extract, linearize, normal_equations
    s = st.copy()
    for _ in range(iters):
        ex = extract(prob, s, opts)
        g = normal_equations(linearize(prob, s, ex, opts.huber_px))[1]
        s = candidate(s, ex, -np.linalg.solve(full_hessian(prob, s, opts), g))
    return s


def _huber_scene(n_points=40):
    from dataclasses import replace
    sc = make_scene("tiny", n_points=n_points, noise_px=1.0, prior_frac=1.0, use_depth=True,
                    lambda_d=50.0, exact=True)
    return replace(sc, fixed=np.array([0], np.int32), huber_px=1.0)


def test_full_hessian_adjoint_matches_exact_resolves():
    """With the second-order residual term kept (the full Hessian), the implicit gradient
    equals central differences of exact re-solves (Newton-polished) to 1e-5 relative, on a
    noisy scene with a third of its residuals in the Huber regime; the Gauss-Newton adjoint,
    which drops sum rho' e . d^2 e, misses them by 1e-3 to 5e-2. The whole gap of the
    Gauss-Newton adjoint to finite differences is therefore that term."""
    from oracle.lm import extract
    from oracle.model import residuals
    sc = _huber_scene()
    opts = Options(huber_px=1.0, lambda_init=1e-4, cost_rel_tol=0.0, grad_tol=0.0,
                   max_iters=400)
    prob = Problem.from_scene(sc)
    st, _ = solve(prob, State.initial(sc.cams0, sc.points0, opts), opts)
    st = _newton_polish(prob, st, opts)
    ex = extract(prob, st, opts)
    e, _, _ = residuals(prob, st.q, st.c, st.X, ex.obs)
    s = np.sqrt(np.sum(e * e, axis=1))
    assert np.mean(s > 1.0) > 0.2
    gt_c = sc.cams_gt[:, 4:]
    gcam = np.zeros((sc.n_cams, 7))
    gcam[:, 4:] = 2 * (st.c - gt_c)
    zero = np.zeros_like(st.X)
    gxy, gd, _ = adjoint(prob, st, opts, gcam, zero)
    gxyF, gdF, _ = adjoint(prob, st, opts, gcam, zero, hessian="full")
    rng_l = np.random.default_rng(5)
    e_full, e_gn = [], []
    for k in rng_l.choice(ex.obs[np.abs(s - 1.0) > 0.05], 4, replace=False):
        for j in (0, 2):
            h = 1e-3 if j < 2 else 1e-4 / prob.dinv[k]
            vals = []
            for sg in (1, -1):
                p2 = Problem.from_scene(sc)
                if j < 2:
                    p2.xy[k, j] += sg * h
                else:
                    p2.dinv[k] = 1.0 / (1.0 / prob.dinv[k] + sg * h)
                s2 = _newton_polish(p2, st, opts)
                vals.append(float(np.sum((s2.c - gt_c) ** 2)))
            fd = (vals[0] - vals[1]) / (2 * h)
            e_full.append(abs(fd - (gxyF[k, j] if j < 2 else gdF[k])) / abs(fd))
            e_gn.append(abs(fd - (gxy[k, j] if j < 2 else gd[k])) / abs(fd))
    assert max(e_full) < 1e-5, e_full
    assert np.median(e_gn) > 1e-3 and max(e_gn) > 1e-2, e_gn


def test_lm_resolve_floor_on_adjoint_subscene():
    """On a ten-camera sub-scene of the adjoint workload (Huber 2 px, 4 px filter, metric
    depth rows, camera 0 fixed) differences of Newton-polished re-solves match the
    full-Hessian adjoint to 1e-5, while differences of LM re-solves (the GPU's solver, which
    stops when its steps no longer lower the cost measurably) are off by up to a few
    percent: the floor of finite-difference checks made with LM re-solves."""
    from oracle.lm import extract
    from scenes import subscene
    sc = subscene(make_scene("adjoint"), np.arange(10), max_points=120, seed=1)
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px, cost_rel_tol=0.0,
                   grad_tol=0.0, max_iters=300, lambda_init=1e-4)
    prob = Problem.from_scene(sc)
    st, _ = solve(prob, State.initial(sc.cams0, sc.points0, opts), opts)
    stn = _newton_polish(prob, st, opts, iters=3)
    gt_c = sc.cams_gt[:, 4:]
    gcam = np.zeros((sc.n_cams, 7))
    gcam[:, 4:] = 2 * (stn.c - gt_c)
    gxy, gd, _ = adjoint(prob, stn, opts, gcam, np.zeros_like(stn.X), hessian="full")
    ex = extract(prob, stn, opts)
    k = int(ex.obs[~sc.is_outlier[ex.obs]][7])
    e_newton, e_lm = [], []
    for j in (0, 2):
        h = 1e-3 if j < 2 else 1e-4 / prob.dinv[k]
        vn, vl = [], []
        for sg in (1, -1):
            p2 = Problem.from_scene(sc)
            if j < 2:
                p2.xy[k, j] += sg * h
            else:
                p2.dinv[k] = 1.0 / (1.0 / prob.dinv[k] + sg * h)
            vn.append(float(np.sum((_newton_polish(p2, stn, opts).c - gt_c) ** 2)))
            warm = stn.copy()
            warm.lam, warm.nu = 1e-4, 2.0
            vl.append(float(np.sum((solve(p2, warm, opts)[0].c - gt_c) ** 2)))
        ref = gxy[k, j] if j < 2 else gd[k]
        e_newton.append(abs((vn[0] - vn[1]) / (2 * h) - ref) / abs(ref))
        e_lm.append(abs((vl[0] - vl[1]) / (2 * h) - ref) / abs(ref))
    print(f"sub-scene: Newton re-solves {e_newton}, LM re-solves {e_lm}")
    assert max(e_newton) < 1e-5, e_newton
    assert max(e_lm) > 1e-4, e_lm
