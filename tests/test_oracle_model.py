"""Pins of the oracle's residual model: closed forms, finite differences, Huber identities."""
import numpy as np
import pytest

from oracle.geometry import retract_cameras
from oracle.model import Problem, residuals, jacobians, huber, cost
from oracle.lm import Options, State, extract, linearize, normal_equations
from scenes import make_scene

rng = np.random.default_rng(7)


def _one_obs_problem(X, q, c, f=500.0, cx=320.0, cy=240.0, xy=(0.0, 0.0), d_hat=None,
                     lam=0.0):
    m = d_hat is not None and d_hat > 0
    return Problem(n_cams=1, n_points=1, intr=np.array([[f, cx, cy]]),
                   cam_idx=np.array([0]), pt_idx=np.array([0]), xy=np.array([xy], float),
                   dinv=np.array([1.0 / d_hat if m else 0.0]), prior_mask=np.array([m]),
                   lambda_d=lam, img_w=640, img_h=480)


def test_projection_and_depth_residual_closed_form():
    """Identity camera at the origin: Pi = (f x/z + cx, f y/z + cy); r^d = 1/z - m/d_hat."""
    X = np.array([[0.4, -0.3, 2.5]])
    q = np.array([[1.0, 0, 0, 0]])
    c = np.zeros((1, 3))
    prob = _one_obs_problem(X, q, c, xy=(300.0, 200.0), d_hat=2.0, lam=3.0)
    e, Xc, _ = residuals(prob, q, c, X)
    np.testing.assert_allclose(Xc, X)
    np.testing.assert_allclose(e[0], [500 * 0.4 / 2.5 + 320 - 300, 500 * -0.3 / 2.5 + 240 - 200,
                                      3.0 * (1 / 2.5 - 1 / 2.0)], rtol=1e-15)
    # invalid prior: the row stays, with reference inverse depth 0 (Eq. (9))
    prob2 = _one_obs_problem(X, q, c, xy=(300.0, 200.0), d_hat=None, lam=3.0)
    e2, _, _ = residuals(prob2, q, c, X)
    assert e2.shape == (1, 3)
    np.testing.assert_allclose(e2[0, 2], 3.0 / 2.5, rtol=1e-15)


def test_camera_translation_closed_form():
    """A camera at centre c with identity rotation sees X - c."""
    q = np.array([[1.0, 0, 0, 0]])
    c = np.array([[1.0, 2.0, -3.0]])
    X = np.array([[1.5, 1.0, 1.0]])
    prob = _one_obs_problem(X, q, c, xy=(0.0, 0.0))
    e, Xc, _ = residuals(prob, q, c, X)
    np.testing.assert_allclose(Xc[0], [0.5, -1.0, 4.0])
    np.testing.assert_allclose(e[0], [500 * 0.5 / 4 + 320, 500 * -1.0 / 4 + 240])


@pytest.mark.parametrize("lam", [0.0, 2.0])
def test_jacobians_match_central_differences(lam):
    sc = make_scene("tiny", noise_px=0.5)
    prob = Problem.from_scene(sc, use_depth=lam > 0, lambda_d=lam)
    prob.prior_mask[:] = True
    prob.dinv = 1.0 / sc.depth.astype(np.float64)
    q, c, X = sc.cams0[:, :4].copy(), sc.cams0[:, 4:].copy(), sc.points0.copy()
    obs = rng.choice(prob.n_obs, size=40, replace=False)
    e, Xc, R = residuals(prob, q, c, X, obs)
    Jc, Jp = jacobians(prob, Xc, R, prob.cam_idx[obs])
    h = 1e-6
    for k, o in enumerate(obs):
        ci, pi = prob.cam_idx[o], prob.pt_idx[o]
        for j in range(6):
            d = np.zeros((1, 6))
            d[0, j] = h
            qp, cp = q.copy(), c.copy()
            qm, cm = q.copy(), c.copy()
            qp[ci:ci + 1], cp[ci:ci + 1] = retract_cameras(q[ci:ci + 1], c[ci:ci + 1], d)
            qm[ci:ci + 1], cm[ci:ci + 1] = retract_cameras(q[ci:ci + 1], c[ci:ci + 1], -d)
            fd = (residuals(prob, qp, cp, X, [o])[0] - residuals(prob, qm, cm, X, [o])[0]) / (2 * h)
            np.testing.assert_allclose(Jc[k, :, j], fd[0], rtol=1e-6, atol=1e-6 * np.abs(Jc[k]).max())
        for j in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[pi, j] += h
            Xm[pi, j] -= h
            fd = (residuals(prob, q, c, Xp, [o])[0] - residuals(prob, q, c, Xm, [o])[0]) / (2 * h)
            np.testing.assert_allclose(Jp[k, :, j], fd[0], rtol=1e-6, atol=1e-6 * np.abs(Jp[k]).max())


def test_huber_identities():
    delta = 2.0
    s = np.linspace(0.0, 30.0, 3001)
    rho, d1, d2 = huber(s, delta)
    # continuity of value and slope at the kink s = delta^2
    r0, g0, _ = huber(np.array([delta ** 2 - 1e-9, delta ** 2 + 1e-9]), delta)
    assert abs(r0[0] - r0[1]) < 1e-8 and abs(g0[0] - g0[1]) < 1e-8
    # derivatives by central differences away from the kink
    h = 1e-5
    mask = np.abs(s - delta ** 2) > 1e-3
    mask &= s > 1e-3
    fd1 = (huber(s + h, delta)[0] - huber(s - h, delta)[0]) / (2 * h)
    fd2 = (huber(s + h, delta)[1] - huber(s - h, delta)[1]) / (2 * h)
    np.testing.assert_allclose(d1[mask], fd1[mask], rtol=1e-8, atol=1e-9)
    np.testing.assert_allclose(d2[mask], fd2[mask], rtol=1e-5, atol=1e-9)
    # linear growth in the norm: rho(s) = 2 delta |e| - delta^2 above the kink
    np.testing.assert_allclose(rho[s > 4], 2 * delta * np.sqrt(s[s > 4]) - 4)
    # disabled robustifier is plain least squares
    r, w, dd = huber(s, 0.0)
    np.testing.assert_array_equal(r, s)
    assert np.all(w == 1) and np.all(dd == 0)


def test_gradient_is_derivative_of_cost():
    """g = sum rho' J^T e is the gradient of F = 1/2 sum rho(|e|^2): pins the weights, the
    factor 1/2 and the tangent convention together."""
    sc = make_scene("medium", n_cams=12, n_points=300)
    prob = Problem.from_scene(sc)
    opts = Options(huber_px=2.0, filter_px=0.0)
    st = State.initial(sc.cams0, sc.points0, opts)
    ex = extract(prob, st, opts)
    lin = linearize(prob, st, ex, opts.huber_px)
    H, g = normal_equations(lin)
    obs = ex.obs
    nc = 6 * ex.cams.size
    h = 1e-6
    for col in list(rng.choice(nc, 8, replace=False)) + list(nc + rng.choice(g.size - nc, 8, replace=False)):
        d = np.zeros(g.size)
        d[col] = h
        vals = []
        for sgn in (1, -1):
            s2 = st.copy()
            if col < nc:
                xi = (sgn * d[:nc]).reshape(-1, 6)
                s2.q[ex.cams], s2.c[ex.cams] = retract_cameras(st.q[ex.cams], st.c[ex.cams], xi)
            else:
                s2.X[ex.pts] += (sgn * d[nc:]).reshape(-1, 3)
            vals.append(cost(prob, s2.q, s2.c, s2.X, obs, opts.huber_px))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[col]) <= 1e-5 * max(1.0, abs(g[col])), (col, fd, g[col])
