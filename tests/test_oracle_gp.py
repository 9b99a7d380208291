"""Pins of the oracle's depth-constrained global positioning (Eqs. (1), (4), (5), (8)).

* rays: unit length, and the camera-frame direction reprojects onto the observed pixel;
* the residual vanishes at the ground truth of a noise-free scene with exact priors, for
  pinned scales 1 / (d_hat |a|) and for free scales 1 / |X - c| (closed form);
* the Jacobian columns (centre, point, free scale) against central differences;
* the scale-then-point elimination against a dense solve of the whole damped system;
* the GP activity fixpoint (3 rows pinned, 2 free; points and cameras need 3) against brute
  force over all observation subsets of tiny incidences;
* noise-free recovery: from centres and points at 1.5x the true scale and perturbed, with
  half the scales free, GP converges to the ground truth itself (pinned priors fix the
  metric scale, one fixed camera the translation); accepted steps never raise the cost;
* without any pinned prior the same start converges to a similarity of the truth at about
  the starting scale, so the metric information comes from the pinned rows.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle.geometry import quat_to_rot
from oracle.gp import (GpOptions, GpState, gp_damped, gp_extract, gp_linearize,
                       gp_normal_equations, gp_residuals, gp_solve, gp_solve_system, gp_step,
                       rays)
from oracle.model import Problem, huber
from scenes import make_scene
from tests._align import aligned_error
from tests._constructed import gp_behind_scene
from tests.test_oracle_extract import _brute_force_greatest_closed_set, _random_incidence


def _exact_scene(prior_frac=0.5, **kw):
    return make_scene("tiny", noise_px=0.0, exact=True, depth_sigma=0.0, prior_frac=prior_frac,
                      use_depth=True, lambda_d=1.0, n_points=250, **kw)


def _gt_state(sc, prob):
    q = sc.cams_gt[:, :4]
    st = GpState.initial(prob, q, sc.cams_gt, sc.points_gt, GpOptions())
    return q, st


def test_rays_unit_and_reproject():
    sc = _exact_scene()
    prob = Problem.from_scene(sc)
    q = sc.cams_gt[:, :4]
    v, na = rays(prob, q)
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, rtol=1e-14)
    R = quat_to_rot(q)[prob.cam_idx]
    a = np.einsum("nij,nj->ni", R, v)            # camera-frame direction
    f, cx, cy = prob.intr[prob.cam_idx].T
    np.testing.assert_allclose(f * a[:, 0] / a[:, 2] + cx, prob.xy[:, 0], atol=1e-9)
    np.testing.assert_allclose(f * a[:, 1] / a[:, 2] + cy, prob.xy[:, 1], atol=1e-9)
    np.testing.assert_allclose(na, 1.0 / a[:, 2] * 1.0, rtol=1e-12)   # |a| = 1 / cos


def test_residual_vanishes_at_ground_truth():
    sc = _exact_scene()
    prob = Problem.from_scene(sc)
    q, st = _gt_state(sc, prob)
    assert prob.prior_mask.any() and (~prob.prior_mask).any()
    u, d = gp_residuals(prob, q, st, np.arange(prob.n_obs))
    assert np.max(np.abs(u)) < 1e-12
    # the pinned scale is the inverse distance along the ray
    m = prob.prior_mask
    np.testing.assert_allclose(st.s[m], 1.0 / np.linalg.norm(d[m], axis=1), rtol=1e-12)


def test_jacobian_matches_central_differences():
    sc = make_scene("tiny", prior_frac=0.5, use_depth=True, lambda_d=1.0)
    prob = Problem.from_scene(sc)
    q = sc.cams_gt[:, :4]
    st = GpState.initial(prob, q, sc.cams0, sc.points0, GpOptions())
    ex = gp_extract(prob)
    lin = gp_linearize(prob, q, st, ex, 0.0)
    J = lin.J.toarray()
    h = 1e-6
    cols = []
    for (arr, idx, k) in [("c", ex.cams[1], 0), ("c", ex.cams[3], 2), ("X", ex.pts[5], 1),
                          ("X", ex.pts[77], 2), ("s", ex.free[4], None), ("s", ex.free[9], None)]:
        sp_, sm = st.copy(), st.copy()
        if arr == "s":
            sp_.s[idx] += h
            sm.s[idx] -= h
            col = 3 * ex.cams.size + 3 * ex.pts.size + ex.free_rank[idx]
        else:
            getattr(sp_, arr)[idx, k] += h
            getattr(sm, arr)[idx, k] -= h
            col = (3 * ex.cam_rank[idx] + k if arr == "c"
                   else 3 * ex.cams.size + 3 * ex.pt_rank[idx] + k)
        up, _ = gp_residuals(prob, q, sp_, ex.obs)
        um, _ = gp_residuals(prob, q, sm, ex.obs)
        fd = ((up - um) / (2 * h)).ravel()
        np.testing.assert_allclose(J[:, col], fd, rtol=1e-6, atol=1e-9)
        cols.append(col)
    assert len(set(cols)) == len(cols)


@pytest.mark.parametrize("lam", [1e-4, 1.0])
def test_elimination_equals_dense_solve(lam):
    sc = make_scene("tiny", prior_frac=0.5, use_depth=True, lambda_d=1.0, n_points=150)
    prob = Problem.from_scene(sc)
    q = sc.cams_gt[:, :4]
    st = GpState.initial(prob, q, sc.cams0, sc.points0, GpOptions())
    ex = gp_extract(prob)
    lin = gp_linearize(prob, q, st, ex, 0.1)
    H, g = gp_normal_equations(lin)
    Hd = gp_damped(H, lam, GpOptions())
    x = gp_solve_system(Hd, -g, lin.ncol_cam, lin.ncol_pt)
    ref = np.linalg.solve(Hd.toarray(), -g)
    np.testing.assert_allclose(x, ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("seed", range(6))
def test_gp_fixpoint_equals_brute_force(seed):
    rng = np.random.default_rng(200 + seed)
    prob = _random_incidence(rng, C=4, P=6, N=12, fixed=(0,) if seed % 2 else ())
    ex = gp_extract(prob)
    valid = np.ones(prob.n_obs, bool)
    ref = _brute_force_greatest_closed_set(prob, valid, 3, 3)   # rows: 3 pinned, 2 free
    np.testing.assert_array_equal(ex.obs_active, ref)
    np.testing.assert_array_equal(ex.free, np.nonzero(ref & ~prob.prior_mask)[0])


def _perturbed_start(sc, rng, zoom):
    """Ground-truth rotations; centres and points scaled by ``zoom`` about camera 0's centre,
    then perturbed by 0.3 (scene units)."""
    q = sc.cams_gt[:, :4]
    o = sc.cams_gt[0, 4:7]
    cams = sc.cams_gt.copy()
    cams[:, 4:7] = o + zoom * (cams[:, 4:7] - o) + 0.3 * rng.standard_normal((sc.n_cams, 3))
    cams[0, 4:7] = o
    pts = o + zoom * (sc.points_gt - o) + 0.3 * rng.standard_normal(sc.points_gt.shape)
    return q, cams, pts


def _solve_from(sc, zoom, seed):
    sc.fixed = np.array([0], np.int32)
    prob = Problem.from_scene(sc)
    q, cams, pts = _perturbed_start(sc, np.random.default_rng(seed), zoom)
    opts = GpOptions(huber=0.0, cost_rel_tol=1e-16, grad_tol=1e-13, max_iters=60)
    st = GpState.initial(prob, q, cams, pts, opts)
    return prob, q, gp_solve(prob, q, st, opts)


def test_noise_free_recovery_metric():
    """Half the scales pinned, start at 1.5x the true scale: GP returns to the truth."""
    sc = _exact_scene(prior_frac=0.5)
    prob, q, (st, reps) = _solve_from(sc, 1.5, 7)
    costs = [r.cost_before for r in reps if r.accepted]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    assert reps[-1].rms < 1e-9, reps[-1].rms
    np.testing.assert_allclose(st.X, sc.points_gt, atol=1e-7)
    np.testing.assert_allclose(st.c, sc.cams_gt[:, 4:7], atol=1e-7)


def test_without_priors_scale_stays_free():
    """No pinned scale, same start: GP fits the data exactly at the starting scale (a
    similarity of the truth), so the metric scale above came from the pinned rows."""
    sc = _exact_scene(prior_frac=0.0)
    prob, q, (st, reps) = _solve_from(sc, 1.5, 7)
    assert not prob.prior_mask.any()
    assert reps[-1].rms < 1e-8
    est = np.concatenate([q, st.c], axis=1)
    err_sim, (s, R, t) = aligned_error(est, st.X, sc.cams_gt, sc.points_gt)
    assert err_sim < 1e-6
    assert abs(s - 1.0 / 1.5) < 0.05, s


# ---------------------------------------------------------------- Huber-weighted system
def _huber_system(huber_t):
    sc = replace(make_scene("tiny", prior_frac=0.5, use_depth=True, lambda_d=1.0, n_points=150),
                 fixed=np.array([0], np.int32))
    prob = Problem.from_scene(sc)
    q = sc.cams_gt[:, :4]
    opts = GpOptions(huber=huber_t)
    st = GpState.initial(prob, q, sc.cams0, sc.points0, opts)
    ex = gp_extract(prob)
    lin = gp_linearize(prob, q, st, ex, huber_t)
    return prob, q, opts, st, ex, lin


def _gp_cost(prob, q, st, obs, huber_t):
    u, _ = gp_residuals(prob, q, st, obs)
    return 0.5 * float(np.sum(huber(np.sum(u * u, axis=1), huber_t)[0]))


def test_huber_gradient_is_derivative_of_cost():
    """g = J^T W u is the gradient of F = 1/2 sum rho(|u|^2) (Eq. (1) with Huber): central
    differences of the cost over camera centres, points and free scales, with residuals on
    both sides of the threshold (a missing, squared or misplaced weight fails here)."""
    ht = 0.012
    prob, q, opts, st, ex, lin = _huber_system(ht)
    assert (lin.w < 1).sum() > 50 and (lin.w == 1).sum() > 50   # both Huber regimes
    H, g = gp_normal_equations(lin)
    nc, npt = 3 * ex.cams.size, 3 * ex.pts.size
    h = 1e-6
    coords = ([("c", i, k) for i in ex.cams for k in range(3)] +
              [("X", j, k) for j in ex.pts[::7] for k in range(3)] +
              [("s", o, None) for o in ex.free[::13]])
    for arr, idx, k in coords:
        sp_, sm = st.copy(), st.copy()
        if arr == "s":
            sp_.s[idx] += h
            sm.s[idx] -= h
            col = nc + npt + ex.free_rank[idx]
        else:
            getattr(sp_, arr)[idx, k] += h
            getattr(sm, arr)[idx, k] -= h
            col = 3 * ex.cam_rank[idx] + k if arr == "c" else nc + 3 * ex.pt_rank[idx] + k
        fd = (_gp_cost(prob, q, sp_, ex.obs, ht) - _gp_cost(prob, q, sm, ex.obs, ht)) / (2 * h)
        assert abs(g[col] - fd) <= 1e-6 * abs(fd) + 1e-8 * np.abs(g).max(), (arr, idx, k)


def test_irls_step_is_weighted_least_squares():
    """The undamped IRLS step solves min_d sum_k w_k |u_k + J_k d|^2: the normal equations
    H = J^T W J, g = J^T W u must give the same step as a QR least-squares solve of the
    sqrt(w)-scaled Jacobian (camera 0 fixed, pinned scales fix the metric scale)."""
    prob, q, opts, st, ex, lin = _huber_system(0.012)
    H, g = gp_normal_equations(lin)
    x = gp_solve_system(gp_damped(H, 0.0, opts), -g, lin.ncol_cam, lin.ncol_pt)
    sw = np.repeat(np.sqrt(lin.w), 3)
    A = lin.J.toarray() * sw[:, None]
    ref, *_ = np.linalg.lstsq(A, -sw * lin.u.ravel(), rcond=None)
    np.testing.assert_allclose(x, ref, rtol=1e-7, atol=1e-8 * np.abs(ref).max())


# ---------------------------------------------------------------- free scale <= 0
def test_candidate_with_nonpositive_free_scale_rejected():
    """A point 2 m behind a fixed camera that sees it at its principal point: that free
    scale's own optimum is -0.5 from a start of 0.5, so the lightly damped candidate takes it
    below 0 and the step is rejected with an infinite cost; as the damping grows a step is
    accepted and every free scale stays positive."""
    sc = gp_behind_scene()
    prob = Problem.from_scene(sc)
    q = sc.cams0[:, :4]
    opts = GpOptions(huber=0.0)
    st = GpState.initial(prob, q, sc.cams0, sc.points0, opts)
    k = sc.n_obs - int((sc.pt_idx == sc.n_points - 1).sum())   # camera 0's observation
    assert sc.cam_idx[k] == 0 and not prob.prior_mask[k]
    assert st.s[k] == pytest.approx(0.5, rel=0.02)   # the start centre is perturbed by 2 cm
    decisions = []
    for _ in range(8):
        st2, rep = gp_step(prob, q, st, opts)
        ex = rep.extraction
        assert ex.obs_active[k]
        s_cand = st.s[k] + rep.delta[3 * ex.cams.size + 3 * ex.pts.size + ex.free_rank[k]]
        if s_cand <= 0:
            assert not rep.accepted and rep.cost_after == np.inf
            np.testing.assert_array_equal(st2.s, st.s)
        decisions.append(rep.accepted)
        st = st2
    assert decisions[0] is False and any(decisions)
    assert (st.s > 0).all()
