"""Pins of the oracle's focal-length refinement (the seventh camera parameter).

* de/df by central differences of the residuals in the focal length;
* the 7 x 7-camera Schur + Cholesky solve against a dense solve of the full system;
* the activity fixpoint with 7 rows per camera against brute force on tiny incidences;
* a noise-free scene (float64 observations) with every focal length perturbed by 2 %:
  LM recovers the focal lengths (invariant under the similarity gauge) and the geometry.
"""
import numpy as np
import pytest

from oracle.extract import activity_fixpoint
from oracle.lm import (Options, State, damped, extract, linearize, normal_equations,
                       problem_at, schur_solve, solve)
from oracle.model import Problem, residuals
from scenes import make_scene
from tests._align import aligned_error
from tests.test_oracle_extract import _brute_force_greatest_closed_set, _random_incidence


def _focal_state(sc, opts, scale=1.0):
    return State.initial(sc.cams0, sc.points0, opts, focal=sc.intr[:, 0] * scale)


def test_focal_jacobian_matches_central_differences():
    sc = make_scene("medium", n_cams=12, n_points=300)
    opts = Options(huber_px=2.0, filter_px=4.0, refine_focal=True)
    prob = Problem.from_scene(sc)
    st = _focal_state(sc, opts)
    ex = extract(prob, st, opts)
    lin = linearize(prob, st, ex, opts.huber_px)
    assert lin.Jc.shape[2] == 7
    h = 1e-3
    cams = prob.cam_idx[ex.obs]
    fp, fm = st.copy(), st.copy()
    fp.f = st.f + h
    fm.f = st.f - h
    ep = residuals(problem_at(prob, fp), st.q, st.c, st.X, ex.obs)[0]
    em = residuals(problem_at(prob, fm), st.q, st.c, st.X, ex.obs)[0]
    fd = (ep - em) / (2 * h)          # every observation moves with its own camera's f
    np.testing.assert_allclose(lin.Jc[:, :, 6], fd, rtol=1e-7, atol=1e-10)
    assert np.all(lin.Jc[:, 2, 6] == 0.0) and np.all(cams >= 0)


@pytest.mark.parametrize("lam", [1e-3, 1.0])
def test_focal_schur_equals_dense_solve(lam):
    sc = make_scene("tiny")
    opts = Options(refine_focal=True)
    prob = Problem.from_scene(sc)
    st = _focal_state(sc, opts, 1.01)
    ex = extract(prob, st, opts)
    lin = linearize(prob, st, ex, 0.0)
    H, g = normal_equations(lin)
    assert lin.ncol_cam == 7 * ex.cams.size
    Hd = damped(H, lam, opts)
    x = schur_solve(Hd, -g, lin.ncol_cam)
    ref = np.linalg.solve(Hd.toarray(), -g)
    np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("seed", range(4))
def test_fixpoint_with_seven_rows_per_camera(seed):
    rng = np.random.default_rng(100 + seed)
    prob = _random_incidence(rng, C=4, P=5, N=11, fixed=(0,) if seed % 2 else ())
    valid = rng.random(prob.n_obs) < 0.9
    act, cam_ok, pt_ok, _ = activity_fixpoint(prob, valid, "rows", cam_dim=7)
    ref = _brute_force_greatest_closed_set(prob, valid, 3, 7)
    np.testing.assert_array_equal(act, ref)


def test_noise_free_focal_recovery():
    sc = make_scene("tiny", noise_px=0.0, exact=True)
    opts = Options(refine_focal=True, lambda_init=1e-4, cost_rel_tol=0.0, grad_tol=1e-14,
                   max_iters=80)
    prob = Problem.from_scene(sc)
    st = _focal_state(sc, opts, 1.02)
    st, reps = solve(prob, st, opts)
    np.testing.assert_allclose(st.f, sc.intr[:, 0], rtol=1e-8)
    err, _ = aligned_error(st.cams(), st.X, sc.cams_gt, sc.points_gt)
    assert err < 1e-8, err
    assert reps[-1].rms_px < 1e-6
