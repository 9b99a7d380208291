"""Pins of the oracle's LM step: brute-force dense solve, closed-form model decrease,
exact recovery of noise-free scenes (up to gauge), metric scale from exact depth priors,
monotone cost."""
import numpy as np
import pytest

from oracle.model import Problem
from oracle.lm import (Options, State, lm_step, solve, extract, linearize, normal_equations,
                       schur_solve, damped)
from scenes import make_scene
from tests._align import aligned_error, rotation_error


def _system(sc, opts, **kw):
    prob = Problem.from_scene(sc, **kw)
    st = State.initial(sc.cams0, sc.points0, opts)
    ex = extract(prob, st, opts)
    lin = linearize(prob, st, ex, opts.huber_px)
    H, g = normal_equations(lin)
    return prob, st, ex, lin, H, g


@pytest.mark.parametrize("lam", [1e-3, 1.0])
def test_schur_cholesky_equals_dense_solve(lam):
    sc = make_scene("tiny")
    opts = Options()
    prob, st, ex, lin, H, g = _system(sc, opts)
    Hd = damped(H, lam, opts)
    x = schur_solve(Hd, -g, lin.ncol_cam)
    ref = np.linalg.solve(Hd.toarray(), -g)
    np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_schur_with_depth_rows_and_fixed_camera():
    sc = make_scene("medium", n_cams=15, n_points=400)
    sc.fixed = np.array([0, 3], np.int32)
    opts = Options(huber_px=2.0, filter_px=4.0)
    prob, st, ex, lin, H, g = _system(sc, opts)
    assert not ex.cam_active[[0, 3]].any()
    Hd = damped(H, 1e-2, opts)
    x = schur_solve(Hd, -g, lin.ncol_cam)
    ref = np.linalg.solve(Hd.toarray(), -g)
    np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_model_decrease_closed_form():
    """For an exact solve of (H + lam D) d = -g: -(g.d + d.H.d/2) = d.H.d/2 + lam d.D.d."""
    sc = make_scene("tiny")
    opts = Options(lambda_init=0.05)
    prob = Problem.from_scene(sc)
    st = State.initial(sc.cams0, sc.points0, opts)
    _, rep = lm_step(prob, st, opts)
    ex = rep.extraction
    lin = linearize(prob, st, ex, 0.0)
    H, g = normal_equations(lin)
    d = rep.delta
    D = np.clip(H.diagonal(), opts.diag_min, opts.diag_max)
    ref = 0.5 * d @ (H @ d) + 0.05 * d @ (D * d)
    np.testing.assert_allclose(rep.model_decrease, ref, rtol=1e-9)


def test_noise_free_recovers_ground_truth_up_to_similarity():
    sc = make_scene("tiny", noise_px=0.0, exact=True)
    opts = Options()
    prob = Problem.from_scene(sc)
    st, reps = solve(prob, State.initial(sc.cams0, sc.points0, opts), opts)
    final = min(r.cost_after if r.accepted else r.cost_before for r in reps)
    assert final < 1e-20
    costs = [r.cost_after for r in reps if r.accepted]
    assert all(b < a for a, b in zip(costs, costs[1:]))
    err, (s, R, t) = aligned_error(st.cams(), st.X, sc.cams_gt, sc.points_gt)
    assert err < 1e-8
    assert rotation_error(st.cams(), sc.cams_gt, R) < 1e-8


def test_exact_depth_priors_fix_metric_scale():
    """Without priors the scale is free; exact priors pin it to 1 (Sec. IV-A)."""
    sc = make_scene("tiny", noise_px=0.0, prior_frac=1.0, depth_sigma=0.0, use_depth=True,
                    lambda_d=2.0, trans_m=0.2, point_m=0.2, exact=True)
    opts = Options()
    prob = Problem.from_scene(sc)
    st, _ = solve(prob, State.initial(sc.cams0, sc.points0, opts), opts)
    err, (s, R, t) = aligned_error(st.cams(), st.X, sc.cams_gt, sc.points_gt, with_scale=True)
    assert abs(s - 1.0) < 1e-9 and err < 1e-8
    # rigid alignment alone suffices
    err_rigid, _ = aligned_error(st.cams(), st.X, sc.cams_gt, sc.points_gt, with_scale=False)
    assert err_rigid < 1e-8


def test_monotone_cost_and_report_consistency_medium():
    sc = make_scene("medium")
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px)
    prob = Problem.from_scene(sc)
    st = State.initial(sc.cams0, sc.points0, opts)
    prev = None
    for _ in range(6):
        st2, rep = lm_step(prob, st, opts)
        if rep.accepted:
            assert rep.cost_after < rep.cost_before
            assert rep.gain_ratio > opts.accept_ratio
            assert st2.lam < rep.lam * 1.0000001
        else:
            assert st2.lam > rep.lam
            np.testing.assert_array_equal(st2.X, st.X)
        st = st2
