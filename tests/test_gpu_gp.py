"""GPU parity of depth-constrained global positioning (Eqs. (1), (4), (5), (8)) against the FP64
oracle (``oracle/gp.py``), through the C ABI.

Scenes keep the true rotations (GP takes them from rotation averaging) with perturbed centres
and points; half of the depth priors are valid (pinned scales), the rest of the scales are
free. Tolerances: active sets bit-exact; initial scales 1e-12 relative; one step against the
oracle's direct solve 1e-6 relative (PCG to 1e-13); ten fixed-gauge steps with the same
accept decisions, costs within 1e-9 relative and parameters within 1e-6; the mixed path
follows FP64 within 1e-6 relative in cost. At the 1000-camera workload: extraction bit-exact,
the cost before the step and the candidate cost after it equal the oracle's cost evaluated
at the same parameters (1e-10 relative).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle.gp import GpOptions, GpState, gp_extract, gp_residuals, gp_step, gp_solve
from oracle.model import Problem, huber
from scenes import make_scene
from tests._common import gpu_setup, rel_err

pytestmark = pytest.mark.gpu

_SC = {}


def gp_scene(name, **kw):
    """The named scene with true rotations in the starting cameras and 50 % valid priors."""
    key = (name, tuple(sorted(kw.items())))
    if key not in _SC:
        kw = dict(dict(prior_frac=0.5, use_depth=True, lambda_d=1.0), **kw)
        sc = make_scene(name, **kw)
        cams0 = np.concatenate([sc.cams_gt[:, :4], sc.cams0[:, 4:7]], axis=1)
        _SC[key] = replace(sc, cams0=cams0)
    return _SC[key]


def oracle_gp(sc, **kw):
    opts = GpOptions(**kw)
    prob = Problem.from_scene(sc)
    q = sc.cams0[:, :4]
    return prob, q, opts, GpState.initial(prob, q, sc.cams0, sc.points0, opts)


def gpu_gp(sc, precision, **kw):
    base = dict(gp_huber=0.1, pcg_rel_tol=1e-13, pcg_max_iters=3000)
    base.update(kw)
    return gpu_setup(sc, precision, **base)


def _params(ba):
    cams, pts = ba.get_params()
    return cams[:, 4:7], pts, ba.gp_scales()


def test_gp_extraction_and_initial_scales():
    sc = gp_scene("medium")
    prob, q, opts, st = oracle_gp(sc)
    ex = gp_extract(prob)
    ba = gpu_gp(sc, "fp64")
    np.testing.assert_allclose(ba.gp_scales(), st.s, rtol=1e-12)
    rep = ba.gp_step()
    ac, ap, ao = ba.get_active()
    np.testing.assert_array_equal(ao, ex.obs_active)
    np.testing.assert_array_equal(ac, ex.cam_active)
    np.testing.assert_array_equal(ap, ex.pt_active)
    assert rep["n_obs_active"] == ex.obs.size and rep["fixpoint_rounds"] == ex.rounds


@pytest.mark.parametrize("name,lam", [("tiny", 1e-3), ("medium", 1e-2), ("medium", 1.0)])
def test_gp_single_step_matches_oracle(name, lam):
    sc = replace(gp_scene(name), fixed=np.array([0], np.int32))
    prob, q, opts, st = oracle_gp(sc, lambda_init=lam)
    new, orep = gp_step(prob, q, st, opts)
    ba = gpu_gp(sc, "fp64", lambda_init=lam)
    rep = ba.gp_step()
    assert abs(rep["cost_before"] - orep.cost_before) <= 1e-12 * orep.cost_before
    assert abs(rep["model_decrease"] - orep.model_decrease) <= 1e-6 * abs(orep.model_decrease)
    assert bool(rep["accepted"]) == orep.accepted
    if orep.accepted:
        assert abs(rep["cost_after"] - orep.cost_after) <= 1e-9 * orep.cost_before
    c, X, s = _params(ba)
    print(f"{name} lam {lam}: centres {rel_err(c, new.c):.2e}, points {rel_err(X, new.X):.2e}, "
          f"scales {rel_err(s, new.s):.2e}")
    assert rel_err(c - st.c, new.c - st.c) < 1e-6
    assert rel_err(X - st.X, new.X - st.X) < 1e-6
    assert rel_err(s - st.s, new.s - st.s) < 1e-6


def test_gp_trajectory_fp64_fixed_gauge():
    sc = replace(gp_scene("medium"), fixed=np.array([0], np.int32))
    prob, q, opts, st = oracle_gp(sc)
    ba = gpu_gp(sc, "fp64")
    for k in range(10):
        st, orep = gp_step(prob, q, st, opts)
        rep = ba.gp_step()
        assert bool(rep["accepted"]) == orep.accepted, k
        assert abs(rep["cost_before"] - orep.cost_before) <= 1e-9 * orep.cost_before, k
    c, X, s = _params(ba)
    d = max(rel_err(c, st.c), rel_err(X, st.X), rel_err(s, st.s))
    print(f"GP trajectory: max rel diff {d:.3e}, final rms {orep.rms:.3e}")
    assert d < 1e-6


def test_gp_mixed_follows_fp64():
    sc = replace(gp_scene("medium"), fixed=np.array([0], np.int32))
    runs = {}
    for prec in ("fp64", "mixed"):
        ba = gpu_gp(sc, prec, pcg_rel_tol=1e-8, pcg_max_iters=500)
        runs[prec] = [ba.gp_step() for _ in range(6)]
    for k, (a, b) in enumerate(zip(runs["fp64"], runs["mixed"])):
        print(f"GP step {k}: cost fp64 {a['cost_before']:.9e} mixed {b['cost_before']:.9e}")
        assert abs(a["cost_before"] - b["cost_before"]) <= 1e-6 * a["cost_before"], k
        assert a["accepted"] == b["accepted"], k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gp_metric_recovery_noise_free(precision):
    """Noise-free pixels (float32) and exact priors on half the observations, centres and
    points started at 1.5x the true scale: GP returns to the metric truth, as the oracle."""
    sc = gp_scene("tiny", noise_px=0.0, depth_sigma=0.0, n_points=250)
    o = sc.cams_gt[0, 4:7]
    rng = np.random.default_rng(7)
    cams0 = sc.cams0.copy()
    cams0[:, 4:7] = o + 1.5 * (sc.cams_gt[:, 4:7] - o) + 0.3 * rng.standard_normal((sc.n_cams, 3))
    cams0[0, 4:7] = o
    pts0 = o + 1.5 * (sc.points_gt - o) + 0.3 * rng.standard_normal(sc.points_gt.shape)
    sc = replace(sc, cams0=cams0, points0=pts0, fixed=np.array([0], np.int32))
    prob, q, opts, st = oracle_gp(sc, huber=0.0, cost_rel_tol=1e-16, grad_tol=1e-13,
                                  max_iters=60)
    st, reps = gp_solve(prob, q, st, opts)
    ba = gpu_gp(sc, precision, gp_huber=0.0, cost_rel_tol=1e-16, grad_tol=1e-13,
                max_lm_iters=60, pcg_rel_tol=1e-12)
    srep = ba.gp_solve()
    c, X, s = _params(ba)
    err_truth = max(rel_err(X, sc.points_gt), rel_err(c, sc.cams_gt[:, 4:7]))
    print(f"GP recovery {precision}: vs oracle {rel_err(X, st.X):.2e}, vs truth {err_truth:.2e}, "
          f"rms {srep['final_rms_px']:.2e}, {srep['iterations']} iterations")
    assert rel_err(X, st.X) < (1e-9 if precision == "fp64" else 1e-6)
    assert err_truth < 1e-5


def _oracle_cost(prob, q, c, X, s, obs, delta):
    st = GpState(c=c, X=X, s=s)
    u, _ = gp_residuals(prob, q, st, obs)
    return 0.5 * float(np.sum(huber(np.sum(u * u, axis=1), delta)[0]))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gp_large_workload_costs(precision):
    """The 1000-camera workload: extraction bit-exact; the reported cost before a step and
    the candidate cost after it equal the oracle's cost at the same parameters."""
    sc = gp_scene("large")
    prob = Problem.from_scene(sc)
    q = sc.cams0[:, :4]
    ex = gp_extract(prob)
    ba = gpu_gp(sc, precision, pcg_rel_tol=1e-6, pcg_max_iters=100)
    c0, X0, s0 = _params(ba)
    F0 = _oracle_cost(prob, q, c0, X0, s0, ex.obs, 0.1)
    for k in range(6):   # the first steps may be rejected while the damping grows
        rep = ba.gp_step()
        assert abs(rep["cost_before"] - F0) <= 1e-10 * F0, k
        if rep["accepted"]:
            break
    assert rep["accepted"] == 1
    ac, ap, ao = ba.get_active()
    np.testing.assert_array_equal(ao, ex.obs_active)
    np.testing.assert_array_equal(ac, ex.cam_active)
    np.testing.assert_array_equal(ap, ex.pt_active)
    c1, X1, s1 = _params(ba)
    F1 = _oracle_cost(prob, q, c1, X1, s1, ex.obs, 0.1)
    print(f"large GP {precision}: F {F0:.6e} -> {F1:.6e} after {k + 1} steps, "
          f"PCG {rep['pcg_iters']}")
    assert abs(rep["cost_after"] - F1) <= 1e-10 * F0
    inactive = ~ex.pt_active
    np.testing.assert_array_equal(X1[inactive], X0[inactive])


def test_gp_and_ba_steps_interleave():
    """BA and GP steps on one context share the compaction buffers: a GP step after BA
    steps (which also move the rotations) evaluates its cost at the current estimate, a
    rejected GP step reuses its own linearisation, and a BA step after GP re-extracts."""
    sc = replace(gp_scene("medium"), fixed=np.array([0], np.int32))
    prob = Problem.from_scene(sc)
    ba = gpu_gp(sc, "fp64", huber_px=sc.huber_px)
    for _ in range(2):
        ba.lm_step()
    cams, pts = ba.get_params()
    s = ba.gp_scales()
    ex = gp_extract(prob)
    prev_accepted = True   # the first GP step after BA steps must linearise
    for k in range(4):
        rep = ba.gp_step()
        assert rep["relinearized"] == (1 if prev_accepted else 0), k
        cams2, pts2 = ba.get_params()
        F = _oracle_cost(prob, cams[:, :4], cams[:, 4:7], pts, s, ex.obs, 0.1)
        assert abs(rep["cost_before"] - F) <= 1e-12 * F, k
        if rep["accepted"]:
            cams, pts, s = cams2, pts2, ba.gp_scales()
        else:
            np.testing.assert_array_equal(pts2, pts)
        prev_accepted = bool(rep["accepted"])
    brep = ba.lm_step()
    assert brep["relinearized"] == 1
