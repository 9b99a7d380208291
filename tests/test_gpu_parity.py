"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
scenes. Sizes span many 256-thread blocks and scan tiles and end on ragged tails.

Tolerances (float64 path): active sets and ranks bit-exact; normal-equation blocks and
gradients 1e-9 relative to the largest entry; one LM step 1e-6 relative (PCG to 1e-12 vs a
direct Cholesky); the tiny scene solved to convergence within 1e-6 relative gauge-aligned
parameters; the adjoint workload (the medium scene with camera 0 fixed and metric depth rows,
so no gauge freedom is left) solved by both to max |g| <= 1e-3 within 1e-6 relative
parameters and 1e-6 rad rotations. Mixed precision (float32 Jacobians and matvecs): blocks
2e-5; on the same solve final RMS within 1e-3 px of the oracle's and parameters within 1e-6
relative (the float32 Jacobian perturbs the stationary point itself, see the test).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle.lm import extract, linearize, normal_equations, lm_step, solve, Options, State
from scenes import make_scene
from tests._align import aligned_error, rotation_error
from tests._common import oracle_setup, gpu_setup, full_delta, rel_err

pytestmark = pytest.mark.gpu

SCENES = {}


def scene(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in SCENES:
        SCENES[key] = make_scene(name, **kw)
    return SCENES[key]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_extraction_bit_exact(name, precision):
    sc = scene(name)
    prob, opts, st = oracle_setup(sc)
    ex = extract(prob, st, opts)
    ba = gpu_setup(sc, precision)
    rep = ba.lm_step()
    ac, ap, ao = ba.get_active()
    np.testing.assert_array_equal(ac, ex.cam_active)
    np.testing.assert_array_equal(ap, ex.pt_active)
    np.testing.assert_array_equal(ao, ex.obs_active)
    assert rep["n_obs_active"] == ex.obs.size
    assert rep["n_cams_active"] == ex.cams.size
    assert rep["n_points_active"] == ex.pts.size
    assert rep["fixpoint_rounds"] == ex.rounds


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 2e-5)])
def test_normal_blocks_and_cost(precision, tol):
    sc = scene("medium")
    prob, opts, st = oracle_setup(sc)
    ex = extract(prob, st, opts)
    lin = linearize(prob, st, ex, opts.huber_px)
    H, g = normal_equations(lin)
    nc = 6 * ex.cams.size
    ba = gpu_setup(sc, precision)
    rep = ba.lm_step()
    U, gc, V, gp = ba.get_normal_blocks()
    F = 0.5 * float(np.sum(lin.rho))
    assert abs(rep["cost_before"] - F) <= 1e-12 * F
    rms = float(np.sqrt(np.mean(np.sum(lin.e[:, :2] ** 2, axis=1))))
    assert abs(rep["rms_px"] - rms) <= 1e-12 * rms
    Hd = H.tocsr()
    # camera blocks
    Uo = np.zeros_like(U)
    gco = np.zeros_like(gc)
    for s, c in enumerate(ex.cams):
        Uo[c] = Hd[6 * s:6 * s + 6, 6 * s:6 * s + 6].toarray()
        gco[c] = g[6 * s:6 * s + 6]
    Vo = np.zeros_like(V)
    gpo = np.zeros_like(gp)
    for r, p in enumerate(ex.pts):
        Vo[p] = Hd[nc + 3 * r:nc + 3 * r + 3, nc + 3 * r:nc + 3 * r + 3].toarray()
        gpo[p] = g[nc + 3 * r:nc + 3 * r + 3]
    assert rel_err(U, Uo) < tol
    assert rel_err(V, Vo) < tol
    # gradients are accumulated in float64 in both precisions
    assert rel_err(gc, gco) < (1e-9 if precision == "fp64" else 1e-5)
    assert rel_err(gp, gpo) < (1e-9 if precision == "fp64" else 1e-5)
    assert abs(rep["grad_inf"] - np.max(np.abs(g))) <= 1e-6 * np.max(np.abs(g))


@pytest.mark.parametrize("name,lam", [("tiny", 1e-3), ("medium", 1e-2), ("medium", 1.0)])
def test_single_step_matches_cholesky(name, lam):
    sc = scene(name)
    prob, opts, st = oracle_setup(sc, lambda_init=lam)
    new, orep = lm_step(prob, st, opts)
    ba = gpu_setup(sc, "fp64", lambda_init=lam, pcg_rel_tol=1e-13, pcg_max_iters=2000)
    rep = ba.lm_step()
    dc, dp = ba.get_last_step()
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points)
    assert rel_err(dc, odc) < 1e-6, rel_err(dc, odc)
    assert rel_err(dp, odp) < 1e-6, rel_err(dp, odp)
    assert bool(rep["accepted"]) == orep.accepted
    if np.isfinite(orep.cost_after):
        assert abs(rep["cost_after"] - orep.cost_after) <= 1e-9 * orep.cost_after
    else:
        assert not np.isfinite(rep["cost_after"])
    assert abs(rep["model_decrease"] - orep.model_decrease) <= 1e-7 * abs(orep.model_decrease)
    cams, pts = ba.get_params()
    np.testing.assert_allclose(cams, new.cams(), rtol=0, atol=1e-9 * max(1, np.abs(new.c).max()))
    np.testing.assert_allclose(pts, new.X, rtol=0, atol=1e-9 * np.abs(new.X).max())


@pytest.mark.parametrize("n_points", [5, 13])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-5)])
def test_single_step_few_points(n_points, precision, tol):
    """Fewer active points than the 8 point ranges of the matrix-free passes (4 and 13 here):
    some XCD ranges are empty and every camera's segment splits into one-point items; the
    step still equals the oracle's dense Schur + Cholesky step."""
    sc = make_scene("tiny", n_points=n_points)
    prob, opts, st = oracle_setup(sc, lambda_init=1.0)
    new, orep = lm_step(prob, st, opts)
    ba = gpu_setup(sc, precision, lambda_init=1.0, pcg_rel_tol=1e-13, pcg_max_iters=2000)
    rep = ba.lm_step()
    assert rep["n_obs_active"] == orep.extraction.obs.size
    dc, dp = ba.get_last_step()
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points)
    print(f"{n_points} points {precision}: step error cameras {rel_err(dc, odc):.2e}, "
          f"points {rel_err(dp, odp):.2e}")
    assert rel_err(dc, odc) < tol, rel_err(dc, odc)
    assert rel_err(dp, odp) < tol, rel_err(dp, odp)
    assert bool(rep["accepted"]) == orep.accepted


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-5)])
def test_single_step_split_items(precision, tol):
    """80,000 observations of 20,000 points on the 10 tiny-scene cameras: every camera's piece
    of each of the 8 point ranges (920 to 1053 positions) exceeds the 512-position item bound,
    so the camera assembly and the PCG camera pass both sum cameras over several items per
    range; the step still equals the oracle's dense Schur + Cholesky step."""
    sc = make_scene("tiny", n_points=20_000)
    prob, opts, st = oracle_setup(sc, lambda_init=1.0)
    new, orep = lm_step(prob, st, opts)
    ba = gpu_setup(sc, precision, lambda_init=1.0, pcg_rel_tol=1e-13, pcg_max_iters=2000)
    rep = ba.lm_step()
    assert rep["n_obs_active"] == orep.extraction.obs.size
    dc, dp = ba.get_last_step()
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points)
    print(f"split items {precision}: step error cameras {rel_err(dc, odc):.2e}, "
          f"points {rel_err(dp, odp):.2e}")
    assert rel_err(dc, odc) < tol, rel_err(dc, odc)
    assert rel_err(dp, odp) < tol, rel_err(dp, odp)
    assert bool(rep["accepted"]) == orep.accepted
    # the camera blocks and gradients, summed over several items per camera and range, against
    # the oracle's (float64 1e-9; mixed 2e-5 for the float32 blocks, 1e-5 for the gradient)
    U, gc, _, _ = ba.get_normal_blocks()
    ex = orep.extraction
    H, g = normal_equations(linearize(prob, st, ex, opts.huber_px))
    Hd = H.tocsr()
    Uo = np.zeros_like(U)
    gco = np.zeros_like(gc)
    for k, c in enumerate(ex.cams):
        Uo[c] = Hd[6 * k:6 * k + 6, 6 * k:6 * k + 6].toarray()
        gco[c] = g[6 * k:6 * k + 6]
    assert rel_err(U, Uo) < (1e-9 if precision == "fp64" else 2e-5), rel_err(U, Uo)
    assert rel_err(gc, gco) < (1e-9 if precision == "fp64" else 1e-5), rel_err(gc, gco)


_CONVERGED = {}


def _converge_oracle(sc):
    if sc.name not in _CONVERGED:
        prob, opts, st = oracle_setup(sc, cost_rel_tol=0.0, grad_tol=0.0, max_iters=60)
        _CONVERGED[sc.name] = solve(prob, st, opts)
    return _CONVERGED[sc.name]


def test_converged_solution_fp64_tiny():
    """No outliers, no robust loss: LM converges quadratically, so the converged solutions
    of both implementations coincide up to the free similarity gauge."""
    sc = scene("tiny")
    st, reps = _converge_oracle(sc)
    ba = gpu_setup(sc, "fp64", pcg_rel_tol=1e-12, pcg_max_iters=2000, cost_rel_tol=0.0,
                   grad_tol=0.0, max_lm_iters=60)
    srep = ba.solve()
    cams, pts = ba.get_params()
    assert abs(srep["final_rms_px"] - reps[-1].rms_px) < 1e-3
    err, (s, R, t) = aligned_error(cams, pts, st.cams(), st.X)
    print(f"tiny converged: aligned parameter error {err:.3e}")
    assert err < 1e-6, err
    assert rotation_error(cams, st.cams(), R) < 1e-6


def test_lm_trajectory_fp64_medium_fixed_gauge():
    """Twelve LM iterations on the medium scene (outliers, Huber, filter, depth priors,
    dynamic extraction every iteration) with camera 0 fixed: identical accept/reject
    decisions and costs each iteration, parameters within 1e-6 relative."""
    sc = replace(scene("medium"), fixed=np.array([0], np.int32))
    prob, opts, st = oracle_setup(sc)
    ba = gpu_setup(sc, "fp64", pcg_rel_tol=1e-13, pcg_max_iters=3000)
    for k in range(12):
        st, orep = lm_step(prob, st, opts)
        rep = ba.lm_step()
        assert bool(rep["accepted"]) == orep.accepted, k
        assert rep["n_obs_active"] == orep.n_obs, k
        assert abs(rep["cost_before"] - orep.cost_before) <= 1e-9 * orep.cost_before, k
    cams, pts = ba.get_params()
    err, _ = aligned_error(cams, pts, st.cams(), st.X, with_scale=False)
    d = max(rel_err(pts, st.X), rel_err(cams[:, 4:], st.c))
    print(f"medium trajectory: max rel diff {d:.3e}, rigid-aligned error {err:.3e}")
    assert err < 1e-6 and d < 1e-6, (err, d)


def _rel(a, b):
    """|a - b|_F / |b - mean(b)|_F over stacked centres and points."""
    return float(np.linalg.norm(a - b) / np.linalg.norm(b - b.mean(axis=0)))


_FIXED_GAUGE = {}


def _converge_oracle_fixed_gauge():
    if "adjoint" not in _FIXED_GAUGE:
        sc = scene("adjoint")
        prob, opts, st = oracle_setup(sc, cost_rel_tol=0.0, grad_tol=1e-3, max_iters=150)
        _FIXED_GAUGE["adjoint"] = solve(prob, st, opts)
    return _FIXED_GAUGE["adjoint"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_converged_parameters_fixed_gauge(precision):
    """The adjoint workload (medium scene: outliers, Huber 2 px, 4 px filter, dynamic
    extraction, camera 0 fixed, depth rows with lambda_d = 300 fixing the metric scale) solved
    by both implementations with the same stopping rule, max |g| <= 1e-3 at the start of a
    step (cost about 6e4). The robust problem converges linearly under IRLS (about 0.84 per
    iteration once the damping bottoms out), so the rule stops both after the same iteration.

    The stopping point is converged to far below the tolerances: continuing the oracle from
    it to the float64 floor (steps rejected until the damping reaches its maximum) moves the
    points by 5.4e-9 and the centres by 2.8e-11 relative.

    float64: same iteration count, parameters within 1e-6 relative (|d|_F over stacked
    centres and points against their spread) and rotations within 1e-6 rad, RMS within
    1e-3 px. Mixed: the float32 Jacobian moves the point where the float64-accumulated
    gradient vanishes by a few float32 roundings (6e-8) amplified by the weak directions of
    the reduced system; mixed is held to RMS within 1e-3 px and parameters and rotations
    within 1e-6 (17 float32 roundings)."""
    sc = scene("adjoint")
    st, reps = _converge_oracle_fixed_gauge()
    o_rms = reps[-1].rms_px
    kw = dict(cost_rel_tol=0.0, grad_tol=1e-3, max_lm_iters=150)
    if precision == "fp64":
        ba = gpu_setup(sc, "fp64", pcg_rel_tol=1e-12, pcg_max_iters=3000, **kw)
    else:
        ba = gpu_setup(sc, "mixed", pcg_rel_tol=1e-8, pcg_max_iters=1000, **kw)
    srep = ba.solve()
    cams, pts = ba.get_params()
    np.testing.assert_array_equal(cams[0], sc.cams0[0])
    err = _rel(np.vstack([cams[:, 4:7], pts]), np.vstack([st.c, st.X]))
    rot = rotation_error(cams, st.cams(), np.eye(3))
    print(f"adjoint workload {precision}: {srep['iterations']} iterations (oracle {len(reps)}), "
          f"stop {srep['stop_reason']}, rms {srep['final_rms_px']:.9f} (oracle {o_rms:.9f}), "
          f"parameter error {err:.3e}, rotation error {rot:.3e} rad")
    assert abs(srep["final_rms_px"] - o_rms) < 1e-3
    if precision == "fp64":
        assert srep["iterations"] == len(reps) and srep["stop_reason"] == 2
        assert err < 1e-6, err
        assert rot < 1e-6, rot
    else:
        assert err < 1e-6, err
        assert rot < 1e-6, rot


def test_converged_medium_rms_both_precisions():
    """Free gauge (the medium scene as generated), run to the stopping rule: final RMS of the
    float64 and mixed GPU paths within 1e-3 px of the oracle's and final costs within 1e-6
    relative. Parameters are compared with the gauge fixed in the test above."""
    sc = scene("medium")
    st, reps = _converge_oracle(sc)
    o_rms = reps[-1].rms_px
    out = {}
    for prec in ("fp64", "mixed"):
        ba = gpu_setup(sc, prec, pcg_rel_tol=1e-8, pcg_max_iters=500, cost_rel_tol=1e-12,
                       max_lm_iters=60)
        srep = ba.solve()
        out[prec] = srep["final_rms_px"]
        o_cost = min(r.cost_after if r.accepted else r.cost_before for r in reps)
        print(f"medium {prec}: rms {srep['final_rms_px']:.6f} (oracle {o_rms:.6f}), "
              f"cost {srep['final_cost']:.6f} (oracle {o_cost:.6f}), "
              f"{srep['iterations']} iterations")
        assert abs(srep["final_rms_px"] - o_rms) < 1e-3
        assert abs(srep["final_cost"] - o_cost) <= 1e-6 * o_cost
    assert abs(out["mixed"] - out["fp64"]) < 1e-3


def test_inactive_parameters_bit_identical_and_deterministic():
    """Two runs, the second with per-launch timing events: bitwise identical results, and
    the timing statistics cover every kernel of the step."""
    sc = scene("medium")
    runs = []
    for timing in (0, 1):
        ba = gpu_setup(sc, "mixed", timing=timing)
        for _ in range(4):
            ba.lm_step()
        ac, ap, _ = ba.get_active()
        runs.append(ba.get_params() + (ac, ap))
        stats = {k["name"]: k for k in ba.kernel_stats()}
    (c1, p1, ac, ap), (c2, p2, _, _) = runs
    np.testing.assert_array_equal(c1, c2)          # bitwise reproducible
    np.testing.assert_array_equal(p1, p2)
    for name in ("validate", "scan", "compact", "lin_point", "cam_assemble", "schur_point",
                 "schur_cam", "pcg_update", "backsub", "point_candidate"):
        assert stats[name]["launches"] > 0 and stats[name]["total_ms"] > 0, (name, stats)
    assert stats["schur_point"]["launches"] == stats["pcg_update"]["launches"]
    bad = sc.notes["perturbed_cameras"]
    np.testing.assert_array_equal(c1[bad], sc.cams0[bad])
    outl = sc.notes["all_outlier_points"]
    np.testing.assert_array_equal(p1[outl], sc.points0[outl])


def test_empty_active_set_is_a_no_op():
    sc = scene("tiny")
    ba = gpu_setup(sc, "fp64")
    far = np.tile(np.array([0.0, 100.0, 0.0]), (sc.n_points, 1))
    ba.set_params(points=far)
    rep = ba.lm_step()
    assert rep["status"] == 1 and rep["n_obs_active"] == 0
    cams, pts = ba.get_params()
    np.testing.assert_array_equal(pts, far)
    np.testing.assert_array_equal(cams, sc.cams0)


def test_ragged_degrees_and_literal_rule():
    """Points with 1..9 views (ragged segments), the paper-literal activity rule."""
    sc = scene("medium", n_cams=40, n_points=3001, views=9)
    rng = np.random.default_rng(5)
    keep = rng.random(sc.n_obs) < 0.55
    sc2 = replace(sc, **{f: getattr(sc, f)[keep] for f in
                         ("cam_idx", "pt_idx", "xy", "depth", "depth_valid", "is_outlier")})
    for rule in ("rows", "literal"):
        prob, opts, st = oracle_setup(sc2, rule=rule)
        ex = extract(prob, st, opts)
        ba = gpu_setup(sc2, "fp64", activity_rule=rule)
        ba.lm_step()
        ac, ap, ao = ba.get_active()
        np.testing.assert_array_equal(ao, ex.obs_active)
        np.testing.assert_array_equal(ap, ex.pt_active)
        np.testing.assert_array_equal(ac, ex.cam_active)


def test_fixed_cameras_never_move():
    sc = scene("medium", n_cams=30, n_points=2000)
    sc.fixed = np.array([0, 7, 29], np.int32)
    prob, opts, st = oracle_setup(sc, lambda_init=0.1)
    new, orep = lm_step(prob, st, opts)
    ba = gpu_setup(sc, "fp64", lambda_init=0.1, pcg_rel_tol=1e-13, pcg_max_iters=2000)
    rep = ba.lm_step()
    cams, _ = ba.get_params()
    np.testing.assert_array_equal(cams[sc.fixed], sc.cams0[sc.fixed])
    dc, dp = ba.get_last_step()
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points)
    assert rel_err(dc, odc) < 1e-6 and rel_err(dp, odp) < 1e-6


def test_abi_errors_on_device():
    from paper_2510_13310_amd import BundleAdjuster, BAError
    sc = scene("tiny")
    ba = BundleAdjuster(sc.cams0, sc.intr, sc.points0, precision="fp64")
    with pytest.raises(BAError) as e:
        ba.lm_step()
    assert e.value.status == -2
    bad = sc.cam_idx.copy()
    bad[3] = sc.n_cams
    with pytest.raises(BAError) as e:
        ba.set_observations(bad, sc.pt_idx, sc.xy)
    assert e.value.status == -1
    with pytest.raises(BAError) as e:
        ba.set_fixed_cameras(np.array([-1], np.int32))
    assert e.value.status == -1
    # sizes beyond what the scans index are refused before any array is read
    import ctypes
    from paper_2510_13310_amd import _abi
    lib = _abi.load()
    assert lib.ba_set_observations(ba.ctx, ctypes.c_int64(2**31 - 1), None, None, None) == -1
    assert lib.ba_set_observations(ba.ctx, ctypes.c_int64(-1), None, None, None) == -1
    out = ctypes.c_void_p()
    assert lib.ba_create(None, 2**31 - 1, 10, None, None, None, ctypes.byref(out)) == -1
    ba.set_observations(sc.cam_idx, sc.pt_idx, sc.xy)
    with pytest.raises(BAError) as e:
        ba.adjoint(np.zeros((sc.n_cams, 7)), np.zeros((sc.n_points, 3)))
    assert e.value.status == -2
    xy = sc.xy.copy()
    xy[0, 0] = np.nan
    ba.set_observations(sc.cam_idx, sc.pt_idx, xy)
    with pytest.raises(BAError) as e:
        ba.lm_step()
    assert e.value.status == -5
    cams, pts = ba.get_params()
    np.testing.assert_array_equal(pts, sc.points0)
