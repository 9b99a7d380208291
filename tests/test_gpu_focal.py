"""GPU parity of focal-length refinement (each camera's focal length as a seventh camera
unknown, 7 x 7 camera blocks) against the FP64 oracle with ``refine_focal``.

Every scene starts from focal lengths scaled by a per-camera factor in [0.98, 1.02], the
intrinsics handed to both sides. Tolerances as for the pose-only path: active sets
bit-exact, normal-equation blocks 1e-9 (float64) / 2e-5 (mixed) relative, one LM step 1e-6
relative against the oracle's direct Cholesky solve, twelve fixed-gauge LM iterations with
identical decisions and parameters (focal lengths included) within 1e-6 relative.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle.lm import extract, linearize, lm_step, normal_equations, solve, Options, State
from oracle.model import Problem
from scenes import make_scene
from tests._common import gpu_setup, full_delta, rel_err

pytestmark = pytest.mark.gpu

SCENES = {}


def focal_scene(name, seed=3, **kw):
    """The named scene with every camera's focal length scaled by a seeded factor."""
    key = (name, seed, tuple(sorted(kw.items())))
    if key not in SCENES:
        sc = make_scene(name, **kw)
        rng = np.random.default_rng(seed)
        intr = sc.intr.copy()
        intr[:, 0] *= 1.0 + rng.uniform(-0.02, 0.02, size=sc.n_cams)
        SCENES[key] = replace(sc, intr=intr)
    return SCENES[key]


def oracle_focal(sc, **kw):
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px, refine_focal=True, **kw)
    prob = Problem.from_scene(sc)
    st = State.initial(sc.cams0, sc.points0, opts, focal=sc.intr[:, 0])
    return prob, opts, st


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 2e-5)])
def test_focal_extraction_and_normal_blocks(precision, tol):
    sc = focal_scene("medium")
    prob, opts, st = oracle_focal(sc)
    ex = extract(prob, st, opts)
    lin = linearize(prob, st, ex, opts.huber_px)
    H, g = normal_equations(lin)
    ba = gpu_setup(sc, precision, refine_focal=1)
    rep = ba.lm_step()
    ac, ap, ao = ba.get_active()
    np.testing.assert_array_equal(ac, ex.cam_active)
    np.testing.assert_array_equal(ap, ex.pt_active)
    np.testing.assert_array_equal(ao, ex.obs_active)
    assert rep["fixpoint_rounds"] == ex.rounds
    F = 0.5 * float(np.sum(lin.rho))
    assert abs(rep["cost_before"] - F) <= 1e-12 * F
    U, gc, V, gp = ba.get_normal_blocks()
    assert U.shape == (sc.n_cams, 7, 7) and gc.shape == (sc.n_cams, 7)
    Hd = H.tocsr()
    nc = 7 * ex.cams.size
    Uo, gco = np.zeros_like(U), np.zeros_like(gc)
    for s, c in enumerate(ex.cams):
        Uo[c] = Hd[7 * s:7 * s + 7, 7 * s:7 * s + 7].toarray()
        gco[c] = g[7 * s:7 * s + 7]
    Vo, gpo = np.zeros_like(V), np.zeros_like(gp)
    for r, p in enumerate(ex.pts):
        Vo[p] = Hd[nc + 3 * r:nc + 3 * r + 3, nc + 3 * r:nc + 3 * r + 3].toarray()
        gpo[p] = g[nc + 3 * r:nc + 3 * r + 3]
    assert rel_err(U, Uo) < tol
    assert rel_err(V, Vo) < tol
    # the focal row and column on their own (their scale differs from the pose entries)
    assert rel_err(U[:, 6, :], Uo[:, 6, :]) < tol
    assert rel_err(gc, gco) < (1e-9 if precision == "fp64" else 1e-5)
    assert rel_err(gp, gpo) < (1e-9 if precision == "fp64" else 1e-5)


def test_focal_single_step_split_items():
    """7 x 7 camera blocks summed over split items: 80,000 observations on the 10 tiny-scene
    cameras, every camera's piece of each of the 8 point ranges longer than the 512-position
    item bound; one float64 step against the oracle's Cholesky step (1e-6)."""
    sc = focal_scene("tiny", n_points=20_000)
    prob, opts, st = oracle_focal(sc, lambda_init=1.0)
    new, orep = lm_step(prob, st, opts)
    ba = gpu_setup(sc, "fp64", refine_focal=1, lambda_init=1.0, pcg_rel_tol=1e-13,
                   pcg_max_iters=3000)
    rep = ba.lm_step()
    assert rep["n_obs_active"] == orep.extraction.obs.size
    dc, dp = ba.get_last_step()
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points, d=7)
    print(f"focal split items: step error cameras {rel_err(dc, odc):.2e}, focal "
          f"{rel_err(dc[:, 6], odc[:, 6]):.2e}, points {rel_err(dp, odp):.2e}")
    assert rel_err(dc, odc) < 1e-6, rel_err(dc, odc)
    assert rel_err(dc[:, 6], odc[:, 6]) < 1e-6
    assert rel_err(dp, odp) < 1e-6, rel_err(dp, odp)
    assert bool(rep["accepted"]) == orep.accepted


@pytest.mark.parametrize("name,lam", [("tiny", 1e-3), ("medium", 1e-2), ("medium", 1.0)])
def test_focal_single_step_matches_cholesky(name, lam):
    sc = focal_scene(name)
    prob, opts, st = oracle_focal(sc, lambda_init=lam)
    new, orep = lm_step(prob, st, opts)
    ba = gpu_setup(sc, "fp64", refine_focal=1, lambda_init=lam, pcg_rel_tol=1e-13,
                   pcg_max_iters=3000)
    rep = ba.lm_step()
    dc, dp = ba.get_last_step()
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points, d=7)
    assert rel_err(dc, odc) < 1e-6, rel_err(dc, odc)
    assert rel_err(dc[:, 6], odc[:, 6]) < 1e-6
    assert rel_err(dp, odp) < 1e-6, rel_err(dp, odp)
    assert bool(rep["accepted"]) == orep.accepted
    if np.isfinite(orep.cost_after):
        assert abs(rep["cost_after"] - orep.cost_after) <= 1e-9 * orep.cost_after
    assert abs(rep["model_decrease"] - orep.model_decrease) <= 1e-7 * abs(orep.model_decrease)
    cams, pts = ba.get_params()
    intr = ba.get_intrinsics()
    np.testing.assert_allclose(cams, new.cams(), rtol=0, atol=1e-9 * max(1, np.abs(new.c).max()))
    np.testing.assert_allclose(pts, new.X, rtol=0, atol=1e-9 * np.abs(new.X).max())
    np.testing.assert_allclose(intr[:, 0], new.f, rtol=1e-12)
    np.testing.assert_array_equal(intr[:, 1:], sc.intr[:, 1:])     # cx, cy stay fixed


def test_focal_trajectory_fp64_medium_fixed_gauge():
    sc = replace(focal_scene("medium"), fixed=np.array([0], np.int32))
    prob, opts, st = oracle_focal(sc)
    ba = gpu_setup(sc, "fp64", refine_focal=1, pcg_rel_tol=1e-13, pcg_max_iters=3000)
    for k in range(12):
        st, orep = lm_step(prob, st, opts)
        rep = ba.lm_step()
        assert bool(rep["accepted"]) == orep.accepted, k
        assert rep["n_obs_active"] == orep.n_obs, k
        assert abs(rep["cost_before"] - orep.cost_before) <= 1e-9 * orep.cost_before, k
    cams, pts = ba.get_params()
    f = ba.get_intrinsics()[:, 0]
    d = max(rel_err(pts, st.X), rel_err(cams[:, 4:], st.c), rel_err(f, st.f))
    print(f"medium focal trajectory: max rel diff {d:.3e}")
    assert d < 1e-6, d
    assert f[0] == sc.intr[0, 0]                     # the fixed camera keeps its focal length


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_focal_recovery_noise_free(precision, tol):
    """Noise-free observations (rounded to float32 like a detector's), focal lengths off by
    up to 2 %: both the oracle and the GPU converge to the same focal lengths, and these are
    the true ones to the precision the float32 observations allow."""
    sc = focal_scene("tiny", noise_px=0.0)
    prob, opts, st = oracle_focal(sc, lambda_init=1e-4, cost_rel_tol=0.0, grad_tol=1e-14,
                                  max_iters=60)
    st, _ = solve(prob, st, opts)
    ba = gpu_setup(sc, precision, refine_focal=1, lambda_init=1e-4, pcg_rel_tol=1e-12,
                   pcg_max_iters=3000, cost_rel_tol=0.0, grad_tol=1e-14, max_lm_iters=60)
    srep = ba.solve()
    f = ba.get_intrinsics()[:, 0]
    truth = make_scene("tiny").intr[:, 0]
    print(f"focal recovery {precision}: max rel error vs oracle {rel_err(f, st.f):.3e}, "
          f"vs truth {rel_err(f, truth):.3e}, rms {srep['final_rms_px']:.3e} px")
    assert rel_err(f, st.f) < tol
    assert rel_err(f, truth) < 1e-5
    assert srep["final_rms_px"] < 1e-3


def test_focal_adjoint_is_rejected():
    from paper_2510_13310_amd import BAError, BA_ERR_STATE
    sc = replace(focal_scene("tiny"), fixed=np.array([0, 1], np.int32))
    ba = gpu_setup(sc, "fp64", refine_focal=1)
    ba.lm_step()
    with pytest.raises(BAError) as e:
        ba.adjoint(np.zeros((sc.n_cams, 7)), np.zeros((sc.n_points, 3)))
    assert e.value.status == BA_ERR_STATE
