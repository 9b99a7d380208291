"""GPU parity of the paths the oracle pins by construction, through the C ABI:

* the block-Jacobi preconditioner (the paper names PCG, Sec. IV-B, not its preconditioner):
  the M^-1 the PCG applies against the inverses of the diagonal 6x6 blocks of the oracle's
  dense damped camera Schur complement (Eq. (3)), compared as |S M S - S| / |S| so that the
  comparison does not grow with the blocks' condition number (up to 1e6 on the medium scene):
  1e-9 in float64, 1e-5 in mixed precision (the blocks are sums of float32 Jacobian products
  accumulated in float64: a relative error of about 6e-8 times the cancellation factor
  (|U| + |W V^-1 W^T|) / |S|, at most 6.3 here, so 4e-7; the bound leaves a factor 25);
* the true residual |b - S x| / |b| of the PCG solution against the oracle's dense S and b at
  the same damping (PCG stopped at 1e-3, so the residual is large against rounding);
* candidates that leave the domain of the cost: a point pushed to z <= 0.1 (Eq. (10)) and a
  global-positioning free scale pushed to <= 0 must be rejected with an infinite cost, with
  the oracle's damping sequence (Nielsen's rule, pinned by value on the CPU);
* the adjoint's status when its PCG stops at the iteration cap, and the size limits.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle.gp import GpOptions, GpState, gp_step
from oracle.lm import (Options, State, extract, linearize, normal_equations, damped,
                       reduced_camera_system, lm_step)
from oracle.model import Problem
from scenes import make_scene
from tests._common import oracle_setup, gpu_setup
from tests._constructed import near_depth_scene, embedded_near_depth_scene, gp_behind_scene

pytestmark = pytest.mark.gpu


def _oracle_reduced_system(sc, lam):
    prob, opts, st = oracle_setup(sc)
    ex = extract(prob, st, opts)
    lin = linearize(prob, st, ex, opts.huber_px)
    H, g = normal_equations(lin)
    S, b, _, _ = reduced_camera_system(damped(H, lam, opts), -g, lin.ncol_cam)
    return ex, S, b


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_preconditioner_inverts_schur_diagonal_blocks(name, precision, tol):
    sc = make_scene(name)
    ba = gpu_setup(sc, precision)
    rep = ba.lm_step()
    M = ba.get_preconditioner()
    ex, S, _ = _oracle_reduced_system(sc, rep["lambda"])
    worst = 0.0
    for s, c in enumerate(ex.cams):
        Sc = S[6 * s:6 * s + 6, 6 * s:6 * s + 6]
        worst = max(worst, np.abs(Sc @ M[c] @ Sc - Sc).max() / np.abs(Sc).max())
        if precision == "fp64" and name == "tiny":   # well conditioned: compare directly
            Mo = np.linalg.inv(Sc)
            assert np.abs(M[c] - Mo).max() <= 1e-9 * np.abs(Mo).max()
    inactive = np.setdiff1d(np.arange(sc.n_cams), ex.cams)
    assert np.all(M[inactive] == 0)
    print(f"{name} {precision}: max |S M S - S| / |S| = {worst:.3e}")
    assert worst <= tol, worst


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-2)])
def test_true_residual_against_oracle_schur(precision, tol):
    sc = make_scene("medium")
    ba = gpu_setup(sc, precision, timing=1, pcg_rel_tol=1e-3, pcg_max_iters=500)
    rep = ba.lm_step()
    ex, S, b = _oracle_reduced_system(sc, rep["lambda"])
    dc, _ = ba.get_last_step()
    x = dc[ex.cams].ravel()
    ref = np.linalg.norm(b - S @ x) / np.linalg.norm(b)
    got = rep["pcg_true_residual"]
    print(f"{precision}: true residual {got:.6e} (oracle S: {ref:.6e}), recursive "
          f"{rep['pcg_rel_residual']:.6e}, {rep['pcg_iters']} iterations")
    assert 1e-5 < ref < 2e-3
    assert abs(got - ref) <= tol * ref


def test_true_residual_only_when_timing():
    sc = make_scene("tiny")
    assert gpu_setup(sc, "fp64").lm_step()["pcg_true_residual"] == -1.0
    r = gpu_setup(sc, "fp64", timing=1, pcg_rel_tol=1e-12, pcg_max_iters=500).lm_step()
    assert 0.0 <= r["pcg_true_residual"] < 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_candidate_below_min_depth_rejected(precision):
    """One fixed camera and one point at 0.2 m pulled to a 0.05 m prior: the first five
    candidates cross z = 0.1 and are rejected with an infinite cost; the damping follows the
    oracle (1e-3, 2e-3, 8e-3, 6.4e-2, 1.024, 32.768) and the sixth step lands on its depth."""
    sc = near_depth_scene()
    prob = Problem.from_scene(sc)
    opts = Options()
    st = State.initial(sc.cams0, sc.points0, opts)
    ba = gpu_setup(sc, precision)
    for k in range(6):
        st, orep = lm_step(prob, st, opts)
        rep = ba.lm_step()
        assert rep["lambda"] == pytest.approx(orep.lam, rel=1e-12), k
        assert bool(rep["accepted"]) == orep.accepted, k
        assert rep["n_points_active"] == 1 and rep["n_cams_active"] == 0
        if not orep.accepted:
            assert rep["cost_after"] == np.inf, k
    assert orep.accepted
    _, pts = ba.get_params()
    assert pts[0, 2] == pytest.approx(st.X[0, 2], rel=1e-12 if precision == "fp64" else 1e-6)


def test_candidate_below_min_depth_inside_scene():
    sc = embedded_near_depth_scene()
    prob, opts, st = oracle_setup(sc)
    ba = gpu_setup(sc, "fp64", pcg_rel_tol=1e-13, pcg_max_iters=2000)
    seen = []
    for k in range(6):
        st, orep = lm_step(prob, st, opts)
        rep = ba.lm_step()
        assert bool(rep["accepted"]) == orep.accepted, k
        assert rep["lambda"] == pytest.approx(orep.lam, rel=1e-12), k
        if not orep.accepted:
            assert rep["cost_after"] == np.inf, k
        seen.append(orep.accepted)
    assert seen[0] is False and any(seen)
    cams, pts = ba.get_params()
    np.testing.assert_allclose(pts, st.X, rtol=0, atol=1e-9 * np.abs(st.X).max())


def test_gp_free_scale_below_zero_rejected():
    sc = gp_behind_scene()
    prob = Problem.from_scene(sc)
    q = sc.cams0[:, :4]
    opts = GpOptions(huber=0.0)
    st = GpState.initial(prob, q, sc.cams0, sc.points0, opts)
    ba = gpu_setup(sc, "fp64", gp_huber=0.0, pcg_rel_tol=1e-13, pcg_max_iters=2000)
    np.testing.assert_allclose(ba.gp_scales(), st.s, rtol=1e-12)
    seen = []
    for k in range(6):
        st, orep = gp_step(prob, q, st, opts)
        rep = ba.gp_step()
        assert bool(rep["accepted"]) == orep.accepted, k
        assert rep["lambda"] == pytest.approx(orep.lam, rel=1e-12), k
        if not orep.accepted:
            assert rep["cost_after"] == np.inf, k
        seen.append(orep.accepted)
    assert seen[0] is False and any(seen)
    np.testing.assert_allclose(ba.gp_scales(), st.s, rtol=1e-8)
    assert (ba.gp_scales() > 0).all()


def test_adjoint_status_at_iteration_cap():
    """An adjoint PCG stopped at its cap above the tolerance reports BA_NOT_CONVERGED (the
    gradients are still written); with enough iterations the same solve reports BA_OK."""
    from paper_2510_13310_amd import BA_NOT_CONVERGED, BA_OK
    sc = replace(make_scene("tiny", prior_frac=1.0, use_depth=True, lambda_d=50.0),
                 fixed=np.array([0], np.int32))
    ba = gpu_setup(sc, "fp64", pcg_rel_tol=1e-12, pcg_max_iters=500, max_lm_iters=30)
    ba.solve()
    gc = np.zeros((sc.n_cams, 7))
    gc[:, 4:7] = 1.0
    gpt = np.zeros((sc.n_points, 3))
    few = gpu_setup(sc, "fp64", pcg_rel_tol=1e-12, pcg_max_iters=500, max_lm_iters=30,
                    adjoint_max_iters=2)
    few.solve()
    with pytest.warns(RuntimeWarning, match="adjoint PCG stopped"):
        gxy_few, _ = few.adjoint(gc, gpt)
    assert few.last_adjoint_status == BA_NOT_CONVERGED
    assert np.isfinite(gxy_few).all()
    gxy, _ = ba.adjoint(gc, gpt)
    assert ba.last_adjoint_status == BA_OK
    assert np.abs(gxy).max() > 0


def test_size_limits_refused_with_real_arrays():
    """Sizes past the 32-bit index products of the kernels are refused before any array is
    read, also when the arrays are real (only the size check can refuse the call)."""
    import ctypes
    from paper_2510_13310_amd import _abi
    lib = _abi.load()
    sc = make_scene("tiny")
    ba = gpu_setup(sc, "fp64")
    ci = np.ascontiguousarray(sc.cam_idx)
    pi = np.ascontiguousarray(sc.pt_idx)
    xy = np.ascontiguousarray(sc.xy)
    n = ctypes.c_int64(2**29)
    assert lib.ba_set_observations(ba.ctx, n, ci.ctypes.data, pi.ctypes.data,
                                   xy.ctypes.data) == -1
    assert "2^29" in lib.ba_last_error(ba.ctx).decode()
    # the context is unchanged: a step still runs on the observations set before
    assert ba.lm_step()["n_obs_active"] > 0
    cams = np.ascontiguousarray(sc.cams0)
    intr = np.ascontiguousarray(sc.intr)
    pts = np.ascontiguousarray(sc.points0)
    out = ctypes.c_void_p()
    opts = ba.opts
    assert lib.ba_create(ctypes.byref(opts), 10, 2**27, cams.ctypes.data, intr.ctypes.data,
                         pts.ctypes.data, ctypes.byref(out)) == -1
    assert lib.ba_create(ctypes.byref(opts), 2**27, 10, cams.ctypes.data, intr.ctypes.data,
                         pts.ctypes.data, ctypes.byref(out)) == -1
    assert out.value is None
