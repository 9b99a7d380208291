"""GPU parity of the implicit adjoint (ba_adjoint / BASolve.backward).

* Against the oracle's direct adjoint (full robust-corrected Gauss-Newton system solved
  without a Schur reduction), evaluated at the GPU's converged parameters: relative error
  1e-5 of the largest gradient (the ABI returns float32 gradients), float64 path.
* Against central differences of converged GPU re-solves on the medium scene (camera 0
  fixed, loss = sum of squared camera-centre errors): 50 coordinates (40 pixel, 10 depth),
  steps 1e-3 px and 1e-4 d_hat, coordinates away from the Huber and filter thresholds.
  Without noise the Gauss-Newton Hessian is exact at the optimum (bound 1e-3); with the
  workload's noise it drops the second-derivative residual term, whose gap is measured and
  printed (median bound 3e-2, max 0.25, relative to the largest gradient).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle.adjoint import adjoint as oracle_adjoint
from oracle.lm import Options, State, extract
from oracle.model import Problem
from scenes import make_scene, subscene
from tests._common import gpu_setup

pytestmark = pytest.mark.gpu

SOLVE = dict(pcg_rel_tol=1e-12, pcg_max_iters=3000, cost_rel_tol=0.0, grad_tol=0.0,
             max_lm_iters=150, lambda_init=1e-4)
# warm-started re-solves of the 100k-observation scene (100 of them). IRLS converges
# linearly (about 0.84 per iteration on this scene), so 200 iterations bring the gradient
# ~15 orders of magnitude below a 1e-3 px perturbation's.
FD_SOLVE = dict(pcg_rel_tol=1e-10, pcg_max_iters=400, cost_rel_tol=0.0, grad_tol=0.0,
                max_lm_iters=200, lambda_init=1e-4)


def _loss_grads(sc, cams, pts, rng):
    """L = sum |c_i - c_i^gt|^2 + sum W . X: gradients with respect to cams and points."""
    W = rng.normal(size=pts.shape) * 1e-2
    g_c = np.zeros_like(cams)
    g_c[:, 4:7] = 2.0 * (cams[:, 4:7] - sc.cams_gt[:, 4:7])
    return g_c, W


def _loss(sc, cams, pts, W):
    return float(np.sum((cams[:, 4:7] - sc.cams_gt[:, 4:7]) ** 2) + np.sum(W * pts))


def _oracle_at(sc, cams, pts, g_c, g_p):
    prob = Problem.from_scene(sc)
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px)
    st = State(q=cams[:, :4].copy(), c=cams[:, 4:7].copy(), X=pts.copy(), lam=0.0)
    gxy, gd, _ = oracle_adjoint(prob, st, opts, g_c, g_p)
    return gxy, gd, extract(prob, st, opts)


@pytest.mark.parametrize("which", ["tiny-exact-priors", "adjoint-sub-cams0-9"])
def test_adjoint_matches_oracle_direct_solve(which):
    rng = np.random.default_rng(3)
    if which == "tiny-exact-priors":
        sc = make_scene("tiny", n_points=150, noise_px=0.5, prior_frac=0.7, use_depth=True,
                        lambda_d=30.0)
        sc = replace(sc, fixed=np.array([0], np.int32))
    else:
        sc = subscene(make_scene("adjoint"), np.arange(10), max_points=1500, seed=1)
    ba = gpu_setup(sc, "fp64", **SOLVE)
    ba.solve()
    cams, pts = ba.get_params()
    g_c, g_p = _loss_grads(sc, cams, pts, rng)
    gxy, gd = ba.adjoint(g_c, g_p)
    ogxy, ogd, ex = _oracle_at(sc, cams, pts, g_c, g_p)
    _, _, act = ba.get_active()
    np.testing.assert_array_equal(act, ex.obs_active)
    scale = max(np.abs(ogxy).max(), np.abs(ogd).max())
    err = max(np.abs(gxy - ogxy).max(), np.abs(gd - ogd).max()) / scale
    huber_obs = 0
    if sc.huber_px > 0:
        prob = Problem.from_scene(sc)
        from oracle.model import residuals
        e, _, _ = residuals(prob, cams[:, :4], cams[:, 4:], pts, ex.obs)
        huber_obs = int(np.sum(np.sum(e * e, axis=1) > sc.huber_px ** 2))
    print(f"{which}: adjoint vs oracle direct solve, max rel error {err:.3e} "
          f"({ex.obs.size} active observations, {huber_obs} in the Huber regime)")
    assert err < 1e-5, err
    assert np.all(gxy[~act] == 0) and np.all(gd[~act] == 0)


def test_damped_adjoint_matches_oracle():
    """adjoint_damping > 0: the GPU's damped Schur/PCG solve against the oracle's damped
    direct solve (same Marquardt diagonal), float64, 1e-5 of the largest gradient."""
    rng = np.random.default_rng(9)
    sc = subscene(make_scene("adjoint"), np.arange(10), max_points=1500, seed=1)
    ba = gpu_setup(sc, "fp64", adjoint_damping=1e-2, **SOLVE)
    ba.solve()
    cams, pts = ba.get_params()
    g_c, g_p = _loss_grads(sc, cams, pts, rng)
    gxy, gd = ba.adjoint(g_c, g_p)
    prob = Problem.from_scene(sc)
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px)
    st = State(q=cams[:, :4].copy(), c=cams[:, 4:7].copy(), X=pts.copy(), lam=0.0)
    ogxy, ogd, _ = oracle_adjoint(prob, st, opts, g_c, g_p, damping=1e-2)
    ugxy, _, _ = oracle_adjoint(prob, st, opts, g_c, g_p)
    scale = max(np.abs(ogxy).max(), np.abs(ogd).max())
    err = max(np.abs(gxy - ogxy).max(), np.abs(gd - ogd).max()) / scale
    print(f"damped adjoint vs oracle: max rel error {err:.3e} (damping moves the gradient by "
          f"{np.abs(ogxy - ugxy).max() / scale:.2e})")
    assert err < 1e-5, err


def test_adjoint_mixed_precision_close_to_fp64():
    rng = np.random.default_rng(4)
    sc = subscene(make_scene("adjoint"), np.arange(10), max_points=1500, seed=1)
    ba = gpu_setup(sc, "fp64", **SOLVE)
    ba.solve()
    cams, pts = ba.get_params()
    g_c, g_p = _loss_grads(sc, cams, pts, rng)
    ref = ba.adjoint(g_c, g_p)
    bm = gpu_setup(sc, "mixed", **SOLVE)
    bm.set_params(cams, pts)
    out = bm.adjoint(g_c, g_p)
    scale = max(np.abs(ref[0]).max(), np.abs(ref[1]).max())
    err = max(np.abs(out[0] - ref[0]).max(), np.abs(out[1] - ref[1]).max()) / scale
    print(f"mixed vs fp64 adjoint: max rel error {err:.3e}")
    assert err < 1e-2, err


def _pick_coords(sc, cams, pts, act, rng, n_xy=40, n_d=10, margin=0.05):
    prob = Problem.from_scene(sc)
    from oracle.model import residuals
    obs = np.nonzero(act)[0]
    e, Xc, _ = residuals(prob, cams[:, :4], cams[:, 4:], pts, obs)
    r2 = np.sqrt(e[:, 0] ** 2 + e[:, 1] ** 2)
    n3 = np.sqrt(np.sum(e * e, axis=1))
    ok = (np.abs(n3 - sc.huber_px) > margin) & (r2 < sc.filter_px - margin)
    ok &= ~sc.is_outlier[obs]
    f = sc.intr[0, 0]
    u = f * Xc[:, 0] / Xc[:, 2] + sc.intr[0, 1]
    v = f * Xc[:, 1] / Xc[:, 2] + sc.intr[0, 2]
    ok &= (u > 2) & (u < sc.img_w - 2) & (v > 2) & (v < sc.img_h - 2)
    cand = obs[ok]
    xy_k = rng.choice(cand, size=n_xy, replace=False)
    dcand = cand[prob.prior_mask[cand]]
    d_k = rng.choice(dcand, size=n_d, replace=False)
    return [(int(k), int(rng.integers(2))) for k in xy_k] + [(int(k), 2) for k in d_k]


def _fd_check(sc, rng, tag):
    ba = gpu_setup(sc, "fp64", **FD_SOLVE)
    srep = ba.solve()
    cams0, pts0 = ba.get_params()
    _, _, act = ba.get_active()
    g_c = np.zeros_like(cams0)
    g_c[:, 4:7] = 2.0 * (cams0[:, 4:7] - sc.cams_gt[:, 4:7])
    gxy, gd = ba.adjoint(g_c, np.zeros_like(pts0))
    coords = _pick_coords(sc, cams0, pts0, act, rng)
    fds, refs = [], []
    for k, j in coords:
        h = 1e-3 if j < 2 else 1e-4 * float(sc.depth[k])
        vals = []
        for sgn in (1.0, -1.0):
            xy = sc.xy.copy()
            depth = sc.depth.copy()
            if j < 2:
                xy[k, j] = np.float32(xy[k, j] + sgn * h)
                step = float(xy[k, j]) - float(sc.xy[k, j])
            else:
                depth[k] = np.float32(depth[k] + sgn * h)
                step = float(depth[k]) - float(sc.depth[k])
            ba.set_observations(sc.cam_idx, sc.pt_idx, xy)
            ba.set_depth_priors(depth, sc.depth_valid, sc.lambda_d)
            ba.set_params(cams0, pts0)
            ba.solve()
            c1, p1 = ba.get_params()
            vals.append((float(np.sum((c1[:, 4:7] - sc.cams_gt[:, 4:7]) ** 2)), step))
        fds.append((vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1]))
        refs.append(gxy[k, j] if j < 2 else gd[k])
    fds, refs = np.array(fds), np.array(refs)
    scale = np.max(np.abs(refs))
    err = np.max(np.abs(fds - refs)) / scale
    med = np.median(np.abs(fds - refs)) / scale
    print(f"{tag}: adjoint vs central differences ({len(coords)} coordinates, "
          f"{srep['iterations']} LM iterations in the base solve, stop {srep['stop_reason']}): "
          f"max rel error {err:.3e}, median {med:.3e}")
    return err, fds, refs


def test_adjoint_finite_differences_noise_free_scene():
    """The adjoint workload without pixel noise, outliers or depth-prior noise: residuals
    vanish at the optimum, the Gauss-Newton Hessian is exact there, and the implicit
    gradient must match central differences of converged re-solves closely."""
    sc = make_scene("adjoint", noise_px=0.0, outlier_frac=0.0, all_outlier_points=0,
                    depth_sigma=0.0)
    err, fds, refs = _fd_check(sc, np.random.default_rng(7), "noise-free adjoint scene")
    assert err < 1e-3, np.c_[fds, refs]


def test_adjoint_medium_finite_differences():
    """The adjoint workload (medium scene, camera 0 fixed) with its noise and outliers. The
    Gauss-Newton Hessian drops the second-order residual term; on this workload the gap is
    about 1 % at the median and up to ~15 % on weakly determined coordinates (the oracle's
    robust-metric pin shows the same few-percent gap on a small noisy scene). The bounds
    below are that measured gap with margin."""
    sc = make_scene("adjoint")
    err, fds, refs = _fd_check(sc, np.random.default_rng(2510), "adjoint scene")
    med = np.median(np.abs(fds - refs)) / np.max(np.abs(refs))
    assert med < 0.03 and err < 0.25, np.c_[fds, refs]


def test_autograd_function_backward_matches_adjoint():
    import torch
    from paper_2510_13310_amd.autograd import BASolve
    sc = replace(make_scene("tiny", n_points=120, noise_px=0.5, prior_frac=0.8, use_depth=True,
                            lambda_d=20.0), fixed=np.array([0], np.int32))
    dev = torch.device("cuda:0")
    xy = torch.tensor(sc.xy, device=dev, requires_grad=True)
    depth = torch.tensor(sc.depth, device=dev, requires_grad=True)
    problem = dict(cam_idx=sc.cam_idx, pt_idx=sc.pt_idx, intr=sc.intr,
                   depth_valid=sc.depth_valid, lambda_d=sc.lambda_d, fixed=sc.fixed,
                   options=dict(precision="fp64", **SOLVE))
    cams, pts = BASolve.apply(xy, depth, torch.tensor(sc.cams0, device=dev),
                              torch.tensor(sc.points0, device=dev), problem)
    gt = torch.tensor(sc.cams_gt[:, 4:7], device=dev)
    loss = ((cams[:, 4:7] - gt) ** 2).sum() + 0.01 * pts.sum()
    loss.backward()
    ba = gpu_setup(sc, "fp64", **SOLVE)
    ba.solve()
    c_np, p_np = ba.get_params()
    np.testing.assert_allclose(cams.detach().cpu().numpy(), c_np, rtol=0, atol=1e-12)
    g_c = np.zeros_like(c_np)
    g_c[:, 4:7] = 2.0 * (c_np[:, 4:7] - sc.cams_gt[:, 4:7])
    gxy, gd = ba.adjoint(g_c, np.full_like(p_np, 0.01))
    np.testing.assert_allclose(xy.grad.cpu().numpy(), gxy, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(depth.grad.cpu().numpy(), gd, rtol=1e-5, atol=1e-7)
