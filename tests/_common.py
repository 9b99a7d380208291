"""Shared test helpers: build a GPU context or an oracle problem from a seeded scene."""
import numpy as np

from oracle.lm import Options, State
from oracle.model import Problem


def oracle_setup(sc, **kw):
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px, **kw)
    prob = Problem.from_scene(sc)
    st = State.initial(sc.cams0, sc.points0, opts)
    return prob, opts, st


def gpu_setup(sc, precision="fp64", **kw):
    from paper_2510_13310_amd import BundleAdjuster
    opts = dict(huber_px=sc.huber_px, filter_px=sc.filter_px, img_w=sc.img_w, img_h=sc.img_h)
    opts.update(kw)
    ba = BundleAdjuster(sc.cams0, sc.intr, sc.points0, precision=precision, **opts)
    ba.set_observations(sc.cam_idx, sc.pt_idx, sc.xy)
    if sc.use_depth:
        ba.set_depth_priors(sc.depth, sc.depth_valid, sc.lambda_d)
    if sc.fixed.size:
        ba.set_fixed_cameras(sc.fixed)
    return ba


def full_delta(ex, delta, n_cams, n_points, d=6):
    """Scatter an oracle compact step into full (C x d, P x 3) arrays."""
    nc = d * ex.cams.size
    dc = np.zeros((n_cams, d))
    dp = np.zeros((n_points, 3))
    dc[ex.cams] = delta[:nc].reshape(-1, d)
    dp[ex.pts] = delta[nc:].reshape(-1, 3)
    return dc, dp


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
