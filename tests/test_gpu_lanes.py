"""GPU parity at both ends of the lanes-per-point choice. The point-major kernels take G = 2,
4, 8 or 16 lanes per point from the mean number of views per point. The other GPU tests run
4-9 views (4 and 8 lanes); here the 10-camera scene is seen by 2 cameras per point (2 lanes)
or by all 10 (16 lanes):

* one LM step, float64, against the oracle's Cholesky solve (1e-6 relative), with the same
  accept decision, candidate cost (1e-9) and model decrease (1e-7);
* the mixed-precision step takes the same decision with a candidate cost within 1e-6 relative
  of float64's (the bar of the other mixed-precision tests; the step vector itself differs by
  the float32 Jacobian's rounding times the conditioning, 7e-5 relative here);
* one global-positioning step at 16 lanes (the candidate's per-lane partial sums) against the
  oracle's (cost before 1e-12, model decrease 1e-6, parameters 1e-6).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle.gp import GpOptions, GpState, gp_step
from oracle.lm import lm_step
from oracle.model import Problem
from scenes import make_scene
from tests._common import oracle_setup, gpu_setup, full_delta, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("views", [2, 10])
def test_lm_step_at_lane_extremes(views):
    sc = make_scene("tiny", views=views)
    assert sc.cam_idx.size == views * sc.n_points
    prob, opts, st = oracle_setup(sc, lambda_init=1e-3)
    new, orep = lm_step(prob, st, opts)
    steps = {}
    for prec in ("fp64", "mixed"):
        ba = gpu_setup(sc, prec, lambda_init=1e-3, pcg_rel_tol=1e-13, pcg_max_iters=2000)
        rep = ba.lm_step()
        steps[prec] = ba.get_last_step() + (rep,)
        ba.close()
    dc, dp, rep = steps["fp64"]
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points)
    print(f"{views} views: step vs oracle {rel_err(dc, odc):.2e} / {rel_err(dp, odp):.2e}, "
          f"mixed vs fp64 {rel_err(steps['mixed'][0], dc):.2e}")
    assert rel_err(dc, odc) < 1e-6 and rel_err(dp, odp) < 1e-6
    assert bool(rep["accepted"]) == orep.accepted
    if np.isfinite(orep.cost_after):
        assert abs(rep["cost_after"] - orep.cost_after) <= 1e-9 * orep.cost_after
    assert abs(rep["model_decrease"] - orep.model_decrease) <= 1e-7 * abs(orep.model_decrease)
    mrep = steps["mixed"][2]
    assert mrep["accepted"] == rep["accepted"]
    assert abs(mrep["cost_after"] - rep["cost_after"]) <= 1e-6 * rep["cost_before"]


def test_gp_step_at_sixteen_lanes():
    sc = make_scene("tiny", views=10, prior_frac=0.5, use_depth=True, lambda_d=1.0)
    cams0 = np.concatenate([sc.cams_gt[:, :4], sc.cams0[:, 4:7]], axis=1)
    sc = replace(sc, cams0=cams0, fixed=np.array([0], np.int32))
    prob = Problem.from_scene(sc)
    q = sc.cams0[:, :4]
    opts = GpOptions(lambda_init=1e-3)
    st = GpState.initial(prob, q, sc.cams0, sc.points0, opts)
    new, orep = gp_step(prob, q, st, opts)
    ba = gpu_setup(sc, "fp64", gp_huber=0.1, lambda_init=1e-3, pcg_rel_tol=1e-13,
                   pcg_max_iters=3000)
    rep = ba.gp_step()
    assert abs(rep["cost_before"] - orep.cost_before) <= 1e-12 * orep.cost_before
    assert abs(rep["model_decrease"] - orep.model_decrease) <= 1e-6 * abs(orep.model_decrease)
    assert bool(rep["accepted"]) == orep.accepted
    cams, pts = ba.get_params()
    s = ba.gp_scales()
    print(f"GP 16 lanes: centres {rel_err(cams[:, 4:7] - st.c, new.c - st.c):.2e}, "
          f"points {rel_err(pts - st.X, new.X - st.X):.2e}, scales {rel_err(s - st.s, new.s - st.s):.2e}")
    assert rel_err(cams[:, 4:7] - st.c, new.c - st.c) < 1e-6
    assert rel_err(pts - st.X, new.X - st.X) < 1e-6
    assert rel_err(s - st.s, new.s - st.s) < 1e-6
