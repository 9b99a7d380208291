"""GPU parity of the explicit reduced camera system (solver = explicit): the same LM step with
S assembled as D x D blocks and multiplied as a sparse block matrix.

* one step against the oracle's dense Schur complement + Cholesky (PCG to 1e-13): 1e-6
  relative, as the matrix-free solver; also with focal-length refinement (7 x 7 blocks);
* twelve fixed-gauge LM steps: the same decisions as the matrix-free solver and the oracle,
  parameters within 1e-6 relative of the oracle's;
* bitwise reproducible (the blocks are summed in a fixed order);
* at the 1000-camera workload in the benchmark's PCG settings, the mixed-precision explicit
  solver follows the matrix-free one over 3 steps (costs 1e-6 relative, same decisions).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle.lm import lm_step, Options, State
from oracle.model import Problem
from scenes import make_scene
from tests._common import oracle_setup, gpu_setup, full_delta, rel_err

pytestmark = pytest.mark.gpu

_SC = {}


def scene(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _SC:
        _SC[key] = make_scene(name, **kw)
    return _SC[key]


@pytest.mark.parametrize("name,lam", [("tiny", 1e-3), ("medium", 1e-2), ("medium", 1.0)])
def test_explicit_single_step_matches_cholesky(name, lam):
    sc = scene(name)
    prob, opts, st = oracle_setup(sc, lambda_init=lam)
    new, orep = lm_step(prob, st, opts)
    ba = gpu_setup(sc, "fp64", solver="explicit", lambda_init=lam, pcg_rel_tol=1e-13,
                   pcg_max_iters=2000)
    rep = ba.lm_step()
    dc, dp = ba.get_last_step()
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points)
    print(f"{name} lam {lam}: cams {rel_err(dc, odc):.2e}, points {rel_err(dp, odp):.2e}, "
          f"PCG {rep['pcg_iters']}")
    assert rel_err(dc, odc) < 1e-6 and rel_err(dp, odp) < 1e-6
    assert bool(rep["accepted"]) == orep.accepted
    assert abs(rep["model_decrease"] - orep.model_decrease) <= 1e-7 * abs(orep.model_decrease)


def test_explicit_focal_single_step():
    sc = scene("medium")
    rng = np.random.default_rng(3)
    intr = sc.intr.copy()
    intr[:, 0] *= 1.0 + rng.uniform(-0.02, 0.02, size=sc.n_cams)
    sc = replace(sc, intr=intr)
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px, refine_focal=True,
                   lambda_init=1e-2)
    prob = Problem.from_scene(sc)
    st = State.initial(sc.cams0, sc.points0, opts, focal=intr[:, 0])
    new, orep = lm_step(prob, st, opts)
    ba = gpu_setup(sc, "fp64", solver="explicit", refine_focal=1, lambda_init=1e-2,
                   pcg_rel_tol=1e-13, pcg_max_iters=3000)
    rep = ba.lm_step()
    dc, dp = ba.get_last_step()
    odc, odp = full_delta(orep.extraction, orep.delta, sc.n_cams, sc.n_points, d=7)
    assert rel_err(dc, odc) < 1e-6 and rel_err(dp, odp) < 1e-6
    assert bool(rep["accepted"]) == orep.accepted


def test_explicit_trajectory_fixed_gauge():
    sc = replace(scene("medium"), fixed=np.array([0], np.int32))
    prob, opts, st = oracle_setup(sc)
    kw = dict(pcg_rel_tol=1e-13, pcg_max_iters=3000)
    be = gpu_setup(sc, "fp64", solver="explicit", **kw)
    bi = gpu_setup(sc, "fp64", **kw)
    for k in range(12):
        st, orep = lm_step(prob, st, opts)
        re, ri = be.lm_step(), bi.lm_step()
        assert bool(re["accepted"]) == orep.accepted == bool(ri["accepted"]), k
        assert abs(re["cost_before"] - orep.cost_before) <= 1e-9 * orep.cost_before, k
    cams, pts = be.get_params()
    d = max(rel_err(pts, st.X), rel_err(cams[:, 4:], st.c))
    print(f"explicit trajectory: max rel diff to the oracle {d:.3e}")
    assert d < 1e-6


def test_explicit_bitwise_reproducible():
    sc = scene("medium")
    runs = []
    for _ in range(2):
        ba = gpu_setup(sc, "mixed", solver="explicit")
        for _ in range(3):
            ba.lm_step()
        runs.append(ba.get_params())
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])


def test_explicit_large_follows_matrix_free():
    sc = scene("large")
    kw = dict(pcg_rel_tol=1e-6, pcg_max_iters=100)
    runs = {}
    for solver in ("implicit", "explicit"):
        ba = gpu_setup(sc, "mixed", solver=solver, **kw)
        runs[solver] = [ba.lm_step() for _ in range(3)]
        ba.close()
    for k, (a, b) in enumerate(zip(runs["implicit"], runs["explicit"])):
        print(f"step {k}: cost {a['cost_before']:.9e} / {b['cost_before']:.9e}, "
              f"PCG {a['pcg_iters']} / {b['pcg_iters']}")
        assert abs(a["cost_before"] - b["cost_before"]) <= 1e-6 * a["cost_before"], k
        assert a["accepted"] == b["accepted"], k
