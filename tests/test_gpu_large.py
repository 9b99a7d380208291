"""GPU checks at the benchmark workload: the 1000-camera scene (500k points, 3,972,448
observations), in the launch configuration bench.py times (PCG eta = 1e-6, 100 iterations).

* extraction: active sets bit-exact against the oracle over the whole scene;
* normal-equation blocks: V_p and g_p of 300 sampled points and U_c, g_c of 6 sampled
  cameras recomputed by the oracle's residual and Jacobian functions, observation by
  observation (float64 path, 1e-9 relative);
* the benchmark configuration itself (mixed precision) stays on the float64 trajectory over
  4 LM steps (costs 1e-6 relative, RMS 1e-4 px), with the same accept decisions.
"""
import numpy as np
import pytest

from oracle.lm import extract, Options, State
from oracle.model import Problem, residuals, jacobians, huber
from scenes import make_scene
from tests._common import gpu_setup, rel_err

pytestmark = pytest.mark.gpu

BENCH = dict(pcg_rel_tol=1e-6, pcg_max_iters=100)
_CACHE = {}


def large():
    if "sc" not in _CACHE:
        sc = make_scene("large")
        prob = Problem.from_scene(sc)
        opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px)
        st = State.initial(sc.cams0, sc.points0, opts)
        _CACHE.update(sc=sc, prob=prob, opts=opts, st=st, ex=extract(prob, st, opts))
    return _CACHE["sc"], _CACHE["prob"], _CACHE["st"], _CACHE["ex"]


def test_large_extraction_bit_exact():
    sc, prob, st, ex = large()
    ba = gpu_setup(sc, "mixed", **BENCH)
    rep = ba.lm_step()
    ac, ap, ao = ba.get_active()
    np.testing.assert_array_equal(ac, ex.cam_active)
    np.testing.assert_array_equal(ap, ex.pt_active)
    np.testing.assert_array_equal(ao, ex.obs_active)
    assert rep["n_obs_active"] == ex.obs.size and rep["fixpoint_rounds"] == ex.rounds


def _blocks(prob, st, obs, huber_px):
    """Per-observation w J^T J and w J^T e pieces of the oracle (float64)."""
    e, Xc, R = residuals(prob, st.q, st.c, st.X, obs)
    _, w, _ = huber(np.sum(e * e, axis=1), huber_px)
    Jc, Jp = jacobians(prob, Xc, R, prob.cam_idx[obs])
    return e, w, Jc, Jp


def test_large_normal_blocks_sampled():
    sc, prob, st, ex = large()
    ba = gpu_setup(sc, "fp64", **BENCH)
    ba.lm_step()
    U, gc, V, gp = ba.get_normal_blocks()
    rng = np.random.default_rng(11)
    pts = rng.choice(ex.pts, size=300, replace=False)
    obs = ex.obs[np.isin(prob.pt_idx[ex.obs], pts)]
    e, w, Jc, Jp = _blocks(prob, st, obs, sc.huber_px)
    Vo = np.zeros((sc.n_points, 3, 3))
    go = np.zeros((sc.n_points, 3))
    np.add.at(Vo, prob.pt_idx[obs], w[:, None, None] * np.einsum("nri,nrj->nij", Jp, Jp))
    np.add.at(go, prob.pt_idx[obs], w[:, None] * np.einsum("nri,nr->ni", Jp, e))
    assert rel_err(V[pts], Vo[pts]) < 1e-9
    assert rel_err(gp[pts], go[pts]) < 1e-9
    cams = rng.choice(ex.cams, size=6, replace=False)
    for c in cams:
        o = ex.obs[prob.cam_idx[ex.obs] == c]
        e, w, Jc, Jp = _blocks(prob, st, o, sc.huber_px)
        Uo = np.einsum("n,nri,nrj->ij", w, Jc, Jc)
        gco = np.einsum("n,nri,nr->i", w, Jc, e)
        assert rel_err(U[c], Uo) < 1e-9, c
        assert rel_err(gc[c], gco) < 1e-9, c


def test_large_bench_configuration_tracks_fp64():
    sc, _, _, _ = large()
    runs = {}
    for prec in ("fp64", "mixed"):
        ba = gpu_setup(sc, prec, **BENCH)
        runs[prec] = [ba.lm_step() for _ in range(4)]
        ba.close()
    for k, (a, b) in enumerate(zip(runs["fp64"], runs["mixed"])):
        print(f"step {k}: cost fp64 {a['cost_before']:.9e} mixed {b['cost_before']:.9e}, "
              f"PCG {a['pcg_iters']}/{b['pcg_iters']}, accepted {a['accepted']}/{b['accepted']}")
        assert abs(a["cost_before"] - b["cost_before"]) <= 1e-6 * a["cost_before"], k
        assert abs(a["rms_px"] - b["rms_px"]) <= 1e-4, k
        assert a["accepted"] == b["accepted"], k
