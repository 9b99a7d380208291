"""GPU checks at the 5000-camera workload (2M points, about 12M observations, 5 % outliers,
depth priors on 30 %), in the launch configuration bench.py --scene xl times (PCG eta = 1e-6,
100 iterations). Here the matvec records of the 5000 cameras (400 KB in float32) exceed the
LDS, so the point pass reads them through L2 (the other per-observation kernels likewise).

* extraction: active sets bit-exact against the oracle over the whole scene;
* normal-equation blocks: V_p and g_p of 300 sampled points and U_c, g_c of 6 sampled
  cameras recomputed by the oracle's residual and Jacobian functions (float64, 1e-9);
* the mixed path stays on the float64 trajectory over 3 LM steps (costs 1e-6 relative,
  RMS 1e-4 px, the same decisions).
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


def xl():
    if "sc" not in _CACHE:
        sc = make_scene("xl")
        prob = Problem.from_scene(sc)
        opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px)
        st = State.initial(sc.cams0, sc.points0, opts)
        _CACHE.update(sc=sc, prob=prob, st=st, ex=extract(prob, st, opts))
    return _CACHE["sc"], _CACHE["prob"], _CACHE["st"], _CACHE["ex"]


def test_xl_extraction_bit_exact():
    sc, prob, st, ex = xl()
    assert sc.n_cams == 5000 and sc.n_obs > 11_000_000
    ba = gpu_setup(sc, "mixed", **BENCH)
    rep = ba.lm_step()
    ac, ap, ao = ba.get_active()
    np.testing.assert_array_equal(ac, ex.cam_active)
    np.testing.assert_array_equal(ap, ex.pt_active)
    np.testing.assert_array_equal(ao, ex.obs_active)
    assert rep["n_obs_active"] == ex.obs.size and rep["fixpoint_rounds"] == ex.rounds


def test_xl_normal_blocks_sampled():
    sc, prob, st, ex = xl()
    ba = gpu_setup(sc, "fp64", **BENCH)
    ba.lm_step()
    U, gc, V, gp = ba.get_normal_blocks()
    rng = np.random.default_rng(12)
    pts = rng.choice(ex.pts, size=300, replace=False)
    obs = ex.obs[np.isin(prob.pt_idx[ex.obs], pts)]
    e, Xc, R = residuals(prob, st.q, st.c, st.X, obs)
    _, w, _ = huber(np.sum(e * e, axis=1), sc.huber_px)
    Jc, Jp = jacobians(prob, Xc, R, prob.cam_idx[obs])
    Vo = np.zeros((sc.n_points, 3, 3))
    go = np.zeros((sc.n_points, 3))
    np.add.at(Vo, prob.pt_idx[obs], w[:, None, None] * np.einsum("nri,nrj->nij", Jp, Jp))
    np.add.at(go, prob.pt_idx[obs], w[:, None] * np.einsum("nri,nr->ni", Jp, e))
    assert rel_err(V[pts], Vo[pts]) < 1e-9
    assert rel_err(gp[pts], go[pts]) < 1e-9
    for c in rng.choice(ex.cams, size=6, replace=False):
        o = ex.obs[prob.cam_idx[ex.obs] == c]
        e, Xc, R = residuals(prob, st.q, st.c, st.X, o)
        _, w, _ = huber(np.sum(e * e, axis=1), sc.huber_px)
        Jc, _ = jacobians(prob, Xc, R, prob.cam_idx[o])
        assert rel_err(U[c], np.einsum("n,nri,nrj->ij", w, Jc, Jc)) < 1e-9, c
        assert rel_err(gc[c], np.einsum("n,nri,nr->i", w, Jc, e)) < 1e-9, c


def test_xl_mixed_tracks_fp64():
    sc, _, _, _ = xl()
    runs = {}
    for prec in ("fp64", "mixed"):
        ba = gpu_setup(sc, prec, **BENCH)
        runs[prec] = [ba.lm_step() for _ in range(3)]
        ba.close()
    for k, (a, b) in enumerate(zip(runs["fp64"], runs["mixed"])):
        print(f"xl step {k}: cost fp64 {a['cost_before']:.9e} mixed {b['cost_before']:.9e}, "
              f"PCG {a['pcg_iters']}/{b['pcg_iters']}, accepted {a['accepted']}/{b['accepted']}")
        assert abs(a["cost_before"] - b["cost_before"]) <= 1e-6 * a["cost_before"], k
        assert abs(a["rms_px"] - b["rms_px"]) <= 1e-4, k
        assert a["accepted"] == b["accepted"], k
