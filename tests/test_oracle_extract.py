"""Pins of the oracle's dynamic parameter extraction (Sec. IV-B, Eqs. (10)-(15))."""
import itertools

import numpy as np
import pytest

from oracle.extract import geometric_validity, activity_fixpoint, ranks, observation_rows
from oracle.model import Problem
from oracle.lm import Options, State, lm_step, extract, linearize
from scenes import make_scene


def _random_incidence(rng, C, P, N, fixed=(), prior_p=0.5, lam=1.0):
    pairs = set()
    while len(pairs) < N:
        pairs.add((int(rng.integers(C)), int(rng.integers(P))))
    cam, pt = np.array(sorted(pairs)).T
    m = rng.random(N) < prior_p
    return Problem(n_cams=C, n_points=P, intr=np.tile([500.0, 320, 240], (C, 1)),
                   cam_idx=cam, pt_idx=pt, xy=np.zeros((N, 2)), dinv=m * 0.5,
                   prior_mask=m, lambda_d=lam, img_w=640, img_h=480,
                   fixed=np.array(fixed, np.int64))


def _brute_force_greatest_closed_set(prob, valid, need_p, need_c):
    """Union of all observation subsets S of the valid set such that every observation in S
    has a point with >= need_p rows in S and a camera that is fixed or has >= need_c rows
    in S. Closed sets are closed under union, so the union is the greatest one."""
    fixed = np.zeros(prob.n_cams, bool)
    fixed[prob.fixed] = True
    rows = observation_rows(prob)
    idx = np.nonzero(valid)[0]
    best = np.zeros(prob.n_obs, bool)
    for r in range(len(idx) + 1):
        for sub in itertools.combinations(idx, r):
            S = np.zeros(prob.n_obs, bool)
            S[list(sub)] = True
            ok = True
            for k in sub:
                rp = rows[S & (prob.pt_idx == prob.pt_idx[k])].sum()
                rc = rows[S & (prob.cam_idx == prob.cam_idx[k])].sum()
                if rp < need_p or not (fixed[prob.cam_idx[k]] or rc >= need_c):
                    ok = False
                    break
            if ok:
                best |= S
    return best


@pytest.mark.parametrize("seed", range(6))
def test_fixpoint_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    prob = _random_incidence(rng, C=4, P=6, N=12, fixed=(0,) if seed % 2 else ())
    valid = rng.random(prob.n_obs) < 0.85
    act, cam_ok, pt_ok, _ = activity_fixpoint(prob, valid, "rows")
    ref = _brute_force_greatest_closed_set(prob, valid, 3, 6)
    np.testing.assert_array_equal(act, ref)
    # entity flags are consistent with the surviving observations
    rows = observation_rows(prob)
    rp = np.bincount(prob.pt_idx[act], rows[act], minlength=prob.n_points)
    np.testing.assert_array_equal(pt_ok, rp >= 3)


def test_literal_rule_keeps_every_valid_observation():
    rng = np.random.default_rng(3)
    prob = _random_incidence(rng, C=5, P=8, N=16)
    valid = rng.random(prob.n_obs) < 0.6
    act, cam_ok, pt_ok, rounds = activity_fixpoint(prob, valid, "literal")
    np.testing.assert_array_equal(act, valid)
    np.testing.assert_array_equal(pt_ok, np.bincount(prob.pt_idx[valid], minlength=8) > 0)
    assert rounds == 1


def test_ranks_are_ascending_original_order():
    a = np.array([0, 1, 1, 0, 1, 0, 0, 1], bool)
    rank, members = ranks(a)
    np.testing.assert_array_equal(members, [1, 2, 4, 7])
    np.testing.assert_array_equal(rank, [-1, 0, 1, -1, 2, -1, -1, 3])


def test_validity_depth_frustum_and_filter():
    """z > 0.1 strictly, projection inside [0,W)x[0,H), 2-D error <= filter."""
    q = np.tile([1.0, 0, 0, 0], (1, 1))
    c = np.zeros((1, 3))
    X = np.array([[0.0, 0.0, 0.1], [0.0, 0.0, 0.1000001], [0.0, 0.0, -5.0],
                  [10.0, 0.0, 2.0], [0.0, 0.0, 3.0], [0.0, 0.0, 3.0],
                  [-320.0 * 2.0 / 500.0, 0.0, 2.0]])   # last one projects onto u = 0 (inside)
    P = X.shape[0]
    xy = np.array([[320, 240]] * P, float)
    xy[5] = [320 + 3.0, 240 + 4.0]         # 5 px error
    prob = Problem(n_cams=1, n_points=P, intr=np.array([[500.0, 320, 240]]),
                   cam_idx=np.zeros(P, np.int64), pt_idx=np.arange(P), xy=xy,
                   dinv=np.zeros(P), prior_mask=np.zeros(P, bool), lambda_d=0.0,
                   img_w=640, img_h=480)
    v = geometric_validity(prob, q, c, X, 0.1, 0.0)
    np.testing.assert_array_equal(v, [False, True, False, False, True, True, True])
    v = geometric_validity(prob, q, c, X, 0.1, 5.0)
    assert v[5]
    v = geometric_validity(prob, q, c, X, 0.1, 4.999)
    assert not v[5]


def test_validity_is_reevaluated_each_iteration():
    """A point pushed behind z = 0.1 drops out of the active set and returns when moved
    back (extraction is a pure function of the current parameters)."""
    sc = make_scene("tiny")
    prob = Problem.from_scene(sc)
    opts = Options()
    st = State.initial(sc.cams_gt, sc.points_gt, opts)
    j = 5
    ex0 = extract(prob, st, opts)
    assert ex0.pt_active[j]
    cam = prob.cam_idx[prob.pt_idx == j][0]
    from oracle.geometry import quat_to_rot
    R = quat_to_rot(st.q[cam])
    moved = st.copy()
    moved.X[j] = st.c[cam] + R.T @ np.array([0.0, 0.0, 0.05])   # 5 cm in front: z < 0.1
    ex1 = extract(prob, moved, opts)
    k = np.nonzero((prob.pt_idx == j) & (prob.cam_idx == cam))[0][0]
    assert not ex1.valid[k]
    ex2 = extract(prob, st, opts)
    assert ex2.valid[k] and ex2.pt_active[j]


def test_medium_extraction_invariants():
    """No all-zero Jacobian column (Sec. IV-B), the injected perturbed cameras and
    all-outlier points are inactive, and a step leaves inactive parameters bit-identical."""
    sc = make_scene("medium")
    prob = Problem.from_scene(sc)
    opts = Options(huber_px=sc.huber_px, filter_px=sc.filter_px)
    st = State.initial(sc.cams0, sc.points0, opts)
    ex = extract(prob, st, opts)
    bad = sc.notes["perturbed_cameras"]
    assert not ex.cam_active[bad].any()
    assert not ex.pt_active[sc.notes["all_outlier_points"]].any()
    lin = linearize(prob, st, ex, opts.huber_px)
    colnorm = np.sqrt(np.asarray(lin.J.multiply(lin.J).sum(axis=0))).ravel()
    assert colnorm.min() > 0
    # every active entity carries at least its dimension in rows
    rows = observation_rows(prob)
    rp = np.bincount(prob.pt_idx[ex.obs], rows[ex.obs], minlength=prob.n_points)
    rc = np.bincount(prob.cam_idx[ex.obs], rows[ex.obs], minlength=prob.n_cams)
    assert rp[ex.pt_active].min() >= 3 and rc[ex.cam_active].min() >= 6
    st.lam = 1.0
    new, rep = lm_step(prob, st, opts)
    assert rep.accepted
    np.testing.assert_array_equal(new.q[~ex.cam_active], st.q[~ex.cam_active])
    np.testing.assert_array_equal(new.c[~ex.cam_active], st.c[~ex.cam_active])
    np.testing.assert_array_equal(new.X[~ex.pt_active], st.X[~ex.pt_active])
    assert np.any(new.X[ex.pt_active] != st.X[ex.pt_active])


def test_empty_active_set():
    sc = make_scene("tiny")
    prob = Problem.from_scene(sc)
    opts = Options()
    st = State.initial(sc.cams0, sc.points0, opts)
    st.X[:] = np.array([0.0, 100.0, 0.0])        # far above every camera: out of frustum
    new, rep = lm_step(prob, st, opts)
    assert rep.status == "empty" and rep.n_obs == 0
    np.testing.assert_array_equal(new.X, st.X)
