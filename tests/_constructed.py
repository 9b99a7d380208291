"""Hand-built scenes whose LM behaviour has a closed form, shared by the oracle pins and the
GPU parity tests.

* ``near_depth_scene``: one fixed camera at the origin looking down +z, one point on its
  optical axis at z = 0.2 m observed exactly at the principal point, with a valid depth
  prior of 0.05 m (closer than the 0.1 m validity bound, Eq. (10)). The two pixel rows have
  zero residual and do not involve z; the inverse-depth row r = lambda_d (1/z - 1/d) pulls
  the point towards 0.05 m. With H_zz = lambda_d^2 / z^4 and the Marquardt damping
  lambda H_zz, the damped Gauss-Newton step on z is (z - z^2/d) / (1 + lambda), so the
  candidate depth is 0.2 - 0.6 / (1 + lambda): at or below 0.1 m for every lambda < 5, when
  the candidate must be rejected with an infinite cost.
* ``embedded_near_depth_scene``: the same point added in front of camera 0 (fixed) of the
  tiny scene; the rest of the scene is free, so the same rejection happens inside an
  ordinary step.
* ``gp_behind_scene``: for global positioning, a point 2 m behind camera 0 (fixed) of an
  exact tiny scene, seen by camera 0 at its principal point with a free scale and by the
  cameras that have it in front with pinned scales. The free scale's own optimum is
  v.(X - c) / |X - c|^2 = -0.5 while it starts at 1 / |X - c| = 0.5, so a lightly damped
  step takes it below 0 (rejected: a scale is an inverse distance).
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from scenes import make_scene
from scenes.generate import Scene


def near_depth_scene(z0: float = 0.2, d_prior: float = 0.05, lambda_d: float = 1.0) -> Scene:
    cams = np.array([[1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]])
    intr = np.array([[500.0, 320.0, 240.0]])
    pts = np.array([[0.0, 0.0, z0]])
    return Scene(name="near_depth", seed=0, img_w=640, img_h=480, cams_gt=cams.copy(),
                 points_gt=pts.copy(), intr=intr, cams0=cams.copy(), points0=pts.copy(),
                 cam_idx=np.array([0], np.int32), pt_idx=np.array([0], np.int32),
                 xy=np.array([[320.0, 240.0]], np.float32),
                 depth=np.array([d_prior], np.float32), depth_valid=np.array([1], np.uint8),
                 is_outlier=np.array([False]), use_depth=True, lambda_d=lambda_d,
                 fixed=np.array([0], np.int32))


def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def embedded_near_depth_scene(n_points: int = 200) -> Scene:
    """The tiny scene (camera 0 fixed, depth rows with lambda_d = 1, every other prior
    invalid) plus one point 0.2 m in front of camera 0 on its optical axis, observed at the
    principal point, with a valid prior of 0.05 m."""
    sc = make_scene("tiny", n_points=n_points)
    R0 = _rot(sc.cams0[0, :4])
    c0 = sc.cams0[0, 4:7]
    X = c0 + 0.2 * R0[2]                 # R0 maps world to camera: row 2 is the optical axis
    n = sc.n_obs
    return replace(
        sc, points_gt=np.vstack([sc.points_gt, X]), points0=np.vstack([sc.points0, X]),
        cam_idx=np.append(sc.cam_idx, 0).astype(np.int32),
        pt_idx=np.append(sc.pt_idx, sc.n_points).astype(np.int32),
        xy=np.vstack([sc.xy, np.array([[320.0, 240.0]], sc.xy.dtype)]),
        depth=np.append(sc.depth, 0.05).astype(np.float32),
        depth_valid=np.append(np.zeros(n, np.uint8), 1).astype(np.uint8),
        is_outlier=np.append(sc.is_outlier, False), use_depth=True, lambda_d=1.0,
        fixed=np.array([0], np.int32))


def gp_behind_scene(n_points: int = 120) -> Scene:
    """An exact tiny scene (true rotations, half the priors valid, camera 0 fixed) plus one
    point 2 m behind camera 0, observed by camera 0 at its principal point (free scale) and
    by every camera that has it more than 0.5 m in front (exact pixel and prior, pinned)."""
    sc = make_scene("tiny", noise_px=0.0, exact=True, depth_sigma=0.0, prior_frac=0.5,
                    use_depth=True, lambda_d=1.0, n_points=n_points)
    cams0 = np.concatenate([sc.cams_gt[:, :4], sc.cams0[:, 4:7]], axis=1)
    q0, c0 = sc.cams_gt[0, :4], sc.cams_gt[0, 4:7]
    X = c0 - 2.0 * _rot(q0)[2]
    cam, xy, dep, val = [0], [[320.0, 240.0]], [1.0], [0]
    for i in range(1, sc.n_cams):
        R, c = _rot(sc.cams_gt[i, :4]), sc.cams_gt[i, 4:7]
        Xc = R @ (X - c)
        if Xc[2] > 0.5:
            f, cx, cy = sc.intr[i]
            cam.append(i)
            xy.append([f * Xc[0] / Xc[2] + cx, f * Xc[1] / Xc[2] + cy])
            dep.append(Xc[2])
            val.append(1)
    assert len(cam) >= 3, "the added point needs pinned observations"
    k = len(cam)
    # float32 pixels, as the library takes them (the oracle reads the same rounded values)
    return replace(
        sc, cams0=cams0, points_gt=np.vstack([sc.points_gt, X]),
        points0=np.vstack([sc.points0, X]),
        cam_idx=np.append(sc.cam_idx, cam).astype(np.int32),
        pt_idx=np.append(sc.pt_idx, [sc.n_points] * k).astype(np.int32),
        xy=np.vstack([sc.xy, np.array(xy)]).astype(np.float32),
        depth=np.append(sc.depth, dep).astype(np.float32),
        depth_valid=np.append(sc.depth_valid, val).astype(np.uint8),
        is_outlier=np.append(sc.is_outlier, [False] * k), fixed=np.array([0], np.int32))
