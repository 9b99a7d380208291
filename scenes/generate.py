"""Seeded synthetic scenes for the bundle-adjustment hot path.

Only input generation lives here: camera rigs, 3-D points, which cameras observe which
point, noisy pixel observations, outliers, depth priors and the perturbed initial estimate.
Both the CPU oracle and the GPU library read these arrays; this module imports neither of
them and holds no part of the solver (no Jacobians, no normal equations, no solve).

Conventions shared by every scene
---------------------------------
* Camera ``i`` is ``[qw, qx, qy, qz, cx, cy, cz]``: a unit quaternion for the world-to-camera
  rotation ``R_i`` and the camera centre ``c_i``; a world point maps to ``R_i (X - c_i)``.
  This is the {centre, quaternion} extrinsic layout of the paper's BA objective (Sec. III-B).
* OpenCV camera axes (x right, y down, z forward); look-at with world up ``+y``.
* Pinhole intrinsics ``[f, cx, cy]`` = ``[500, 320, 240]`` px on a 640x480 image.
* Pixel noise N(0, 1 px^2) per coordinate; outliers are replaced by a uniform pixel in the
  image; observations are rounded to float32 once.
* Depth priors: ``d_hat = z_true * exp(N(0, 0.05^2))`` (5 % log-normal), valid by Bernoulli.
* "Perturbed by a degrees": a random axis on S^2 rotated by exactly ``a``; translation and
  point perturbations use a random direction with an exact magnitude.

The paper evaluates on public datasets (MipNeRF360, DTU, ScanNet, ScanNet++, 1DSfM); none is
available here, so these scenes stand in for them with the sizes of the benchmark workloads.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import numpy as np
from scipy.spatial.transform import Rotation

SCENE_NAMES = ("tiny", "medium", "large", "adjoint", "xl")

IMG_W, IMG_H = 640, 480
FOCAL, PPX, PPY = 500.0, 320.0, 240.0


@dataclass
class Scene:
    name: str
    seed: int
    img_w: int
    img_h: int
    cams_gt: np.ndarray      # C x 7 float64
    points_gt: np.ndarray    # P x 3 float64
    intr: np.ndarray         # C x 3 float64 [f, cx, cy]
    cams0: np.ndarray        # C x 7 float64, initial estimate
    points0: np.ndarray      # P x 3 float64, initial estimate
    cam_idx: np.ndarray      # N int32
    pt_idx: np.ndarray       # N int32
    xy: np.ndarray           # N x 2 float32 (float64 for ``exact`` oracle-only scenes)
    depth: np.ndarray        # N float32 (noisy prior for every observation)
    depth_valid: np.ndarray  # N uint8 (1 = prior usable)
    is_outlier: np.ndarray   # N bool
    use_depth: bool = False
    lambda_d: float = 0.0
    huber_px: float = 0.0
    filter_px: float = 0.0
    fixed: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    notes: dict = field(default_factory=dict)

    @property
    def n_cams(self) -> int:
        return int(self.cams_gt.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.points_gt.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.cam_idx.shape[0])


# --------------------------------------------------------------------------- rig helpers

def _look_at(centres: np.ndarray, targets: np.ndarray) -> np.ndarray:
    """World-to-camera rotations whose +z axis points from ``centres`` to ``targets``."""
    up = np.array([0.0, 1.0, 0.0])
    z = targets - centres
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    y = -(up[None, :] - (z @ up)[:, None] * z)       # image y points down
    y /= np.linalg.norm(y, axis=1, keepdims=True)
    x = np.cross(y, z)
    return np.stack([x, y, z], axis=1)                # rows are the camera axes


def _yaw_dirs(yaw: np.ndarray) -> np.ndarray:
    return np.stack([np.sin(yaw), np.zeros_like(yaw), np.cos(yaw)], axis=1)


def _rot_to_quat_wxyz(R: np.ndarray) -> np.ndarray:
    q = Rotation.from_matrix(R).as_quat()              # x, y, z, w
    q = np.concatenate([q[:, 3:4], q[:, :3]], axis=1)
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    return q


def _quat_wxyz_to_rot(q: np.ndarray) -> np.ndarray:
    return Rotation.from_quat(np.concatenate([q[:, 1:4], q[:, 0:1]], axis=1)).as_matrix()


def _unit_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _camera_frame(R: np.ndarray, c: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Synthesis-only pinhole: camera-frame coordinates R (X - c), broadcasting."""
    return np.einsum("...ij,...j->...i", R, X - c)


def _pixels(Xc: np.ndarray) -> np.ndarray:
    return np.stack([FOCAL * Xc[..., 0] / Xc[..., 2] + PPX,
                     FOCAL * Xc[..., 1] / Xc[..., 2] + PPY], axis=-1)


def _visible(Xc: np.ndarray, zmin: float, margin: float) -> np.ndarray:
    z = Xc[..., 2]
    ok = z > zmin
    zs = np.where(ok, z, 1.0)
    u = FOCAL * Xc[..., 0] / zs + PPX
    v = FOCAL * Xc[..., 1] / zs + PPY
    return ok & (u >= margin) & (u < IMG_W - margin) & (v >= margin) & (v < IMG_H - margin)


def _pick_cameras(rng, R, c, pts, k, zmin, margin, n_cand=None, chunk=4096):
    """Per point, up to ``k`` distinct cameras chosen uniformly among those that see it.

    Exhaustive visibility for small rigs; for large rigs ``n_cand`` random candidate cameras
    are tested per point and the first ``k`` distinct visible ones kept.
    Returns (cams P x k int32 with -1 padding, count P).
    """
    C = R.shape[0]
    P = pts.shape[0]
    out = np.full((P, k), -1, np.int32)
    cnt = np.zeros(P, np.int32)
    for s in range(0, P, chunk):
        X = pts[s:s + chunk]
        n = X.shape[0]
        if n_cand is None:
            Xc = _camera_frame(R[None, :, :, :], c[None, :, :], X[:, None, :])
            vis = _visible(Xc, zmin, margin)
            key = np.where(vis, rng.random((n, C)), 2.0)
            order = np.argsort(key, axis=1)[:, :k]
            ok = np.take_along_axis(vis, order, axis=1)
            sel = np.where(ok, order, -1)
        else:
            cand = rng.integers(0, C, size=(n, n_cand))
            Xc = _camera_frame(R[cand], c[cand], X[:, None, :])
            vis = _visible(Xc, zmin, margin)
            # drop repeated candidates: keep the first occurrence in each row
            srt = np.argsort(cand, axis=1, kind="stable")
            cs = np.take_along_axis(cand, srt, axis=1)
            dup_sorted = np.zeros_like(vis)
            dup_sorted[:, 1:] = cs[:, 1:] == cs[:, :-1]
            dup = np.zeros_like(vis)
            np.put_along_axis(dup, srt, dup_sorted, axis=1)
            vis &= ~dup
            rank = np.cumsum(vis, axis=1)
            take = vis & (rank <= k)
            sel = np.full((n, k), -1, np.int64)
            rows, cols = np.nonzero(take)
            sel[rows, rank[rows, cols] - 1] = cand[rows, cols]
        out[s:s + n] = sel
        cnt[s:s + n] = (sel >= 0).sum(axis=1)
    return out, cnt


def _assemble(rng, name, seed, R_gt, c_gt, pts_gt, sel, *, noise_px, outlier_frac,
              prior_frac, rot_deg, trans_m, point_m, use_depth, lambda_d, huber_px,
              filter_px, notes=None, big_rot=None, all_outlier_points=0, depth_sigma=0.05,
              exact=False):
    C = R_gt.shape[0]
    P = pts_gt.shape[0]
    cams_gt = np.concatenate([_rot_to_quat_wxyz(R_gt), c_gt], axis=1)
    intr = np.tile(np.array([FOCAL, PPX, PPY]), (C, 1))

    pt_idx = np.repeat(np.arange(P, dtype=np.int32), sel.shape[1])
    cam_idx = sel.reshape(-1)
    keep = cam_idx >= 0
    pt_idx = pt_idx[keep]
    cam_idx = cam_idx[keep].astype(np.int32)
    N = cam_idx.shape[0]

    Xc = _camera_frame(R_gt[cam_idx], c_gt[cam_idx], pts_gt[pt_idx])
    xy = _pixels(Xc) + rng.normal(scale=noise_px, size=(N, 2)) if noise_px > 0 else _pixels(Xc)
    is_out = rng.random(N) < outlier_frac
    if all_outlier_points:
        bad = rng.choice(P, size=all_outlier_points, replace=False)
        is_out |= np.isin(pt_idx, bad)
        notes = dict(notes or {}, all_outlier_points=np.sort(bad).astype(np.int32))
    n_out = int(is_out.sum())
    xy[is_out] = np.stack([rng.random(n_out) * IMG_W, rng.random(n_out) * IMG_H], axis=1)
    # float32 like every real detector output; ``exact`` keeps float64 (oracle-only pins)
    obs_dtype = np.float64 if exact else np.float32
    xy = xy.astype(obs_dtype)

    depth = (Xc[:, 2] * np.exp(rng.normal(scale=depth_sigma, size=N))).astype(obs_dtype)
    depth_valid = (rng.random(N) < prior_frac).astype(np.uint8)

    # perturbed initial estimate
    axes = _unit_dirs(rng, C)
    rot = Rotation.from_rotvec(axes * np.deg2rad(rot_deg)).as_matrix()
    if big_rot is not None:
        # rotate about the camera's own y axis so every observation moves by ~f tan(deg)
        ids, deg = big_rot
        yaxis = np.tile(np.array([0.0, 1.0, 0.0]), (len(ids), 1))
        rot[ids] = Rotation.from_rotvec(yaxis * np.deg2rad(deg)).as_matrix()
    R0 = rot @ R_gt
    c0 = c_gt + trans_m * _unit_dirs(rng, C)
    p0 = pts_gt + point_m * _unit_dirs(rng, P)
    cams0 = np.concatenate([_rot_to_quat_wxyz(R0), c0], axis=1)

    return Scene(name=name, seed=seed, img_w=IMG_W, img_h=IMG_H, cams_gt=cams_gt,
                 points_gt=pts_gt.copy(), intr=intr, cams0=cams0, points0=p0,
                 cam_idx=cam_idx, pt_idx=pt_idx, xy=xy, depth=depth,
                 depth_valid=depth_valid, is_outlier=is_out, use_depth=use_depth,
                 lambda_d=lambda_d, huber_px=huber_px, filter_px=filter_px,
                 notes=dict(notes or {}))


def _resample_until_seen(rng, draw, R, c, k, min_views, zmin, margin, n_cand, P):
    pts = draw(P)
    sel, cnt = _pick_cameras(rng, R, c, pts, k, zmin, margin, n_cand)
    for _ in range(50):
        bad = np.nonzero(cnt < min_views)[0]
        if bad.size == 0:
            break
        pts[bad] = draw(bad.size)
        s2, c2 = _pick_cameras(rng, R, c, pts[bad], k, zmin, margin, n_cand)
        sel[bad] = s2
        cnt[bad] = c2
    else:
        raise RuntimeError("could not place every point in enough views")
    return pts, sel


def _random_walks(rng, n_seq, n_steps, half_extent, step_m=1.0, yaw_sigma_deg=5.0):
    C = n_seq * n_steps
    pos = np.zeros((C, 3))
    yaw = np.zeros(C)
    for s in range(n_seq):
        p = np.array([rng.uniform(-half_extent, half_extent), 0.0,
                      rng.uniform(-half_extent, half_extent)])
        th = rng.uniform(0, 2 * np.pi)
        for t in range(n_steps):
            i = s * n_steps + t
            pos[i] = p
            yaw[i] = th
            th += np.deg2rad(rng.normal(scale=yaw_sigma_deg))
            p = p + step_m * np.array([np.sin(th), 0.0, np.cos(th)])
            if abs(p[0]) > half_extent:
                p[0] = np.sign(p[0]) * 2 * half_extent - p[0]
                th = -th
            if abs(p[2]) > half_extent:
                p[2] = np.sign(p[2]) * 2 * half_extent - p[2]
                th = np.pi - th
    return pos, yaw


# --------------------------------------------------------------------------- scenes

def _tiny(seed, n_points=500, noise_px=1.0, views=4, **kw):
    rng = np.random.default_rng(seed)
    C = 10
    a = 2 * np.pi * np.arange(C) / C
    c = 5.0 * np.stack([np.cos(a), np.zeros(C), np.sin(a)], axis=1)
    R = _look_at(c, np.zeros((C, 3)))
    pts, sel = _resample_until_seen(
        rng, lambda n: rng.uniform(-1, 1, size=(n, 3)), R, c, views, views, 0.5, 0.0, None,
        n_points)
    opts = dict(noise_px=noise_px, outlier_frac=0.0, prior_frac=0.0, rot_deg=1.0,
                trans_m=0.02, point_m=0.05, use_depth=False, lambda_d=0.0, huber_px=0.0,
                filter_px=0.0)
    opts.update(kw)
    return _assemble(rng, "tiny", seed, R, c, pts, sel, **opts)


def _medium(seed, n_cams=100, n_points=20000, views=5, **kw):
    rng = np.random.default_rng(seed)
    C = n_cams
    c = np.stack([rng.normal(scale=0.2, size=C), rng.normal(scale=0.05, size=C),
                  -100.0 + np.arange(C) * (100.0 / C)], axis=1)
    yaw = np.deg2rad(rng.uniform(-15, 15, size=C))
    R = _look_at(c, c + _yaw_dirs(yaw))

    def draw(n):
        return np.stack([rng.uniform(-25, 25, n), rng.uniform(-5, 5, n),
                         rng.uniform(0, 50, n)], axis=1)

    pts, sel = _resample_until_seen(rng, draw, R, c, views, 2, 2.0, 2.0, None, n_points)
    bad_cams = np.array([17, 42, 77], dtype=np.int64)
    bad_cams = bad_cams[bad_cams < C]
    opts = dict(noise_px=1.0, outlier_frac=0.10, prior_frac=1.0, rot_deg=0.1, trans_m=0.02,
                point_m=0.02, use_depth=True, lambda_d=1.0, huber_px=2.0, filter_px=4.0,
                big_rot=(bad_cams, 3.0), all_outlier_points=min(200, n_points // 10),
                notes=dict(perturbed_cameras=bad_cams.astype(np.int32)))
    opts.update(kw)
    return _assemble(rng, "medium", seed, R, c, pts, sel, **opts)


def _walk_scene(name, seed, n_seq, n_points, half_extent, height, views, outlier_frac,
                prior_frac, n_cand, **kw):
    rng = np.random.default_rng(seed)
    c, yaw = _random_walks(rng, n_seq, 100, half_extent)
    R = _look_at(c, c + _yaw_dirs(yaw))

    def draw(n):
        return np.stack([rng.uniform(-half_extent, half_extent, n),
                         rng.uniform(-height / 2, height / 2, n),
                         rng.uniform(-half_extent, half_extent, n)], axis=1)

    pts, sel = _resample_until_seen(rng, draw, R, c, views, 2, 2.0, 2.0, n_cand, n_points)
    opts = dict(noise_px=1.0, outlier_frac=outlier_frac, prior_frac=prior_frac, rot_deg=0.1,
                trans_m=0.02, point_m=0.02, use_depth=True, lambda_d=1.0, huber_px=2.0,
                filter_px=4.0)
    opts.update(kw)
    return _assemble(rng, name, seed, R, c, pts, sel, **opts)


def make_scene(name: str, seed: int | None = None, **overrides) -> Scene:
    """Build one of the named scenes.

    ``tiny``    10 cameras on a 5 m circle, 500 points, 4 views each, no priors/robust loss.
    ``medium``  100 cameras on a forward track, 20k points, ~5 views, 10 % outliers,
                priors on every observation, Huber 2 px, 4 px filter, 3 cameras perturbed
                by 3 degrees and 200 points whose observations are all outliers.
    ``large``   1000 cameras in 10 random walks, 500k points, 8 views, 5 % outliers,
                priors on 50 % of observations.
    ``adjoint`` the ``medium`` scene with camera 0 held fixed (gauge anchor) and depth rows
                weighted lambda_d = 300 px m (about 1 / sigma of the priors' inverse depth)
                so that the undamped implicit-function system is well conditioned.
    ``xl``      5000 cameras in 50 random walks, 2M points, 6 views, 5 % outliers,
                priors on 30 % of observations.
    Keyword overrides resize a scene (``n_points``, ``n_cams``, ``n_seq`` ...) or change its
    noise/outlier settings; the default seed is the scene's index in ``SCENE_NAMES``.
    """
    if seed is None:
        seed = SCENE_NAMES.index(name)
    if name == "tiny":
        return _tiny(seed, **overrides)
    if name == "medium":
        return _medium(seed, **overrides)
    if name == "adjoint":
        kw = dict(lambda_d=300.0)
        kw.update(overrides)
        sc = _medium(seed, **kw)
        return replace(sc, name="adjoint", fixed=np.array([0], np.int32))
    if name == "large":
        kw = dict(n_seq=10, n_points=500_000, half_extent=100.0, height=20.0, views=8,
                  outlier_frac=0.05, prior_frac=0.5, n_cand=160)
        kw.update(overrides)
        return _walk_scene("large", seed, **kw)
    if name == "xl":
        kw = dict(n_seq=50, n_points=2_000_000, half_extent=200.0, height=20.0, views=6,
                  outlier_frac=0.05, prior_frac=0.3, n_cand=96)
        kw.update(overrides)
        return _walk_scene("xl", seed, **kw)
    raise ValueError(f"unknown scene {name!r}")


def subscene(sc: Scene, cams: np.ndarray, max_points: int | None = None,
             min_views: int = 2, seed: int = 0) -> Scene:
    """Restrict a scene to a camera subset and the points seen at least ``min_views`` times
    by it (optionally at most ``max_points`` of them, chosen at random); re-indexes both."""
    cams = np.asarray(cams, np.int64)
    cam_map = np.full(sc.n_cams, -1, np.int64)
    cam_map[cams] = np.arange(cams.size)
    keep = cam_map[sc.cam_idx] >= 0
    views = np.bincount(sc.pt_idx[keep], minlength=sc.n_points)
    pts = np.nonzero(views >= min_views)[0]
    if max_points is not None and pts.size > max_points:
        rng = np.random.default_rng(seed)
        pts = np.sort(rng.choice(pts, size=max_points, replace=False))
    pt_map = np.full(sc.n_points, -1, np.int64)
    pt_map[pts] = np.arange(pts.size)
    keep &= pt_map[sc.pt_idx] >= 0
    fixed = cam_map[sc.fixed[np.isin(sc.fixed, cams)]] if sc.fixed.size else sc.fixed
    return replace(
        sc, name=sc.name + "-sub", cams_gt=sc.cams_gt[cams], points_gt=sc.points_gt[pts],
        intr=sc.intr[cams], cams0=sc.cams0[cams], points0=sc.points0[pts],
        cam_idx=cam_map[sc.cam_idx[keep]].astype(np.int32),
        pt_idx=pt_map[sc.pt_idx[keep]].astype(np.int32), xy=sc.xy[keep],
        depth=sc.depth[keep], depth_valid=sc.depth_valid[keep],
        is_outlier=sc.is_outlier[keep], fixed=np.asarray(fixed, np.int32), notes={})
