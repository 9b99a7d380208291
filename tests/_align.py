"""Gauge alignment for comparisons (test helper, not solver code).

Umeyama's closed-form least-squares similarity (IEEE TPAMI 1991): find s, R, t minimising
sum |dst - (s R src + t)|^2. BA is invariant to a similarity (no depth priors) or a rigid
motion (metric depth priors), so estimates are compared after this alignment.
"""
import numpy as np


def umeyama(src: np.ndarray, dst: np.ndarray, with_scale: bool = True):
    mu_s, mu_d = src.mean(0), dst.mean(0)
    a, b = src - mu_s, dst - mu_d
    cov = b.T @ a / src.shape[0]
    U, D, Vt = np.linalg.svd(cov)
    S = np.eye(3)
    if np.linalg.det(U) * np.linalg.det(Vt) < 0:
        S[2, 2] = -1
    R = U @ S @ Vt
    var = np.mean(np.sum(a * a, axis=1))
    s = float(np.trace(np.diag(D) @ S) / var) if with_scale else 1.0
    t = mu_d - s * R @ mu_s
    return s, R, t


def aligned_error(cams_est, pts_est, cams_ref, pts_ref, with_scale=True):
    """Relative gauge-aligned error |A(est) - ref|_F / |ref - mean(ref)|_F over stacked
    camera centres and points, plus the similarity used."""
    src = np.concatenate([cams_est[:, 4:7], pts_est])
    dst = np.concatenate([cams_ref[:, 4:7], pts_ref])
    s, R, t = umeyama(src, dst, with_scale)
    al = s * src @ R.T + t
    err = np.linalg.norm(al - dst) / np.linalg.norm(dst - dst.mean(0))
    return float(err), (s, R, t)


def rotation_error(cams_est, cams_ref, R_align):
    """Max angle (rad) between aligned estimated and reference world-to-camera rotations."""
    from scipy.spatial.transform import Rotation
    qe = cams_est[:, [1, 2, 3, 0]]
    qr = cams_ref[:, [1, 2, 3, 0]]
    Re = Rotation.from_quat(qe).as_matrix() @ R_align.T
    Rr = Rotation.from_quat(qr).as_matrix()
    d = Rotation.from_matrix(np.einsum("nji,njk->nik", Rr, Re))
    return float(np.max(np.linalg.norm(d.as_rotvec(), axis=1)))
