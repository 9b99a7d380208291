"""Rotation and rigid-motion helpers of the oracle (FP64, NumPy).

Test infrastructure only (see the package docstring). The camera layout follows the
paper's BA objective (Sec. III-B): extrinsics are a centre and a unit quaternion
``[qw, qx, qy, qz, cx, cy, cz]``; here the quaternion is the world-to-camera rotation, so a
world point ``X`` has camera coordinates ``R (X - c)``.

The LM update of a camera is a left SE(3) perturbation ``T <- Exp(xi) T`` with
``xi = (rho, phi)`` (translation part first). Rodrigues-type coefficients switch to their
Taylor series for ``|phi| < 1e-2`` where direct evaluation loses digits.
"""
from __future__ import annotations

import numpy as np

SMALL_ANGLE = 1e-2


def hat(v: np.ndarray) -> np.ndarray:
    """Skew matrices [v]x of shape (..., 3, 3)."""
    v = np.asarray(v, dtype=np.float64)
    z = np.zeros(v.shape[:-1])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], axis=-1),
        np.stack([v[..., 2], z, -v[..., 0]], axis=-1),
        np.stack([-v[..., 1], v[..., 0], z], axis=-1),
    ], axis=-2)


def quat_normalize(q: np.ndarray) -> np.ndarray:
    return q / np.linalg.norm(q, axis=-1, keepdims=True)


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices of (normalised) quaternions ``[w, x, y, z]``."""
    q = quat_normalize(np.asarray(q, dtype=np.float64))
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], axis=-2)


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product a (x) b for ``[w, x, y, z]`` quaternions."""
    aw, av = a[..., :1], a[..., 1:]
    bw, bv = b[..., :1], b[..., 1:]
    w = aw * bw - np.sum(av * bv, axis=-1, keepdims=True)
    v = aw * bv + bw * av + np.cross(av, bv)
    return np.concatenate([w, v], axis=-1)


def _angle_coeffs(phi: np.ndarray):
    """sin(t)/t, (1-cos t)/t^2, (t - sin t)/t^3 and sin(t/2)/t, cos(t/2) for t = |phi|."""
    t2 = np.sum(phi * phi, axis=-1)
    t = np.sqrt(t2)
    small = t < SMALL_ANGLE
    ts = np.where(small, 1.0, t)
    a = np.where(small, 1 - t2 / 6 + t2 * t2 / 120, np.sin(ts) / ts)
    b = np.where(small, 0.5 - t2 / 24 + t2 * t2 / 720, (1 - np.cos(ts)) / ts ** 2)
    c = np.where(small, 1.0 / 6 - t2 / 120 + t2 * t2 / 5040, (ts - np.sin(ts)) / ts ** 3)
    h = np.where(small, 0.5 - t2 / 48 + t2 * t2 / 3840, np.sin(ts / 2) / ts)
    return a, b, c, h, np.cos(t / 2)


def so3_exp(phi: np.ndarray) -> np.ndarray:
    """Rodrigues' formula R = I + a [phi]x + b [phi]x^2."""
    phi = np.asarray(phi, dtype=np.float64)
    a, b, _, _, _ = _angle_coeffs(phi)
    K = hat(phi)
    return np.eye(3) + a[..., None, None] * K + b[..., None, None] * (K @ K)


def so3_left_jacobian(phi: np.ndarray) -> np.ndarray:
    """V(phi) = I + b [phi]x + c [phi]x^2, the translation factor of the SE(3) exponential."""
    phi = np.asarray(phi, dtype=np.float64)
    _, b, c, _, _ = _angle_coeffs(phi)
    K = hat(phi)
    return np.eye(3) + b[..., None, None] * K + c[..., None, None] * (K @ K)


def quat_from_rotvec(phi: np.ndarray) -> np.ndarray:
    phi = np.asarray(phi, dtype=np.float64)
    _, _, _, h, cw = _angle_coeffs(phi)
    return np.concatenate([cw[..., None], h[..., None] * phi], axis=-1)


def se3_exp_matrix(xi: np.ndarray) -> np.ndarray:
    """4x4 homogeneous Exp(xi) for xi = (rho, phi)."""
    xi = np.asarray(xi, dtype=np.float64)
    T = np.zeros(xi.shape[:-1] + (4, 4))
    T[..., :3, :3] = so3_exp(xi[..., 3:])
    T[..., :3, 3] = np.einsum("...ij,...j->...i", so3_left_jacobian(xi[..., 3:]), xi[..., :3])
    T[..., 3, 3] = 1.0
    return T


def retract_cameras(q: np.ndarray, c: np.ndarray, xi: np.ndarray):
    """Left SE(3) update of world-to-camera poses given as (quaternion, centre).

    With T = [R | -R c], Exp(xi) T has rotation Exp(phi) R and translation
    Exp(phi)(-R c) + V(phi) rho, hence centre c' = c - R'^T V(phi) rho.
    """
    rho, phi = xi[..., :3], xi[..., 3:]
    qn = quat_normalize(quat_mul(quat_from_rotvec(phi), quat_normalize(q)))
    Rn = quat_to_rot(qn)
    Vr = np.einsum("...ij,...j->...i", so3_left_jacobian(phi), rho)
    cn = c - np.einsum("...ji,...j->...i", Rn, Vr)
    return qn, cn
