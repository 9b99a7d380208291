"""Pins of the oracle's rotation / SE(3) helpers against library routines and identities."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.spatial.transform import Rotation

from oracle.geometry import (hat, quat_to_rot, quat_mul, so3_exp, so3_left_jacobian,
                             se3_exp_matrix, retract_cameras, quat_from_rotvec)

rng = np.random.default_rng(1234)


def _rand_quats(n):
    q = rng.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def test_quat_to_rot_matches_scipy():
    q = _rand_quats(50)
    R = quat_to_rot(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-14)


def test_quat_mul_composes_rotations():
    a, b = _rand_quats(20), _rand_quats(20)
    np.testing.assert_allclose(quat_to_rot(quat_mul(a, b)), quat_to_rot(a) @ quat_to_rot(b),
                               atol=1e-14)


@pytest.mark.parametrize("scale", [1e-9, 1e-4, 5e-3, 0.02, 0.5, 2.5])
def test_so3_exp_matches_expm(scale):
    phi = rng.normal(size=(10, 3))
    phi *= scale / np.linalg.norm(phi, axis=1, keepdims=True)
    R = so3_exp(phi)
    for i in range(phi.shape[0]):
        np.testing.assert_allclose(R[i], sla.expm(hat(phi[i])), atol=2e-15)
    # quaternion of the same rotation vector
    np.testing.assert_allclose(quat_to_rot(quat_from_rotvec(phi)), R, atol=2e-15)


@pytest.mark.parametrize("scale", [1e-8, 3e-3, 0.3, 2.0])
def test_se3_exp_matches_twist_expm(scale):
    xi = rng.normal(size=(8, 6)) * scale
    T = se3_exp_matrix(xi)
    for i in range(xi.shape[0]):
        tw = np.zeros((4, 4))
        tw[:3, :3] = hat(xi[i, 3:])
        tw[:3, 3] = xi[i, :3]
        np.testing.assert_allclose(T[i], sla.expm(tw), atol=1e-14)


def test_left_jacobian_series_vs_direct_continuity():
    # just below and above the Taylor switch the two branches agree to rounding
    d = np.array([[1.0, 0.0, 0.0]])
    lo = so3_left_jacobian(d * (1e-2 - 1e-12))
    hi = so3_left_jacobian(d * (1e-2 + 1e-12))
    np.testing.assert_allclose(lo, hi, atol=1e-13)


def test_retraction_is_left_se3_exponential():
    """Camera-frame coordinates after the update equal Exp(xi) applied to the old ones."""
    q = _rand_quats(12)
    c = rng.normal(size=(12, 3)) * 3
    X = rng.normal(size=(12, 3)) * 5
    xi = rng.normal(size=(12, 6)) * 0.3
    qn, cn = retract_cameras(q, c, xi)
    Xc_old = np.einsum("nij,nj->ni", quat_to_rot(q), X - c)
    Xc_new = np.einsum("nij,nj->ni", quat_to_rot(qn), X - cn)
    T = se3_exp_matrix(xi)
    ref = np.einsum("nij,nj->ni", T[:, :3, :3], Xc_old) + T[:, :3, 3]
    np.testing.assert_allclose(Xc_new, ref, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(qn, axis=1), 1.0, atol=1e-15)
