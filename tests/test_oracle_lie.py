"""Pins of the oracle's rotation and state-manifold helpers (Section IV-A).

Checked against an independent library implementation (scipy's Rotation),
round trips and textbook identities.
"""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import lie


def _rng():
    return np.random.default_rng(7)


def test_exp_matches_scipy():
    rng = _rng()
    for _ in range(50):
        phi = rng.normal(size=3) * rng.uniform(1e-9, 3.0)
        assert np.allclose(lie.exp_so3(phi), Rotation.from_rotvec(phi).as_matrix(), atol=1e-13)


def test_quaternion_matches_scipy_hamilton():
    rng = _rng()
    for _ in range(50):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R_ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scipy is scalar-last
        assert np.allclose(lie.quat_to_rot(q), R_ref, atol=1e-13)
        phi = rng.normal(size=3)
        qe = lie.quat_exp(phi)
        assert np.allclose(lie.quat_to_rot(qe), Rotation.from_rotvec(phi).as_matrix(), atol=1e-13)


def test_hamilton_product_composes_rotations():
    rng = _rng()
    for _ in range(20):
        p = rng.normal(size=4)
        q = rng.normal(size=4)
        p /= np.linalg.norm(p)
        q /= np.linalg.norm(q)
        assert np.allclose(lie.quat_to_rot(lie.quat_mul(p, q)), lie.quat_to_rot(p) @ lie.quat_to_rot(q), atol=1e-13)


def test_log_inverts_exp():
    rng = _rng()
    for _ in range(50):
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        for th in (1e-9, 1e-5, 0.3, 2.0, 3.1):
            assert np.allclose(lie.log_so3(lie.exp_so3(th * a)), th * a, atol=1e-10 * max(1, th))


def test_rotation_is_orthonormal():
    rng = _rng()
    for _ in range(20):
        R = lie.quat_to_rot(rng.normal(size=4))
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14


def test_boxplus_boxminus_round_trip():
    rng = _rng()
    x = {"r": rng.normal(size=3), "q": lie.quat_exp(rng.normal(size=3)), "v": rng.normal(size=3),
         "bg": rng.normal(size=3), "ba": rng.normal(size=3)}
    for _ in range(20):
        d = rng.normal(size=15) * 0.3
        assert np.allclose(lie.state_boxminus(lie.state_boxplus(x, d), x), d, atol=1e-12)


def test_boxplus_is_left_perturbation():
    # q [+] da = exp(da) (x) q  (Section IV-A): R(q [+] da) = Exp(da) R(q)
    rng = _rng()
    q = lie.quat_exp(rng.normal(size=3))
    da = rng.normal(size=3) * 0.2
    assert np.allclose(lie.quat_to_rot(lie.quat_boxplus(q, da)), lie.exp_so3(da) @ lie.quat_to_rot(q), atol=1e-13)
