"""Rotations, quaternions and the state manifold (Section IV-A, eqs. (1)-(2)).

Quaternions are Hamilton unit quaternions stored (w, x, y, z) (Section II).
Perturbations are on the left, as the paper defines the box-plus for
orientations: ``q [+] da = exp(da) (x) q`` and ``p [-] q = log(p (x) q^-1)``;
vector parts add.  The per-frame state tangent is
``[dr, dalpha, dv, dbg, dba]`` (15); the gravity orientation q_IW has its own
3-vector dg.
"""
from __future__ import annotations

import numpy as np


def hat(w) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def vee(W) -> np.ndarray:
    return np.array([W[2, 1], W[0, 2], W[1, 0]])


def exp_so3(phi) -> np.ndarray:
    """Rodrigues' formula."""
    phi = np.asarray(phi, dtype=np.float64)
    th = float(np.linalg.norm(phi))
    K = hat(phi)
    if th < 1e-7:
        return np.eye(3) + K + 0.5 * (K @ K)
    return np.eye(3) + (np.sin(th) / th) * K + ((1.0 - np.cos(th)) / th**2) * (K @ K)


def log_so3(R) -> np.ndarray:
    """Inverse of exp_so3 for rotation angles in [0, pi)."""
    R = np.asarray(R, dtype=np.float64)
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = float(np.arccos(c))
    w = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-6:
        return 0.5 * w * (1.0 + th * th / 6.0)
    if np.pi - th < 1e-6:
        # near pi: axis from the symmetric part
        A = (R + np.eye(3)) / 2.0
        k = int(np.argmax(np.diag(A)))
        a = A[:, k] / np.sqrt(A[k, k])
        return th * a / np.linalg.norm(a)
    return (th / (2.0 * np.sin(th))) * w


def quat_mul(p, q) -> np.ndarray:
    """Hamilton product p (x) q."""
    pw, px, py, pz = p
    qw, qx, qy, qz = q
    return np.array([pw * qw - px * qx - py * qy - pz * qz,
                     pw * qx + px * qw + py * qz - pz * qy,
                     pw * qy - px * qz + py * qw + pz * qx,
                     pw * qz + px * qy - py * qx + pz * qw])


def quat_to_rot(q) -> np.ndarray:
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def quat_exp(phi) -> np.ndarray:
    phi = np.asarray(phi, dtype=np.float64)
    th = float(np.linalg.norm(phi))
    if th < 1e-12:
        return np.array([1.0, 0.5 * phi[0], 0.5 * phi[1], 0.5 * phi[2]]) / np.sqrt(1.0 + 0.25 * th * th)
    s = np.sin(0.5 * th) / th
    return np.array([np.cos(0.5 * th), s * phi[0], s * phi[1], s * phi[2]])


def quat_boxplus(q, dalpha) -> np.ndarray:
    """q [+] da = exp(da) (x) q  (Section IV-A), renormalised."""
    r = quat_mul(quat_exp(dalpha), q)
    r = r / np.linalg.norm(r)
    return r if r[0] >= 0 else -r


def quat_boxminus(p, q) -> np.ndarray:
    """p [-] q = log(p (x) q^-1), as a rotation vector (Section IV-A)."""
    return log_so3(quat_to_rot(p) @ quat_to_rot(q).T)


STATE_KEYS = ("r", "q", "v", "bg", "ba")


def copy_state(x: dict) -> dict:
    return {k: np.array(x[k], dtype=np.float64).copy() for k in STATE_KEYS}


def state_boxplus(x: dict, d) -> dict:
    """x [+] dx for the 15-d per-frame tangent [dr, dalpha, dv, dbg, dba]."""
    d = np.asarray(d, dtype=np.float64)
    return {"r": x["r"] + d[0:3], "q": quat_boxplus(x["q"], d[3:6]), "v": x["v"] + d[6:9],
            "bg": x["bg"] + d[9:12], "ba": x["ba"] + d[12:15]}


def state_boxminus(x: dict, y: dict) -> np.ndarray:
    """x [-] y (15)."""
    return np.concatenate([x["r"] - y["r"], quat_boxminus(x["q"], y["q"]), x["v"] - y["v"],
                           x["bg"] - y["bg"], x["ba"] - y["ba"]])


def pose_matrix(x: dict) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = quat_to_rot(x["q"])
    T[:3, 3] = x["r"]
    return T
