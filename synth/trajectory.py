"""Smooth camera trajectories with analytic rates, for image and IMU synthesis.

Frames (paper notation, Section II): I is gravity aligned (z up) and shares its
origin with W, the first camera frame.  A trajectory gives the camera pose in I,
``R_IC(t), p_IC(t)`` with ``p_IC(0) = 0``, its body rate ``omega_C(t)`` (rad/s,
expressed in C) and its linear velocity/acceleration in I.

The paper fits splines through ground-truth poses to obtain continuous motion
(Section VI-A); here a seeded uniform cubic B-spline over position and over a
rotation vector plays that role.
"""
from __future__ import annotations

import numpy as np


# --- generator-local rotation helpers (plain Rodrigues formulas) -------------

def _skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def rotvec_to_matrix(phi) -> np.ndarray:
    phi = np.asarray(phi, dtype=np.float64)
    th = float(np.linalg.norm(phi))
    K = _skew(phi)
    if th < 1e-8:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + (np.sin(th) / th) * K + ((1.0 - np.cos(th)) / th**2) * K @ K


def right_jacobian(phi) -> np.ndarray:
    """d/dt Exp(phi(t)) = Exp(phi) [Jr(phi) phi_dot]x."""
    phi = np.asarray(phi, dtype=np.float64)
    th = float(np.linalg.norm(phi))
    K = _skew(phi)
    if th < 1e-6:
        return np.eye(3) - 0.5 * K + (1.0 / 6.0) * K @ K
    return (np.eye(3) - ((1.0 - np.cos(th)) / th**2) * K
            + ((th - np.sin(th)) / th**3) * K @ K)


# --- uniform cubic B-spline ---------------------------------------------------

def _bspline_basis(u):
    """Uniform cubic B-spline basis and its first two derivatives in u."""
    b = np.array([(1 - u) ** 3, 3 * u**3 - 6 * u**2 + 4, -3 * u**3 + 3 * u**2 + 3 * u + 1, u**3]) / 6.0
    db = np.array([-(1 - u) ** 2, 3 * u**2 - 4 * u, -3 * u**2 + 2 * u + 1, u**2]) / 2.0
    ddb = np.array([1 - u, 3 * u - 2, -3 * u + 1, u])
    return b, db, ddb


class _Spline:
    def __init__(self, ctrl: np.ndarray, dt_knot: float):
        self.c = np.asarray(ctrl, dtype=np.float64)  # (n_ctrl, 3)
        self.dk = float(dt_knot)

    def eval(self, t: float):
        s = t / self.dk
        i = int(np.floor(s))
        i = min(max(i, 0), self.c.shape[0] - 4)
        u = s - i
        b, db, ddb = _bspline_basis(u)
        seg = self.c[i:i + 4]
        return b @ seg, (db @ seg) / self.dk, (ddb @ seg) / self.dk**2


class BSplineTrajectory:
    """Camera motion ``R_IC(t) = R_base Exp(phi(t))``, ``p_IC(t) = p(t) - p(0)``."""

    def __init__(self, R_base: np.ndarray, pos_ctrl: np.ndarray, rot_ctrl: np.ndarray, dt_knot: float,
                 duration: float):
        self.R_base = np.asarray(R_base, dtype=np.float64)
        self.pos = _Spline(pos_ctrl, dt_knot)
        self.rot = _Spline(rot_ctrl, dt_knot)
        self.duration = float(duration)
        self.p0 = self.pos.eval(0.0)[0]

    def pose(self, t):
        phi = self.rot.eval(t)[0]
        return self.R_base @ rotvec_to_matrix(phi), self.pos.eval(t)[0] - self.p0

    def omega_C(self, t):
        phi, dphi, _ = self.rot.eval(t)
        return right_jacobian(phi) @ dphi

    def vel_I(self, t):
        return self.pos.eval(t)[1]

    def acc_I(self, t):
        return self.pos.eval(t)[2]


class ConstantTwistTrajectory:
    """Rotation ``Exp(s theta a)`` and translation ``s d`` in W over ``s = t/T``.

    Used for the single frame pair: the pose at ``t = T`` is exactly the
    requested SE(3) offset from the first camera frame.
    """

    def __init__(self, R_IW: np.ndarray, rotvec_W: np.ndarray, trans_W: np.ndarray, T: float):
        self.R_IW = np.asarray(R_IW, dtype=np.float64)
        self.phi = np.asarray(rotvec_W, dtype=np.float64)
        self.d = np.asarray(trans_W, dtype=np.float64)
        self.T = float(T)
        self.duration = float(T)

    def pose(self, t):
        s = t / self.T
        return self.R_IW @ rotvec_to_matrix(s * self.phi), self.R_IW @ (s * self.d)

    def omega_C(self, t):
        # the rotation axis is fixed, so body and world rates coincide
        return self.phi / self.T

    def vel_I(self, t):
        return self.R_IW @ (self.d / self.T)

    def acc_I(self, t):
        return np.zeros(3)


def base_orientation(rng: np.random.Generator, tilt_sigma: float = 0.12) -> np.ndarray:
    """Camera looking along +y_I (x right, y down, z forward), randomly tilted."""
    R0 = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, -1.0, 0.0]])  # columns: x_C, y_C, z_C in I
    tilt = rng.normal(0.0, tilt_sigma, size=3)
    return rotvec_to_matrix(tilt) @ R0


def make_spline_trajectory(rng: np.random.Generator, duration: float, dt_knot: float = 0.25,
                           peak_speed: float = 1.5, peak_rate: float = np.pi) -> BSplineTrajectory:
    """Seeded smooth trajectory scaled to the requested peak speed and body rate."""
    n_ctrl = int(np.ceil(duration / dt_knot)) + 4
    pos = rng.uniform(-1.0, 1.0, size=(n_ctrl, 3))
    rot = rng.uniform(-1.0, 1.0, size=(n_ctrl, 3)) * np.array([0.6, 1.0, 0.3])
    R_base = base_orientation(rng)
    ts = np.linspace(0.0, duration, int(duration * 400) + 1)
    # position: speed is linear in the control offsets
    tr = BSplineTrajectory(R_base, pos, rot, dt_knot, duration)
    vmax = max(np.linalg.norm(tr.vel_I(t)) for t in ts)
    pos = pos * (peak_speed / vmax)
    # rotation: body rate is close to linear in the amplitude; refine a few times
    for _ in range(4):
        tr = BSplineTrajectory(R_base, pos, rot, dt_knot, duration)
        wmax = max(np.linalg.norm(tr.omega_C(t)) for t in ts)
        rot = rot * (peak_rate / wmax)
    return BSplineTrajectory(R_base, pos, rot, dt_knot, duration)
