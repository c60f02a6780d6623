"""IMU sample synthesis along a trajectory (gyro and accelerometer in frame S).

Model, after the continuous-time noise model the paper cites for its synthetic
IMU data (Section VI-A, Table I):

* gyro  ``w~ = w_S + b_g + n_g``,  accel ``a~ = R_IS^T (a_IS - g_I) + b_a + n_a``;
* white noise of density sigma, i.e. per-sample variance ``sigma^2 / dt``;
* bias random walks of density sigma_rw, i.e. increment variance ``sigma_rw^2 dt``;
* clipping at the sensor saturation (Table I: 7.8 rad/s, 176 m/s^2).

Each sample is stamped at the start of its hold interval ``[t_k, t_k + dt)``
and carries the rates at the interval's midpoint, which keeps the zero-order
hold used by the estimator second-order accurate.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .trajectory import _skew

GRAVITY = 9.81


@dataclass
class ImuNoise:
    sigma_g: float = 1.7e-4      # rad/s/sqrt(Hz)
    sigma_a: float = 2.0e-3      # m/s^2/sqrt(Hz)
    sigma_bg_rw: float = 4.0e-6  # rad/s^2/sqrt(Hz)  (Table I, gyro drift density)
    sigma_ba_rw: float = 2.0e-5  # m/s^3/sqrt(Hz)    (Table I, accel drift density)
    gyro_sat: float = 7.8
    acc_sat: float = 176.0


def _omega_dot(traj, t, h=1e-5):
    return (traj.omega_C(t + h) - traj.omega_C(t - h)) / (2 * h)


def imu_truth(traj, t, R_CS=np.eye(3), t_CS=np.zeros(3)):
    """Noise-free body rate and specific force of the IMU (frame S) at time t."""
    R_IC, _ = traj.pose(t)
    w_C = traj.omega_C(t)
    a_IC = traj.acc_I(t)
    if np.any(t_CS != 0.0):
        W = _skew(w_C)
        Rdd = R_IC @ (W @ W + _skew(_omega_dot(traj, t)))
        a_IS = a_IC + Rdd @ t_CS
    else:
        a_IS = a_IC
    R_IS = R_IC @ R_CS
    g_I = np.array([0.0, 0.0, -GRAVITY])
    return R_CS.T @ w_C, R_IS.T @ (a_IS - g_I)


def state_truth(traj, t, R_CS=np.eye(3), t_CS=np.zeros(3)):
    """Ground-truth camera pose in I and IMU velocity v_IS expressed in I."""
    R_IC, p_IC = traj.pose(t)
    v = traj.vel_I(t) + R_IC @ (_skew(traj.omega_C(t)) @ t_CS)
    return R_IC, p_IC, v


def synth_imu(traj, t_begin, t_end, rate_hz, rng, noise: ImuNoise, bg0, ba0, *, noisy=True,
              bias_walk=True, R_CS=np.eye(3), t_CS=np.zeros(3)):
    """Samples with stamps ``k / rate`` covering ``[t_begin, t_end)``.

    Returns (stamps (n,), gyro (n,3), acc (n,3), true_bg (n,3), true_ba (n,3)).
    """
    dt = 1.0 / rate_hz
    k0 = int(np.floor(t_begin * rate_hz + 1e-9))
    k1 = int(np.ceil(t_end * rate_hz - 1e-9))
    ks = np.arange(k0, k1)
    stamps = ks * dt
    bg = np.array(bg0, dtype=np.float64)
    ba = np.array(ba0, dtype=np.float64)
    G, A, BG, BA = [], [], [], []
    for t in stamps:
        w, f = imu_truth(traj, min(t + 0.5 * dt, traj.duration), R_CS, t_CS)
        if noisy:
            w = w + rng.normal(0.0, noise.sigma_g / np.sqrt(dt), 3)
            f = f + rng.normal(0.0, noise.sigma_a / np.sqrt(dt), 3)
        G.append(np.clip(w + bg, -noise.gyro_sat, noise.gyro_sat))
        A.append(np.clip(f + ba, -noise.acc_sat, noise.acc_sat))
        BG.append(bg.copy())
        BA.append(ba.copy())
        if bias_walk:
            bg = bg + rng.normal(0.0, noise.sigma_bg_rw * np.sqrt(dt), 3)
            ba = ba + rng.normal(0.0, noise.sigma_ba_rw * np.sqrt(dt), 3)
    return stamps, np.array(G).reshape(-1, 3), np.array(A).reshape(-1, 3), np.array(BG).reshape(-1, 3), \
        np.array(BA).reshape(-1, 3)
