"""IMU preintegration and the IMU error term (Section IV-C, eq. (5)), float64.

The paper integrates the IMU "numerically between the previous and current
camera frames", following Leutenegger et al. and Forster et al.'s
preintegration.  Readings taken here:

* samples are held (zero-order hold): the sub-interval [tau_m, tau_m+1) of
  [t0, t1) uses the sample stamped at or before tau_m; within it body rate and
  specific force are constant, so the exact solution of the kinematics is
      dR <- dR Exp(phi),  dv <- dv + dR G1(phi) a dt,
      dp <- dp + dv dt + dR G2(phi) a dt^2,  phi = w dt,
  with G1 = sum_k [phi]^k/(k+1)!, G2 = sum_k [phi]^k/(k+2)!;
* the bias correction is first order (Forster et al.):
  dR~ = dR Exp(J_R^g dbg), dv~ = dv + J_v^g dbg + J_v^a dba, dp~ likewise;
  the bias Jacobians are taken here by central finite differences with
  Richardson extrapolation;
* measurement noise is white with density sigma, i.e. variance sigma^2/dt_m on
  the value held over a sub-interval of length dt_m; the preintegrated noise
  covariance over (dphi, d(dv), d(dp)) with dR <- dR Exp(dphi) is first-order
  propagation of that noise, its Jacobian taken by finite differences;
* the IMU error e = x1_hat(x0) [-] x1 (eq. (5)) is 15-d over
  [r, alpha, v, bg, ba]; the bias rows carry the random-walk variance
  sigma_rw^2 Dt, and W_IMU is the inverse of the resulting covariance;
* frames: R_IS = R_IW R_WC R_CS, p_IS = R_IW (r_WC + R_WC t_CS),
  g_I = (0, 0, -g) with I z-up (Section II, Table I).
"""
from __future__ import annotations

import numpy as np

from .lie import exp_so3, hat, log_so3, quat_to_rot, quat_boxplus, state_boxplus


def _coefficients(th):
    """(1-cos)/th^2, (th-sin)/th^3, (th^2/2+cos-1)/th^4; Taylor series below 0.05
    where the closed forms cancel."""
    if th < 0.05:
        t2 = th * th
        return (0.5 - t2 / 24.0 + t2 * t2 / 720.0, 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0,
                1.0 / 24.0 - t2 / 720.0 + t2 * t2 / 40320.0)
    return ((1 - np.cos(th)) / th**2, (th - np.sin(th)) / th**3, (th * th / 2 + np.cos(th) - 1) / th**4)


def gamma1(phi):
    """G1(phi) = sum_k [phi]^k / (k+1)!."""
    phi = np.asarray(phi, dtype=np.float64)
    c1, c2, _ = _coefficients(float(np.linalg.norm(phi)))
    K = hat(phi)
    return np.eye(3) + c1 * K + c2 * (K @ K)


def gamma2(phi):
    """G2(phi) = sum_k [phi]^k / (k+2)!."""
    phi = np.asarray(phi, dtype=np.float64)
    _, c2, c3 = _coefficients(float(np.linalg.norm(phi)))
    K = hat(phi)
    return 0.5 * np.eye(3) + c2 * K + c3 * (K @ K)


def sub_intervals(stamps, t0, t1):
    """[(sample index, dt)] covering [t0, t1) under the zero-order hold."""
    stamps = np.asarray(stamps, dtype=np.float64)
    if len(stamps) == 0 or stamps[0] > t0:
        raise ValueError("IMU samples must start at or before t0")
    cuts = [t0] + [float(s) for s in stamps if t0 < s < t1] + [t1]
    out = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        k = int(np.searchsorted(stamps, a, side="right")) - 1
        out.append((k, b - a))
    return out


def integrate(stamps, gyro, acc, t0, t1, bg, ba, noise=None):
    """Exact zero-order-hold integration of (dR, dv, dp) at biases (bg, ba).

    ``noise`` optionally adds per-sub-interval offsets (m, 6) to (gyro, acc).
    """
    dR, dv, dp = np.eye(3), np.zeros(3), np.zeros(3)
    for m, (k, dt) in enumerate(sub_intervals(stamps, t0, t1)):
        w = np.asarray(gyro[k], dtype=np.float64) - bg
        a = np.asarray(acc[k], dtype=np.float64) - ba
        if noise is not None:
            w = w + noise[m, 0:3]
            a = a + noise[m, 3:6]
        phi = w * dt
        dp = dp + dv * dt + dR @ gamma2(phi) @ a * dt * dt
        dv = dv + dR @ gamma1(phi) @ a * dt
        dR = dR @ exp_so3(phi)
    return dR, dv, dp


def _tangent(ref, other):
    """(dphi, d(dv), d(dp)) of ``other`` relative to ``ref`` with dR = dR_ref Exp(dphi)."""
    return np.concatenate([log_so3(ref[0].T @ other[0]), other[1] - ref[1], other[2] - ref[2]])


def _richardson(f, n_in, h):
    """Central-difference Jacobian of f: R^n_in -> R^m with one Richardson step."""
    def central(hh):
        cols = []
        for i in range(n_in):
            d = np.zeros(n_in)
            d[i] = hh
            cols.append((f(d) - f(-d)) / (2 * hh))
        return np.stack(cols, axis=1)
    return (4.0 * central(h / 2) - central(h)) / 3.0


def preintegrate(stamps, gyro, acc, t0, t1, bg, ba, sigma_g, sigma_a):
    """Preintegrated measurement between frames (Section IV-C).

    Returns a dict: dR, dv, dp, dt, bg, ba (linearisation biases), J (9x6 bias
    Jacobian of (dphi, dv, dp) w.r.t. (bg, ba)) and Sigma (9x9 noise covariance).
    """
    bg = np.asarray(bg, dtype=np.float64)
    ba = np.asarray(ba, dtype=np.float64)
    ref = integrate(stamps, gyro, acc, t0, t1, bg, ba)
    J = _richardson(lambda d: _tangent(ref, integrate(stamps, gyro, acc, t0, t1, bg + d[:3], ba + d[3:])), 6, 1e-3)
    subs = sub_intervals(stamps, t0, t1)
    M = len(subs)

    def f_noise(n):
        return _tangent(ref, integrate(stamps, gyro, acc, t0, t1, bg, ba, noise=n.reshape(M, 6)))

    G = _richardson(f_noise, 6 * M, 1e-3)
    var = np.concatenate([np.concatenate([np.full(3, sigma_g**2 / dt), np.full(3, sigma_a**2 / dt)])
                          for _, dt in subs])
    Sigma = G @ np.diag(var) @ G.T
    return {"dR": ref[0], "dv": ref[1], "dp": ref[2], "dt": float(t1 - t0), "bg": bg.copy(), "ba": ba.copy(),
            "J": J, "Sigma": Sigma}


def predict(x0, q_IW, pre, params, dnoise=np.zeros(9)):
    """IMU prediction x1_hat(x0) of the camera state at t1 (Section IV-C).

    ``dnoise`` perturbs the preintegrated measurement: dR Exp(dphi), dv + ., dp + .
    Returns (r, R, v, bg, ba) of the predicted state.
    """
    R_CS, t_CS = params["R_CS"], params["t_CS"]
    g_I = np.array([0.0, 0.0, -params["gravity"]])
    R_IW = quat_to_rot(q_IW)
    R0 = quat_to_rot(x0["q"])
    dbg = x0["bg"] - pre["bg"]
    dba = x0["ba"] - pre["ba"]
    J = pre["J"]
    db = np.concatenate([dbg, dba])
    dR = pre["dR"] @ exp_so3(dnoise[0:3]) @ exp_so3(J[0:3] @ db)
    dv = pre["dv"] + dnoise[3:6] + J[3:6] @ db
    dp = pre["dp"] + dnoise[6:9] + J[6:9] @ db
    T = pre["dt"]
    R_IS0 = R_IW @ R0 @ R_CS
    p_IS0 = R_IW @ (x0["r"] + R0 @ t_CS)
    R_IS1 = R_IS0 @ dR
    v1 = x0["v"] + g_I * T + R_IS0 @ dv
    p_IS1 = p_IS0 + x0["v"] * T + 0.5 * g_I * T * T + R_IS0 @ dp
    R1 = R_IW.T @ R_IS1 @ R_CS.T
    r1 = R_IW.T @ p_IS1 - R1 @ t_CS
    return r1, R1, v1, x0["bg"].copy(), x0["ba"].copy()


def residual(x0, x1, q_IW, pre, params, dnoise=np.zeros(9)):
    """e_IMU = x1_hat(x0) [-] x1, eq. (5), ordered [r, alpha, v, bg, ba]."""
    r, R, v, bg, ba = predict(x0, q_IW, pre, params, dnoise)
    return np.concatenate([r - x1["r"], log_so3(R @ quat_to_rot(x1["q"]).T), v - x1["v"], bg - x1["bg"],
                           ba - x1["ba"]])


def factor(x0, x1, q_IW, pre, params):
    """Residual (15), Jacobian (15x33 over [x0 (15), x1 (15), dg (3)]) and weight W_IMU (15x15).

    Jacobians and the noise map are central finite differences on the manifold.
    """
    e = residual(x0, x1, q_IW, pre, params)

    def f(d):
        return residual(state_boxplus(x0, d[0:15]), state_boxplus(x1, d[15:30]), quat_boxplus(q_IW, d[30:33]),
                        pre, params)

    J = _richardson(f, 33, 1e-4)
    Sigma = residual_covariance(x0, x1, q_IW, pre, params)
    W = np.linalg.inv(Sigma)
    W = 0.5 * (W + W.T)
    return e, J, W


def residual_covariance(x0, x1, q_IW, pre, params):
    """Covariance (15x15) of e_IMU: the preintegration noise mapped through the
    residual (finite differences) plus the bias random walks."""
    A = _richardson(lambda d: residual(x0, x1, q_IW, pre, params, dnoise=d), 9, 1e-4)
    Sigma = A @ pre["Sigma"] @ A.T
    T = pre["dt"]
    Sigma[9:12, 9:12] += np.eye(3) * params["sigma_bg_rw"] ** 2 * T
    Sigma[12:15, 12:15] += np.eye(3) * params["sigma_ba_rw"] ** 2 * T
    return Sigma


# Gyro-only variant (the paper's comparison in which the accelerometer-related
# residuals are ignored, Section VI): the IMU rows kept are the rotation
# residual and the gyroscope-bias random walk.
GYRO_ROWS = np.r_[3:6, 9:12]
# z entries that only the dropped rows constrain: x0 and x1 velocity and
# accelerometer bias, and the gravity direction (it cancels from the rotation
# residual); the gyro-only system holds them fixed.
GYRO_FIXED = np.r_[6:9, 12:15, 21:24, 27:30, 30:33]


def factor_gyro(x0, x1, q_IW, pre, params):
    """The gyro-only IMU factor: the kept rows of the full factor, weighted by
    the inverse of their marginal covariance (the rows dropped are not
    measured, so they carry no information about the kept ones)."""
    e = residual(x0, x1, q_IW, pre, params)

    def f(d):
        return residual(state_boxplus(x0, d[0:15]), state_boxplus(x1, d[15:30]), quat_boxplus(q_IW, d[30:33]),
                        pre, params)

    J = _richardson(f, 33, 1e-4)
    Sigma = residual_covariance(x0, x1, q_IW, pre, params)
    Sk = Sigma[np.ix_(GYRO_ROWS, GYRO_ROWS)]
    Wk = np.linalg.inv(0.5 * (Sk + Sk.T))
    return e[GYRO_ROWS], J[GYRO_ROWS], 0.5 * (Wk + Wk.T)


def predict_state_gyro(x0, pre, params):
    """x1 initialised from x0 with the orientation rotated by the gyro-integrated
    rotation (no accelerometer: position, velocity and biases stay at x0's):
    R1 = R0 R_CS dR R_CS^T."""
    from .lie import copy_state
    R_CS = params["R_CS"]
    dbg = x0["bg"] - pre["bg"]
    dR = pre["dR"] @ exp_so3(pre["J"][0:3, 0:3] @ dbg)
    R0 = quat_to_rot(x0["q"])
    R1 = R0 @ R_CS @ dR @ R_CS.T
    x1 = copy_state(x0)
    x1["q"] = quat_boxplus(x0["q"], log_so3(R1 @ R0.T))
    return x1


def predict_state(x0, q_IW, pre, params):
    """x1 initialised at the IMU prediction (as a state dict)."""
    from .lie import copy_state
    r, R, v, bg, ba = predict(x0, q_IW, pre, params)
    x1 = copy_state(x0)
    x1["r"], x1["v"], x1["bg"], x1["ba"] = r, v, bg, ba
    # orientation from R via the box-plus of the rotation difference
    x1["q"] = quat_boxplus(x0["q"], log_so3(R @ quat_to_rot(x0["q"]).T))
    return x1
