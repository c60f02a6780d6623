"""Pins of the oracle's IMU preintegration and IMU error term (Section IV-C, eq. (5))."""
import numpy as np
from scipy.integrate import solve_ivp

from oracle import imu, lie
import synth
from synth.configs import quat_from_matrix


def _ode_truth(w, a, T):
    """High-accuracy ODE solution of dR = R[w]x, dv = R a, dp = v from identity."""
    def f(t, y):
        R = y[:9].reshape(3, 3)
        return np.concatenate([(R @ lie.hat(w)).ravel(), R @ a, y[9:12]])
    y0 = np.concatenate([np.eye(3).ravel(), np.zeros(6)])
    s = solve_ivp(f, (0, T), y0, rtol=1e-12, atol=1e-14, method="DOP853")
    y = s.y[:, -1]
    return y[:9].reshape(3, 3), y[9:12], y[12:15]


def test_zero_order_hold_matches_ode_under_constant_rates():
    w = np.array([1.0, -2.0, 0.5])
    a = np.array([0.3, 9.8, -0.5])
    T = 0.05
    R, v, p = _ode_truth(w, a, T)
    for n in (1, 3, 7):
        stamps = np.arange(n) * (T / n)
        gyro = np.tile(w, (n, 1))
        acc = np.tile(a, (n, 1))
        dR, dv, dp = imu.integrate(stamps, gyro, acc, 0.0, T, np.zeros(3), np.zeros(3))
        assert np.abs(dR - R).max() < 1e-12
        assert np.abs(dv - v).max() < 1e-11
        assert np.abs(dp - p).max() < 1e-12


def test_matrix_series_definitions_of_gamma():
    rng = np.random.default_rng(1)
    for th in (1e-6, 1e-3, 0.4, 2.5):
        phi = rng.normal(size=3)
        phi *= th / np.linalg.norm(phi)
        K = lie.hat(phi)
        G1, G2, term = np.zeros((3, 3)), np.zeros((3, 3)), np.eye(3)
        fact1, fact2 = 1.0, 2.0
        for k in range(40):
            G1 += term / fact1
            G2 += term / fact2
            term = term @ K
            fact1 *= k + 2
            fact2 *= k + 3
        assert np.abs(imu.gamma1(phi) - G1).max() < 1e-12
        assert np.abs(imu.gamma2(phi) - G2).max() < 1e-12


def test_reduces_to_euler_without_rotation():
    # w = 0: dv = sum a dt, dp = sum (dv dt + a dt^2 / 2) exactly
    stamps = np.array([0.0, 0.004, 0.011])
    acc = np.array([[0.1, 9.7, 0.2], [0.4, 9.9, -0.1], [-0.2, 9.8, 0.0]])
    dR, dv, dp = imu.integrate(stamps, np.zeros((3, 3)), acc, 0.0, 0.02, np.zeros(3), np.zeros(3))
    dts = [0.004, 0.007, 0.009]
    v, p = np.zeros(3), np.zeros(3)
    for k, dt in enumerate(dts):
        p = p + v * dt + 0.5 * acc[k] * dt * dt
        v = v + acc[k] * dt
    assert np.allclose(dR, np.eye(3), atol=1e-15)
    assert np.abs(dv - v).max() < 1e-14 and np.abs(dp - p).max() < 1e-15


def test_zero_order_hold_windows():
    subs = imu.sub_intervals(np.array([0.0, 0.005, 0.010, 0.015]), 0.003, 0.012)
    assert [k for k, _ in subs] == [0, 1, 2]
    assert np.allclose([dt for _, dt in subs], [0.002, 0.005, 0.002])


def test_bias_jacobians_closed_forms():
    T = 0.03
    stamps = np.arange(6) * 0.005
    # no rotation: d dv / d ba = -T I, d dp / d ba = -T^2/2 I, d dphi / d bg = -T I
    pre = imu.preintegrate(stamps, np.zeros((6, 3)), np.tile([0.2, 9.8, 0.1], (6, 1)), 0.0, T, np.zeros(3),
                           np.zeros(3), 1e-3, 1e-2)
    J = pre["J"]
    assert np.abs(J[3:6, 3:6] + T * np.eye(3)).max() < 1e-10
    assert np.abs(J[6:9, 3:6] + 0.5 * T * T * np.eye(3)).max() < 1e-10
    assert np.abs(J[0:3, 0:3] + T * np.eye(3)).max() < 1e-10
    assert np.abs(J[0:3, 3:6]).max() < 1e-12
    # constant rate: d dphi / d bg = -Jr(w T) T (right Jacobian of SO(3))
    w = np.array([1.5, -0.7, 2.0])
    pre = imu.preintegrate(stamps, np.tile(w, (6, 1)), np.zeros((6, 3)), 0.0, T, np.zeros(3), np.zeros(3),
                           1e-3, 1e-2)
    phi = w * T
    th = np.linalg.norm(phi)
    K = lie.hat(phi)
    Jr = np.eye(3) - (1 - np.cos(th)) / th**2 * K + (th - np.sin(th)) / th**3 * (K @ K)
    assert np.abs(pre["J"][0:3, 0:3] + Jr * T).max() < 1e-10


def test_noise_covariance_against_monte_carlo():
    rng = np.random.default_rng(5)
    stamps = np.array([0.0, 0.005, 0.010, 0.015])
    gyro = rng.normal(size=(4, 3)) * 2
    acc = rng.normal(size=(4, 3)) + [0, 9.8, 0]
    t0, t1 = 0.002, 0.017
    sg, sa = 0.05, 0.5
    pre = imu.preintegrate(stamps, gyro, acc, t0, t1, np.zeros(3), np.zeros(3), sg, sa)
    subs = imu.sub_intervals(stamps, t0, t1)
    ref = imu.integrate(stamps, gyro, acc, t0, t1, np.zeros(3), np.zeros(3))
    N = 20000
    samples = np.empty((N, 9))
    sd = np.array([[sg / np.sqrt(dt)] * 3 + [sa / np.sqrt(dt)] * 3 for _, dt in subs])
    for n in range(N):
        out = imu.integrate(stamps, gyro, acc, t0, t1, np.zeros(3), np.zeros(3),
                            noise=rng.normal(size=(len(subs), 6)) * sd)
        samples[n] = np.concatenate([lie.log_so3(ref[0].T @ out[0]), out[1] - ref[1], out[2] - ref[2]])
    C = np.cov(samples.T)
    S = pre["Sigma"]
    d = np.sqrt(np.diag(S))
    corr_err = np.abs(C / np.outer(d, d) - S / np.outer(d, d)).max()
    assert corr_err < 0.05
    assert np.all(np.abs(np.diag(C) / np.diag(S) - 1) < 0.05)


def _params(R_CS, t_CS):
    return {"gravity": 9.81, "R_CS": R_CS, "t_CS": t_CS, "sigma_bg_rw": 4e-6, "sigma_ba_rw": 2e-5}


def _rigid_motion_case():
    """Body rate and body-frame specific force constant over [0, T]: the
    zero-order hold is exact and the ODE gives the ground truth."""
    rng = np.random.default_rng(11)
    R_CS = lie.exp_so3([0.1, -0.2, 0.05])
    t_CS = np.array([0.03, -0.01, 0.02])
    R_IW = lie.exp_so3([0.2, -0.1, 0.7])
    w_S = np.array([0.8, -1.1, 0.4])
    f_S = np.array([0.5, -0.3, 9.6])
    bg, ba = np.array([0.01, -0.02, 0.005]), np.array([0.05, 0.02, -0.04])
    T = 1.0 / 30.0
    # initial state of S in I
    R_WC0 = lie.exp_so3(rng.normal(size=3) * 0.3)
    r0 = rng.normal(size=3)
    R_IS0 = R_IW @ R_WC0 @ R_CS
    p_IS0 = R_IW @ (r0 + R_WC0 @ t_CS)
    v0 = rng.normal(size=3)
    g = np.array([0, 0, -9.81])
    dR, dv, dp = _ode_truth(w_S, f_S, T)
    R_IS1 = R_IS0 @ dR
    v1 = v0 + g * T + R_IS0 @ dv
    p_IS1 = p_IS0 + v0 * T + 0.5 * g * T * T + R_IS0 @ dp
    R_WC1 = R_IW.T @ R_IS1 @ R_CS.T
    r1 = R_IW.T @ p_IS1 - R_WC1 @ t_CS
    x0 = {"r": r0, "q": quat_from_matrix(R_WC0), "v": v0, "bg": bg, "ba": ba}
    x1 = {"r": r1, "q": quat_from_matrix(R_WC1), "v": v1, "bg": bg, "ba": ba}
    stamps = np.array([0.0, 0.005, 0.010, 0.015, 0.020, 0.025, 0.030])
    return {"x0": x0, "x1": x1, "q_IW": quat_from_matrix(R_IW), "stamps": stamps,
            "gyro": np.tile(w_S + bg, (7, 1)), "acc": np.tile(f_S + ba, (7, 1)), "T": T,
            "params": _params(R_CS, t_CS)}


def test_noise_free_prediction_reproduces_ground_truth():
    c = _rigid_motion_case()
    pre = imu.preintegrate(c["stamps"], c["gyro"], c["acc"], 0.0, c["T"], c["x0"]["bg"], c["x0"]["ba"], 1e-3, 1e-2)
    e = imu.residual(c["x0"], c["x1"], c["q_IW"], pre, c["params"])
    assert np.abs(e).max() < 1e-10


def test_first_order_bias_correction():
    c = _rigid_motion_case()
    bbar = (np.zeros(3), np.zeros(3))
    pre = imu.preintegrate(c["stamps"], c["gyro"], c["acc"], 0.0, c["T"], *bbar, 1e-3, 1e-2)
    exact = imu.preintegrate(c["stamps"], c["gyro"], c["acc"], 0.0, c["T"], c["x0"]["bg"], c["x0"]["ba"], 1e-3,
                             1e-2)
    e_lin = imu.residual(c["x0"], c["x1"], c["q_IW"], pre, c["params"])
    e_ex = imu.residual(c["x0"], c["x1"], c["q_IW"], exact, c["params"])
    # biases of order 5e-2 act over 1/30 s: second-order remainder well below 1e-5
    assert np.abs(e_ex).max() < 1e-10
    assert np.abs(e_lin - e_ex).max() < 1e-5


def test_factor_jacobian_known_blocks():
    c = _rigid_motion_case()
    pre = imu.preintegrate(c["stamps"], c["gyro"], c["acc"], 0.0, c["T"], c["x0"]["bg"], c["x0"]["ba"], 1e-3, 1e-2)
    e, J, W = imu.factor(c["x0"], c["x1"], c["q_IW"], pre, c["params"])
    I3 = np.eye(3)
    R_IW = lie.quat_to_rot(c["q_IW"])
    assert np.abs(J[0:3, 15:18] + I3).max() < 1e-8          # de_r / d dr1
    assert np.abs(J[0:3, 0:3] - I3).max() < 1e-8            # de_r / d dr0
    assert np.abs(J[6:9, 21:24] + I3).max() < 1e-8          # de_v / d dv1
    assert np.abs(J[6:9, 6:9] - I3).max() < 1e-8            # de_v / d dv0
    assert np.abs(J[0:3, 6:9] - R_IW.T * c["T"]).max() < 1e-8  # de_r / d dv0
    assert np.abs(J[9:15, 9:15] - np.eye(6)).max() < 1e-8   # bias rows
    assert np.abs(J[9:15, 24:30] + np.eye(6)).max() < 1e-8
    assert np.abs(J[3:6, 18:21] + I3).max() < 1e-6          # de_alpha / d da1 at e = 0
    assert np.allclose(W, W.T) and np.linalg.eigvalsh(W).min() > 0


def test_gyro_only_prediction_is_the_closed_form_rotation():
    """Constant body rate w, no noise, zero bias: the gyro-only prediction is
    R1 = R0 R_CS Exp(w T) R_CS^T, position and velocity unchanged."""
    from oracle import lie
    rng = np.random.default_rng(11)
    w = np.array([0.4, -0.9, 1.3])
    T = 0.05
    stamps = np.arange(0.0, T, 0.005)
    gyro = np.tile(w, (len(stamps), 1))
    acc = np.tile([0.3, 9.5, -1.0], (len(stamps), 1))
    x0 = {"r": rng.normal(size=3), "q": lie.quat_exp(rng.normal(size=3)), "v": rng.normal(size=3),
          "bg": np.zeros(3), "ba": np.zeros(3)}
    R_CS = lie.exp_so3(np.array([0.1, 0.2, -0.3]))
    params = {"R_CS": R_CS, "t_CS": np.zeros(3)}
    pre = imu.preintegrate(stamps, gyro, acc, 0.0, T, x0["bg"], x0["ba"], 1.7e-4, 2e-3)
    x1 = imu.predict_state_gyro(x0, pre, params)
    R0 = lie.quat_to_rot(x0["q"])
    want = R0 @ R_CS @ lie.exp_so3(w * T) @ R_CS.T
    assert np.abs(lie.quat_to_rot(x1["q"]) - want).max() < 1e-12
    assert np.array_equal(x1["r"], x0["r"]) and np.array_equal(x1["v"], x0["v"])


def test_gyro_only_factor_is_the_rotation_marginal_of_the_full_factor():
    from oracle import lie, track
    d = synth.configs.frame_pair(seed=1001)
    params = track.default_params(levels=2, iters=(1, 1), mode="gyro")
    pre = imu.preintegrate(d["imu"]["t"], d["imu"]["gyro"], d["imu"]["acc"], d["t0"], d["t1"], d["x0"]["bg"],
                           d["x0"]["ba"], params["sigma_g"], params["sigma_a"])
    x1 = lie.state_boxplus(d["gt1"], np.r_[1e-3 * np.ones(6), np.zeros(9)])
    e, J, W = imu.factor(d["x0"], x1, d["q_IW"], pre, params)
    eg, Jg, Wg = imu.factor_gyro(d["x0"], x1, d["q_IW"], pre, params)
    rows = np.r_[3:6, 9:12]
    assert np.array_equal(eg, e[rows])
    assert np.abs(Jg - J[rows]).max() < 1e-12
    # weights: inverse of the kept rows' block of the full covariance W^-1
    S = np.linalg.inv(W)[np.ix_(rows, rows)]
    assert np.abs(np.linalg.inv(Wg) - S).max() < 1e-9 * np.abs(S).max()


def _aligned_case(seed=23):
    """Constant body rate and specific force over T = 7 sample periods of 5 ms
    (frame times on sample stamps, so each held value spans one full period):
    the zero-order hold is exact and the ODE gives the ground truth."""
    rng = np.random.default_rng(seed)
    R_CS = lie.exp_so3([0.1, -0.2, 0.05])
    t_CS = np.array([0.03, -0.01, 0.02])
    R_IW = lie.exp_so3([0.05, -0.08, 0.9])
    w_S = np.array([1.2, -0.6, 0.9])
    f_S = np.array([0.7, -0.4, 9.5])
    bg, ba = np.array([2e-3, -1e-3, 5e-4]), np.array([3e-2, -2e-2, 1e-2])
    dt, n = 0.005, 7
    T = dt * n
    R_WC0 = lie.exp_so3(rng.normal(size=3) * 0.4)
    r0, v0 = rng.normal(size=3), rng.normal(size=3)
    R_IS0 = R_IW @ R_WC0 @ R_CS
    p_IS0 = R_IW @ (r0 + R_WC0 @ t_CS)
    g = np.array([0.0, 0.0, -9.81])
    dR, dv, dp = _ode_truth(w_S, f_S, T)
    R_WC1 = R_IW.T @ (R_IS0 @ dR) @ R_CS.T
    r1 = R_IW.T @ (p_IS0 + v0 * T + 0.5 * g * T * T + R_IS0 @ dp) - R_WC1 @ t_CS
    v1 = v0 + g * T + R_IS0 @ dv
    x0 = {"r": r0, "q": quat_from_matrix(R_WC0), "v": v0, "bg": bg, "ba": ba}
    x1 = {"r": r1, "q": quat_from_matrix(R_WC1), "v": v1, "bg": bg.copy(), "ba": ba.copy()}
    params = {"gravity": 9.81, "R_CS": R_CS, "t_CS": t_CS, "sigma_bg_rw": 4e-6, "sigma_ba_rw": 2e-5}
    return {"x0": x0, "x1": x1, "q_IW": quat_from_matrix(R_IW), "stamps": np.arange(n) * dt, "T": T,
            "gyro": np.tile(w_S + bg, (n, 1)), "acc": np.tile(f_S + ba, (n, 1)), "dt": dt, "params": params}


def _whitened_gap(S, C):
    """max |L^-1 C L^-T - I| with S = L L^T: how far the sample covariance C
    is from the model covariance S, in units of the model's own spread."""
    Li = np.linalg.inv(np.linalg.cholesky(S))
    return np.abs(Li @ C @ Li.T - np.eye(len(S))).max()


def test_residual_covariance_against_monte_carlo_with_bias_random_walk():
    """W_IMU^-1 (Section IV-C, eq. (5); noise and drift densities of Table I)
    against the sample covariance of the 15-d residual under the generative
    model it describes: every gyro / accelerometer sample carries white noise
    of variance sigma^2 / dt (density sigma over the sample period dt), the
    frame-to-frame bias change is a random walk of variance sigma_rw^2 T, and
    the residual is evaluated at the true states.  A bias random-walk variance
    of sigma_rw^2 / T instead of sigma_rw^2 T (or a per-sample variance of
    sigma^2 dt) moves the whitened covariance far from I."""
    c = _aligned_case()
    sg, sa = 1.7e-4, 2e-3
    x0, x1, q_IW, p = c["x0"], c["x1"], c["q_IW"], c["params"]
    stamps, T, dt = c["stamps"], c["T"], c["dt"]
    pre = imu.preintegrate(stamps, c["gyro"], c["acc"], 0.0, T, x0["bg"], x0["ba"], sg, sa)
    Sigma = imu.residual_covariance(x0, x1, q_IW, pre, p)
    rng = np.random.default_rng(31)
    N = 16000
    E = np.empty((N, 15))
    n = len(stamps)
    for k in range(N):
        gyro = c["gyro"] + rng.normal(size=(n, 3)) * (sg / np.sqrt(dt))
        acc = c["acc"] + rng.normal(size=(n, 3)) * (sa / np.sqrt(dt))
        dR, dv, dp = imu.integrate(stamps, gyro, acc, 0.0, T, x0["bg"], x0["ba"])
        noisy = dict(pre, dR=dR, dv=dv, dp=dp)  # integrated at x0's biases: no bias correction applies
        x1k = dict(x1, bg=x1["bg"] + rng.normal(size=3) * (p["sigma_bg_rw"] * np.sqrt(T)),
                   ba=x1["ba"] + rng.normal(size=3) * (p["sigma_ba_rw"] * np.sqrt(T)))
        E[k] = imu.residual(x0, x1k, q_IW, noisy, p)
    C = (E.T @ E) / N  # zero mean under the model (the truth has zero residual)
    gap = _whitened_gap(Sigma, C)
    # sampling spread of a whitened entry ~ sqrt(2 / N) = 0.011
    assert gap < 0.06, gap
    chi2 = np.einsum("ni,ij,nj->n", E, np.linalg.inv(Sigma), E).mean()
    assert abs(chi2 - 15.0) < 0.5, chi2
    # the planted slip: random-walk variance sigma_rw^2 / T
    slip = Sigma.copy()
    slip[9:12, 9:12] += np.eye(3) * p["sigma_bg_rw"] ** 2 * (1.0 / T - T)
    slip[12:15, 12:15] += np.eye(3) * p["sigma_ba_rw"] ** 2 * (1.0 / T - T)
    assert _whitened_gap(slip, C) > 0.5
    # and a per-sample noise variance sigma^2 dt instead of sigma^2 / dt
    pre_slip = imu.preintegrate(stamps, c["gyro"], c["acc"], 0.0, T, x0["bg"], x0["ba"], sg * dt, sa * dt)
    assert _whitened_gap(imu.residual_covariance(x0, x1, q_IW, pre_slip, p), C) > 0.5
