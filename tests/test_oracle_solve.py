"""Pins of the oracle's Gauss-Newton system, prior and marginalisation (eqs. (6)-(9))."""
import numpy as np

from oracle import imu, lie, solve
from synth.configs import initial_prior
from tests.test_oracle_imu import _rigid_motion_case


def _spd(n, rng):
    A = rng.normal(size=(n, n))
    return A @ A.T + n * np.eye(n)


def test_schur_reduced_solve_equals_joint_solve():
    rng = np.random.default_rng(2)
    H = _spd(33, rng)
    b = rng.normal(size=33)
    x1 = {k: np.zeros(3) for k in ("r", "v", "bg", "ba")}
    x1["q"] = np.array([1.0, 0, 0, 0])
    pr = solve.marginalise(H, b, np.zeros(33), x1, np.array([1.0, 0, 0, 0]))
    dz = np.linalg.solve(H, b)
    assert np.allclose(np.linalg.solve(pr["H"], pr["b"]), dz[15:33], rtol=1e-12, atol=1e-12)
    # marginal information is the inverse of the kept block of the covariance
    C = np.linalg.inv(H)
    assert np.allclose(pr["H"], np.linalg.inv(C[15:33, 15:33]), rtol=1e-9, atol=1e-9)


def test_marginalisation_after_the_update_keeps_the_minimiser():
    # re-expressing b at the updated point: the prior's minimiser is the
    # updated kept state plus the remaining step, i.e. the same minimiser
    rng = np.random.default_rng(3)
    H = _spd(33, rng)
    b = rng.normal(size=33)
    dz = np.linalg.solve(H, b)
    x1 = {k: np.zeros(3) for k in ("r", "v", "bg", "ba")}
    x1["q"] = np.array([1.0, 0, 0, 0])
    pr = solve.marginalise(H, b, dz, x1, np.array([1.0, 0, 0, 0]))
    assert np.abs(pr["b"]).max() < 1e-10 * np.abs(b).max()


def test_first_order_correction_is_exact_for_vector_parts():
    """For vector-space coordinates, the prior of eq. (6) with the correction of
    eq. (9) has the same minimiser whatever point it is evaluated at."""
    rng = np.random.default_rng(4)
    Hs = _spd(18, rng)
    xbar = {"r": rng.normal(size=3), "q": np.array([1.0, 0, 0, 0]), "v": rng.normal(size=3),
            "bg": rng.normal(size=3), "ba": rng.normal(size=3)}
    prior = {"H": Hs, "b": rng.normal(size=18), "xbar": xbar, "qIW_bar": np.array([1.0, 0, 0, 0])}
    q = np.array([1.0, 0, 0, 0])
    minima = []
    for _ in range(3):
        x = lie.copy_state(xbar)
        for k in ("r", "v", "bg", "ba"):
            x[k] = x[k] + rng.normal(size=3)
        H, b = solve.prior_terms(x, q, prior)
        idx = np.r_[0:15, 30:33]
        d = np.linalg.solve(H[np.ix_(idx, idx)], b[idx])
        minima.append(np.concatenate([x["r"] + d[0:3], x["v"] + d[6:9], x["bg"] + d[9:12], x["ba"] + d[12:15]]))
    assert np.allclose(minima[0], minima[1], atol=1e-10) and np.allclose(minima[0], minima[2], atol=1e-10)
    d_expected = np.linalg.solve(Hs, prior["b"])
    assert np.allclose(minima[0][:3], xbar["r"] + d_expected[0:3], atol=1e-10)


def test_gravity_gauge_needs_the_yaw_prior():
    """Yaw of q_IW about gravity is unobservable (Section IV-A): with the pose
    fixed by the prior but no yaw prior, the IMU + prior system is rank deficient."""
    c = _rigid_motion_case()
    pre = imu.preintegrate(c["stamps"], c["gyro"], c["acc"], 0.0, c["T"], c["x0"]["bg"], c["x0"]["ba"], 1e-3, 1e-2)
    e, J, W = imu.factor(c["x0"], c["x1"], c["q_IW"], pre, c["params"])
    prior = initial_prior(c["x0"], c["q_IW"])
    Hp, _ = solve.prior_terms(c["x0"], c["q_IW"], prior)
    H = J.T @ W @ J + Hp
    # a pose-only prior on x1 makes the rest observable except the yaw gauge
    H[15:21, 15:21] += np.eye(6) * 1e8
    ev_with = np.linalg.eigvalsh(H)
    Hp_noyaw = Hp.copy()
    Hp_noyaw[32, 32] = 0.0
    Hn = J.T @ W @ J + Hp_noyaw
    Hn[15:21, 15:21] += np.eye(6) * 1e8
    ev, V = np.linalg.eigh(Hn)
    assert ev[0] < 1e-6 * ev[-1] and ev_with[0] > 1e-2
    # the null vector rotates gravity about z_I (with the velocities turning along)
    assert abs(V[32, 0]) > 0.5
