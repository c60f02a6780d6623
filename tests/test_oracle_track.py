"""End-to-end sanity pins of the oracle tracking step on the frame pair."""
import numpy as np

import synth
from oracle import lie, track


def _run(mode, **kw):
    d = synth.configs.frame_pair(**kw)
    p = track.default_params(levels=2, iters=(4, 4), mode=mode)
    out = track.track_frame(d["depth"].numpy(), d["intensity"].numpy(), d["model_depth"].numpy(),
                            d["model_intensity"].numpy(), d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"],
                            d["x0"], d["q_IW"], d["prior"], p, record=True)
    return d, out


def test_frame_pair_tracks_close_to_ground_truth():
    for mode in ("rgbd", "rgbdi", "gyro"):
        d, out = _run(mode)
        assert out["status"] == "ok"
        gt = d["gt1"]
        assert np.linalg.norm(out["x1"]["r"] - gt["r"]) < 5e-3
        assert np.linalg.norm(lie.quat_boxminus(out["x1"]["q"], gt["q"])) < 3e-3
        assert out["log"][-1]["n_icp"] > 5000 and out["log"][-1]["n_rgb"] > 15000


def test_marginal_prior_is_spd_and_small_gradient():
    d, out = _run("rgbdi")
    pr = out["prior"]
    assert np.allclose(pr["H"], pr["H"].T)
    assert np.linalg.eigvalsh(pr["H"]).min() > 0
    # the prior is expressed at the updated point: its minimiser is close to xbar
    step = np.linalg.solve(pr["H"], pr["b"])
    assert np.abs(step[0:6]).max() < 1e-3


def test_no_valid_depth_is_singular_in_rgbd_mode():
    d = synth.configs.frame_pair()
    p = track.default_params(levels=2, iters=(2, 2), mode="rgbd")
    z = np.zeros_like(d["depth"].numpy())
    out = track.track_frame(z, d["intensity"].numpy(), d["model_depth"].numpy(), d["model_intensity"].numpy(),
                            d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"], d["q_IW"], d["prior"], p)
    assert out["status"] == "singular"
    # with the IMU and prior terms the same frame still solves (IMU carries it)
    p["mode"] = "rgbdi"
    out = track.track_frame(z, d["intensity"].numpy(), d["model_depth"].numpy(), d["model_intensity"].numpy(),
                            d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"], d["q_IW"], d["prior"], p)
    assert out["status"] == "ok"


def test_gyro_only_holds_the_entries_only_accelerometers_observe():
    d, out = _run("gyro")
    assert out["status"] == "ok"
    for k in ("v", "ba"):
        assert np.array_equal(out["x1"][k], d["x0"][k]) and np.array_equal(out["x0"][k], d["x0"][k])
    assert np.array_equal(out["q_IW"], d["q_IW"])
    # the marginal prior keeps them decoupled (identity rows, zero right-hand side)
    H, b = out["prior"]["H"], out["prior"]["b"]
    fixed = np.r_[6:9, 12:15, 15:18]  # x1 velocity, x1 accelerometer bias, gravity direction
    assert np.array_equal(H[np.ix_(fixed, fixed)], np.eye(9))
    free = np.setdiff1d(np.arange(18), fixed)
    assert not H[np.ix_(fixed, free)].any() and not b[fixed].any()
    assert np.linalg.eigvalsh(H).min() > 0


def test_gyro_only_fails_without_visual_input():
    """The paper's observation for the gyro-only variant: with no visual
    constraint the relative position is unconstrained (singular), while the
    full IMU factor still carries the frame."""
    d = synth.configs.frame_pair()
    z = np.zeros_like(d["depth"].numpy())
    for mode, want in (("gyro", "singular"), ("rgbdi", "ok")):
        p = track.default_params(levels=2, iters=(2, 2), mode=mode)
        out = track.track_frame(z, d["intensity"].numpy(), d["model_depth"].numpy(), d["model_intensity"].numpy(),
                                d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"], d["q_IW"], d["prior"], p)
        assert out["status"] == want, mode


def _lost_pair(seed, patch):
    """The 160x120 frame pair with the current depth zeroed outside a small patch: too few inliers (the
    patch's pixels) to track, so the frame is lost (LOW_INLIERS)."""
    d = synth.configs.frame_pair(seed=seed, width=160, height=120)
    z = d["depth"].numpy().copy()
    keep = np.zeros_like(z, dtype=bool)
    r, c = patch
    keep[r:r + 6, c:c + 6] = True
    z[~keep] = 0.0
    return d, z


def _track(d, z, fallback, iters=(4, 4)):
    p = track.default_params(levels=2, iters=iters, mode="rgbdi")
    p["imu_fallback"] = fallback
    return track.track_frame(z, d["intensity"].numpy(), d["model_depth"].numpy(), d["model_intensity"].numpy(),
                             d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"], d["q_IW"], d["prior"], p)


def test_health_flags_clean_and_lost_frames():
    d = synth.configs.frame_pair(seed=1001, width=160, height=120)
    assert _track(d, d["depth"].numpy(), True)["health"] == []
    d, z = _lost_pair(1001, (60, 80))
    o = _track(d, z, False)
    assert "low_inliers" in o["health"] and "imu_only" not in o["health"]


def test_inertial_fallback_is_the_imu_prediction_under_a_consistent_prior():
    """Without visual terms, from the IMU prediction and under a prior centred on x0 with zero gradient,
    every residual of the prior and the IMU factor is zero: the Gauss-Newton step vanishes and the
    fallback returns the prediction itself (Section IV-C), with x0 unchanged."""
    d, z = _lost_pair(1001, (60, 80))
    o = _track(d, z, True)
    assert "low_inliers" in o["health"] and "imu_only" in o["health"]
    pre = o["preint"]
    p = track.default_params(levels=2, iters=(4, 4), mode="rgbdi")
    pred = track.imu_mod.predict_state(d["x0"], d["q_IW"], pre, p)
    for k in ("r", "q", "v", "bg", "ba"):
        assert np.max(np.abs(o["x1"][k] - pred[k])) < 1e-10, k
        assert np.max(np.abs(o["x0"][k] - d["x0"][k])) < 1e-10, k
    assert np.max(np.abs(o["q_IW"] - d["q_IW"])) < 1e-12
    assert np.all(np.linalg.eigvalsh(0.5 * (o["prior"]["H"] + o["prior"]["H"].T)) > 0)


def test_inertial_fallback_ignores_the_frames_visual_data():
    """The fallback drops the lost frame's visual terms: two lost frames that differ only in their few
    valid pixels give the same re-estimate, while their joint estimates differ."""
    d, za = _lost_pair(1001, (60, 80))
    _, zb = _lost_pair(1001, (20, 30))
    a, b = _track(d, za, True), _track(d, zb, True)
    ja, jb = _track(d, za, False), _track(d, zb, False)
    for k in ("r", "q", "v", "bg", "ba"):
        assert np.array_equal(a["x1"][k], b["x1"][k]), k
    assert np.array_equal(a["prior"]["H"], b["prior"]["H"]) and np.array_equal(a["prior"]["b"], b["prior"]["b"])
    assert max(np.max(np.abs(ja["x1"][k] - jb["x1"][k])) for k in ("r", "q", "v")) > 0.0


def test_joint_mode_converges_to_the_common_zero_of_all_residuals():
    """RGB-D-inertial pin with an exact answer.  The IMU reads a constant rate and specific force, so the
    zero-order hold is exact and the IMU prediction is the true x1 (Section IV-C); frame 1 is the plane +
    ramp scene rendered at that pose (every ICP and photometric residual vanishes there, Section IV-B);
    the prior is centred on x0 with zero gradient (Section IV-E).  All residuals of eq. (6) vanish at one
    state, so the joint Gauss-Newton started 1 cm / 1 degree away (x1) must return to it: a sign or
    assembly error in any term of the joint system moves the fixed point or stops the convergence."""
    from tests.oracle_cases import imu_plane_pair
    d = imu_plane_pair()
    x0, x1, q_IW, p = d["x0"], d["x1"], d["q_IW"], d["params"]
    start = lie.state_boxplus(x1, np.r_[0.01 * np.array([0.6, -0.8, 0.0]), np.deg2rad(1.0) * np.array([0.0, 0.6, 0.8]),
                                        np.zeros(9)])
    out = track.track_frame(d["z1"], d["I1"], d["z0"], d["I0"], np.eye(4), d["camera"], d["imu"], 0.0, 0.015, x0,
                            q_IW, d["prior"], p, x1_init=start)
    assert out["status"] == "ok" and out["health"] == []
    assert np.linalg.norm(out["x1"]["r"] - x1["r"]) < 1e-7
    assert np.linalg.norm(lie.quat_boxminus(out["x1"]["q"], x1["q"])) < 1e-7
    assert np.linalg.norm(out["x1"]["v"] - x1["v"]) < 1e-6
    assert np.linalg.norm(out["x0"]["r"] - x0["r"]) < 1e-7 and np.linalg.norm(out["x0"]["v"] - x0["v"]) < 1e-6
    assert np.linalg.norm(lie.quat_boxminus(out["q_IW"], q_IW)) < 1e-7
