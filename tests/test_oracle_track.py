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
