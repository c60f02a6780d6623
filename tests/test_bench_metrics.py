"""Host-side metrics of the benchmark's robustness comparison: the absolute
trajectory error (RMSE of position differences after the optional rigid
alignment) and the rotation angle between two orientations."""
import numpy as np

import bench


def _rot(axis, deg):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    t = np.radians(deg)
    return np.eye(3) + np.sin(t) * K + (1 - np.cos(t)) * K @ K


def test_ate_zero_for_identical_and_rigidly_moved_trajectories():
    rng = np.random.default_rng(7)
    gt = np.cumsum(rng.normal(size=(40, 3)) * 0.05, axis=0)
    assert bench.ate_rmse(gt, gt, align=False) == 0.0
    assert bench.ate_rmse(gt, gt) < 1e-12
    R, t = _rot([1, 2, 3], 37.0), np.array([0.3, -1.2, 2.0])
    moved = gt @ R.T + t
    assert bench.ate_rmse(moved, gt) < 1e-12  # removed by the alignment
    # without it, the error of a pure translation is its length
    assert abs(bench.ate_rmse(gt + t, gt, align=False) - np.linalg.norm(t)) < 1e-12


def test_ate_matches_hand_computed_residual():
    # a fixed offset of +-d along one axis on alternate points cannot be aligned away when the
    # points are spread along an orthogonal axis with zero mean offset: RMSE = d
    d = 0.01
    gt = np.stack([np.zeros(6), np.linspace(-1.0, 1.0, 6), np.zeros(6)], axis=1)
    est = gt.copy()
    est[:, 0] += d * np.array([1, -1, 1, -1, 1, -1])
    raw = bench.ate_rmse(est, gt, align=False)
    assert abs(raw - d) < 1e-15
    assert bench.ate_rmse(est, gt) <= raw + 1e-15  # alignment can only lower it


def test_ate_alignment_is_not_a_reflection():
    # a mirrored planar trajectory must not be "aligned" by a reflection
    rng = np.random.default_rng(3)
    gt = rng.normal(size=(30, 3))
    mirrored = gt * np.array([1.0, 1.0, -1.0])
    assert bench.ate_rmse(mirrored, gt) > 0.1


def test_rotation_angle():
    R = _rot([0, 0, 1], 30.0)
    assert abs(bench.rot_angle_deg(np.eye(3), R) - 30.0) < 1e-9
    assert abs(bench.rot_angle_deg(R, R)) < 1e-6
    assert abs(bench.rot_angle_deg(np.eye(3), _rot([1, 1, 0], 179.0)) - 179.0) < 1e-6


def test_sequence_accuracy_windows():
    rng = np.random.default_rng(11)
    gt = []
    for k in range(50):
        q = rng.normal(size=4)
        gt.append({"r": rng.normal(size=3), "q": q / np.linalg.norm(q), "v": rng.normal(size=3),
                   "bg": rng.normal(size=3) * 1e-3, "ba": rng.normal(size=3) * 1e-2})
    est = [dict(g) for g in gt]
    a = bench.sequence_accuracy(est, gt, windows=((0, 10), (10, None)))
    assert a["frames"] == 50 and a["ate_rmse_m"] == 0.0 and a["max_rot_err_deg"] < 1e-6
    assert [w["frames"] for w in a["windows"]] == [[1, 10], [11, 50]]
    assert all(w["vel_err_mps"] == 0.0 and w["bg_err_radps"] == 0.0 for w in a["windows"])
    # a velocity error of 0.3 m/s on the first 10 frames only, a gyro bias error of 1e-4 on the rest
    for k in range(50):
        est[k] = dict(gt[k])
        if k < 10:
            est[k]["v"] = gt[k]["v"] + np.array([0.0, 0.3, 0.0])
        else:
            est[k]["bg"] = gt[k]["bg"] + np.array([1e-4, 0.0, 0.0])
    a = bench.sequence_accuracy(est, gt, windows=((0, 10), (10, None)))
    assert abs(a["windows"][0]["vel_err_mps"] - 0.3) < 1e-12 and a["windows"][1]["vel_err_mps"] == 0.0
    assert a["windows"][0]["bg_err_radps"] == 0.0 and abs(a["windows"][1]["bg_err_radps"] - 1e-4) < 1e-15


def test_quaternion_angle_matches_rotation_matrices():
    import synth
    rng = np.random.default_rng(3)
    for _ in range(20):
        qa, qb = rng.normal(size=4), rng.normal(size=4)
        qa, qb = qa / np.linalg.norm(qa), qb / np.linalg.norm(qb)
        R = synth.configs._rot_from_quat
        ref = np.radians(bench.rot_angle_deg(R(qa), R(qb)))
        assert abs(bench.quat_angle(qa, qb) - ref) < 1e-9
        assert abs(bench.quat_angle(qa, -qb) - ref) < 1e-9  # q and -q are one rotation
    h = np.sqrt(0.5)
    assert abs(bench.quat_angle([1, 0, 0, 0], [h, h, 0, 0]) - np.pi / 2) < 1e-15


def test_counter_scaling(monkeypatch):
    """Counter readings in KiB become bytes through the calibration copy: a copy of COPY_BYTES each way
    reads c_f KiB and writes c_w KiB, so a kernel reading f KiB moved f / c_f * COPY_BYTES bytes."""
    c = dict(bench.COUNTERS, source_sha256=bench.residual_source_hash()[:16],
             copy_fetch_kib=2.0 * bench.COPY_BYTES / 1024, copy_write_kib=bench.COPY_BYTES / 1024,
             shapes={"2,1": {"fetch_kib": 1000.0, "write_kib": 10.0, "valu_insts": 123.0, "waves": 7}})
    monkeypatch.setattr(bench, "COUNTERS", c)
    f = bench.counter_figures(2, 1)
    assert f["fetch_bytes"] == 1000.0 * 1024 / 2.0 and f["write_bytes"] == 10.0 * 1024
    assert f["traffic_bytes"] == f["fetch_bytes"] + f["write_bytes"] and f["valu_insts"] == 123.0
    assert bench.counter_figures(2, 0) is None and bench.counter_figures(4, 1) is None  # other launch shapes
    monkeypatch.setattr(bench, "COUNTERS", dict(c, source_sha256="0" * 16))
    assert bench.counter_figures(2, 1) is None  # taken for other kernel sources


def test_batch_counter_scaling(monkeypatch):
    """The batched pass's per-pixel figures: scaled bytes and wave instructions over the mix's pixels."""
    c = dict(bench.COUNTERS, source_sha256=bench.residual_source_hash()[:16],
             copy_fetch_kib=2.0 * bench.COPY_BYTES / 1024, copy_write_kib=bench.COPY_BYTES / 1024,
             batch_banded={"pixels": 1000, "fetch_kib": 20.0, "write_kib": 1.0, "valu_insts": 5000})
    monkeypatch.setattr(bench, "COUNTERS", c)
    f = bench.batch_counter_figures()
    assert f["bytes_per_pixel"] == (20.0 * 1024 / 2.0 + 1.0 * 1024) / 1000 and f["valu_insts_per_pixel"] == 5.0
    monkeypatch.setattr(bench, "COUNTERS", dict(c, source_sha256="0" * 16))
    assert bench.batch_counter_figures() is None


def test_model_view_at_reproduces_the_sequence_render():
    """The closed-loop model view rendered at a state's pose equals the sequence's own noise-free render
    at that frame's ground-truth pose (same scene; the pose only goes through the world frame and back)."""
    import synth
    seq = synth.configs.session_sequence(77, 3, 64, 48)
    for j in range(3):
        z, inten, T = synth.configs.model_view_at(seq, seq["gt"][j])
        ref = seq["clean_depth"][j].numpy()
        zz = z.numpy()
        assert np.array_equal(zz > 0, ref > 0) or np.mean((zz > 0) != (ref > 0)) < 1e-3
        both = (zz > 0) & (ref > 0)
        assert np.max(np.abs(zz[both] - ref[both])) < 1e-5
        assert np.mean(inten.numpy() != seq["intensity"][j].numpy()) < 1e-3
        assert np.allclose(T[:3, 3], seq["gt"][j]["r"])


def test_session_sequence_flags_depend_on_the_seed_alone():
    import synth
    a = synth.configs.session_sequence(5011, 12, 32, 24, hole_rate=0.3, low_texture_rate=0.3)
    b = synth.configs.session_sequence(5011, 12, 32, 24, hole_rate=0.3, low_texture_rate=0.3)
    assert a["hole_frames"] == b["hole_frames"] and a["low_texture_frames"] == b["low_texture_frames"]
    assert a["hole_frames"] and a["low_texture_frames"] and 0 not in a["hole_frames"]
    for j in a["hole_frames"]:
        assert (a["depth"][j] == 0).float().mean() > 0.7
    c = synth.configs.session_sequence(5012, 12, 32, 24, hole_rate=0.3, low_texture_rate=0.3)
    assert not np.array_equal(a["depth"][1].numpy(), c["depth"][1].numpy())
