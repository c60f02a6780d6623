"""Workload builders: the frame pair and the long single-session sequence.

Everything is seeded: ``numpy.random.Generator(PCG64(seed))`` for geometry,
trajectory and IMU noise, a seeded ``torch.Generator`` for depth noise.

Camera model at other resolutions: ``fx = fy = 130 W / 160``, ``cx = W/2``,
``cy = H/2`` (pixel centres at integer coordinates).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .imu_gen import GRAVITY, ImuNoise, state_truth, synth_imu
from .scene import make_scene, render
from .trajectory import ConstantTwistTrajectory, base_orientation, make_spline_trajectory, rotvec_to_matrix

# Table I (synthetic column) and the configs' sensor noise
BIAS_PRIOR_G = 0.03
BIAS_PRIOR_A = 0.1
SEQUENCE_SECONDS = 301 / 30.0


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


def camera_for(width: int, height: int) -> Camera:
    f = 130.0 * width / 160.0
    return Camera(width, height, f, f, width / 2.0, height / 2.0)


def quat_from_matrix(R) -> np.ndarray:
    """Hamilton unit quaternion (w, x, y, z) of a rotation matrix (Shepperd's method)."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif R[1, 1] > R[2, 2]:
        s = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    q /= np.linalg.norm(q)
    return q if q[0] >= 0 else -q


def make_state(R_WC, r_WC, v_IS, bg, ba) -> dict:
    return {"r": np.array(r_WC, dtype=np.float64), "q": quat_from_matrix(R_WC),
            "v": np.array(v_IS, dtype=np.float64), "bg": np.array(bg, dtype=np.float64),
            "ba": np.array(ba, dtype=np.float64)}


def initial_prior(state: dict, q_IW: np.ndarray) -> dict:
    """Prior on the first state: pose sigma 1e-4 (W is the first camera frame),
    velocity 0.1 m/s, biases at Table I's bias priors, gravity roll/pitch 0.05 rad,
    yaw 1e-4 rad (fixes the gauge about gravity)."""
    sig = np.concatenate([np.full(3, 1e-4), np.full(3, 1e-4), np.full(3, 0.1), np.full(3, BIAS_PRIOR_G),
                          np.full(3, BIAS_PRIOR_A), [0.05, 0.05, 1e-4]])
    return {"H": np.diag(1.0 / sig**2), "b": np.zeros(18), "xbar": {k: v.copy() for k, v in state.items()},
            "qIW_bar": np.array(q_IW, dtype=np.float64)}


def add_depth_noise(z: torch.Tensor, k: float, generator: torch.Generator) -> torch.Tensor:
    n = torch.randn(z.shape, generator=generator, dtype=torch.float64, device=generator.device).to(z.device)
    z64 = z.to(torch.float64)
    return torch.where(z64 > 0, z64 + n * k * z64 * z64, z64).to(torch.float32)


def imu_window(stamps: np.ndarray, t0: float, t1: float):
    """Indices of the samples whose hold intervals meet [t0, t1): the last
    sample stamped at or before t0 through the last stamped before t1."""
    first = int(np.searchsorted(stamps, t0, side="right")) - 1
    last = int(np.searchsorted(stamps, t1, side="left"))
    return max(first, 0), last


def frame_pair(seed: int = 1001, width: int = 160, height: int = 120, *, noisy_imu: bool = True,
               depth_noise: bool = True, device="cpu") -> dict:
    """Plain method, one frame pair: ground-truth offset of 2 deg about a random
    axis and 2 cm along a random direction over 15 ms; three IMU samples at
    200 Hz; constant biases 1e-3; depth noise N(0, (1e-3 z^2)^2)."""
    rng = np.random.default_rng(seed)
    scene = make_scene(rng, seed)
    R_IW = base_orientation(rng)
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    tdir = rng.normal(size=3)
    tdir /= np.linalg.norm(tdir)
    T = 0.015
    traj = ConstantTwistTrajectory(R_IW, math.radians(2.0) * axis, 0.02 * tdir, T)
    cam = camera_for(width, height)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    frames = []
    for t in (0.0, T):
        z, inten = render(scene, *traj.pose(t), cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, device=device)
        if depth_noise:
            z = add_depth_noise(z, 1e-3, gen)
        frames.append((z, inten))
    noise = ImuNoise()
    bias = np.full(3, 1e-3)
    stamps, gyro, acc, _, _ = synth_imu(traj, 0.0, T, 200.0, rng, noise, bias, bias, noisy=noisy_imu,
                                        bias_walk=False)
    R1 = rotvec_to_matrix(math.radians(2.0) * axis)
    v = traj.vel_I(0.0)
    gt0 = make_state(np.eye(3), np.zeros(3), v, bias, bias)
    gt1 = make_state(R1, 0.02 * tdir, v, bias, bias)
    q_IW = quat_from_matrix(R_IW)
    tilt = rng.normal(0.0, 0.01, size=3)
    tilt[2] = 0.0
    q_IW_init = quat_from_matrix(rotvec_to_matrix(tilt) @ R_IW)
    x0 = make_state(np.eye(3), np.zeros(3), v, np.zeros(3), np.zeros(3))
    return {
        "camera": cam, "scene": scene, "t0": 0.0, "t1": T,
        "model_depth": frames[0][0], "model_intensity": frames[0][1], "T_WM": np.eye(4),
        "depth": frames[1][0], "intensity": frames[1][1],
        "imu": {"t": stamps, "gyro": gyro, "acc": acc},
        "gt0": gt0, "gt1": gt1, "q_IW_gt": q_IW,
        "x0": x0, "q_IW": q_IW_init, "prior": initial_prior(x0, q_IW_init),
        "noise": noise, "gravity": GRAVITY,
    }


def sequence(seed: int = 2001, n_frames: int = 300, width: int = 640, height: int = 480, *, fps: float = 30.0,
             imu_rate: float = 200.0, device="cpu", low_texture_every: int = 0, duration: float | None = None,
             low_texture_frames=(), hole_frames=(), hole_fraction: float = 0.8, layout: str = "room") -> dict:
    """Plain method, single session: a seeded smooth B-spline trajectory (peak
    1.5 m/s, 180 deg/s), IMU at 200 Hz with random-walk biases.  Frame j is
    rendered at its ground-truth pose with depth noise; the model view used to
    track frame j is the noise-free render at frame j-1's ground-truth pose.

    Stress options: frames listed in ``low_texture_frames`` (or every
    ``low_texture_every``-th) get the low-texture albedo (variance x 0.01);
    frames in ``hole_frames`` lose ``hole_fraction`` of their measured depth to
    zero-depth blobs (value noise thresholded at that quantile).  ``layout``
    "wall" renders the back wall alone (same trajectory and IMU stream)."""
    rng = np.random.default_rng(seed)
    scene = make_scene(rng, seed, layout)
    # by default the trajectory and the IMU stream span the full 10 s sequence, so
    # a shorter sequence is a prefix of the long one; an explicit duration (the
    # serving workload's many short sessions) trades that for generation time
    duration = max((n_frames + 1) / fps, SEQUENCE_SECONDS if duration is None else duration)
    traj = make_spline_trajectory(rng, duration)
    cam = camera_for(width, height)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    R_IW = traj.pose(0.0)[0]
    times = np.arange(n_frames) / fps
    clean, noisy, gts, hole_list, lowt_list = [], [], [], [], []
    noise = ImuNoise()
    bg0 = rng.normal(0.0, 2e-3, 3)
    ba0 = rng.normal(0.0, 2e-2, 3)
    stamps, gyro, acc, tbg, tba = synth_imu(traj, 0.0, duration - 1.0 / fps, imu_rate, rng, noise, bg0, ba0)
    for j, t in enumerate(times):
        R_IC, p_IC = traj.pose(t)
        lt = bool(low_texture_every and j % low_texture_every == 0) or j in set(low_texture_frames)
        z, inten = render(scene, R_IC, p_IC, cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                          device=device, low_texture=lt)
        clean.append(z)
        zn = add_depth_noise(z, 1e-3, gen)
        if lt:
            lowt_list.append(j)
        if j in set(hole_frames):
            zn = apply_holes(zn, seed * 1000 + j, hole_fraction)
            hole_list.append(j)
        noisy.append((zn, inten))
        _, _, v = state_truth(traj, t)
        k = min(int(np.searchsorted(stamps, t, side="right")) - 1, len(stamps) - 1)
        gts.append(make_state(R_IW.T @ R_IC, R_IW.T @ p_IC, v, tbg[k], tba[k]))
    q_IW = quat_from_matrix(R_IW)
    tilt = rng.normal(0.0, 0.01, size=3)
    tilt[2] = 0.0
    q_IW_init = quat_from_matrix(rotvec_to_matrix(tilt) @ R_IW)
    g0 = gts[0]
    x0 = {"r": g0["r"].copy(), "q": g0["q"].copy(), "v": g0["v"].copy(), "bg": np.zeros(3), "ba": np.zeros(3)}
    return {
        "camera": cam, "scene": scene, "times": times, "n_frames": n_frames,
        "depth": [f[0] for f in noisy], "intensity": [f[1] for f in noisy], "clean_depth": clean,
        "imu": {"t": stamps, "gyro": gyro, "acc": acc}, "gt": gts, "q_IW_gt": q_IW,
        "x0": x0, "q_IW": q_IW_init, "prior": initial_prior(x0, q_IW_init), "noise": noise,
        "gravity": GRAVITY, "hole_frames": hole_list, "low_texture_frames": lowt_list,
    }


def apply_holes(z: torch.Tensor, seed: int, fraction: float) -> torch.Tensor:
    """Zero the depth where smooth value noise falls below its `fraction` quantile (blob-shaped holes)."""
    from .scene import value_noise2
    H, W = z.shape
    jj, ii = torch.meshgrid(torch.arange(H, dtype=torch.float64, device=z.device),
                            torch.arange(W, dtype=torch.float64, device=z.device), indexing="ij")
    hv = value_noise2(ii, jj, seed, scale=1.0 / (24.0 * max(1.0, W / 640.0)))
    flat = hv.flatten().float()
    if flat.numel() > 4_000_000:  # quantile of a strided sample for very large images
        flat = flat[:: (flat.numel() // 4_000_000) + 1]
    thr = torch.quantile(flat, fraction).to(torch.float64)
    return torch.where(hv < thr, torch.zeros_like(z), z)


def model_view(seq: dict, j: int):
    """Reference for tracking frame j: the noise-free render at frame j-1's
    ground-truth pose, with that pose as the model pose T_WM."""
    g = seq["gt"][j - 1]
    T = np.eye(4)
    T[:3, :3] = _rot_from_quat(g["q"])
    T[:3, 3] = g["r"]
    return seq["clean_depth"][j - 1], seq["intensity"][j - 1], T


def model_view_at(seq: dict, state: dict, *, low_texture: bool = False):
    """Noise-free render of the sequence's scene at the camera pose of
    ``state`` (world frame of the sequence's states, e.g. the previous frame's
    estimate for closed-loop tracking), with that pose as T_WM.  Returned on
    the device the sequence was generated on."""
    R_IW = _rot_from_quat(seq["q_IW_gt"])
    R_WC = _rot_from_quat(np.asarray(state["q"], dtype=np.float64) / np.linalg.norm(state["q"]))
    r_WC = np.asarray(state["r"], dtype=np.float64)
    cam = seq["camera"]
    z, inten = render(seq["scene"], R_IW @ R_WC, R_IW @ r_WC, cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                      device=seq["depth"][0].device, low_texture=low_texture)
    T = np.eye(4)
    T[:3, :3] = R_WC
    T[:3, 3] = r_WC
    return z, inten, T


def session_sequence(seed: int, n_frames: int, width: int, height: int, *, device="cpu", hole_rate: float = 0.0,
                     low_texture_rate: float = 0.0) -> dict:
    """One serving session's own short sequence: scene, trajectory and IMU
    stream from ``seed``, the trajectory spanning the frames alone.  Each of
    frames 1..n_frames-1 independently gets 80% zero-depth holes with
    probability ``hole_rate`` and the low-texture albedo with probability
    ``low_texture_rate`` (draws from a generator seeded by (seed, 7), so the
    frame flags of one session do not depend on the other sessions)."""
    draws = np.random.default_rng([seed, 7]).random((n_frames, 2))
    holes = [j for j in range(1, n_frames) if draws[j, 0] < hole_rate]
    lowt = [j for j in range(1, n_frames) if draws[j, 1] < low_texture_rate]
    return sequence(seed=seed, n_frames=n_frames, width=width, height=height, device=device,
                    duration=(n_frames + 2) / 30.0, hole_frames=holes, low_texture_frames=lowt)


def _rot_from_quat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
