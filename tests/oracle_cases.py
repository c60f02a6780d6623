"""Small seeded scenes shared by the oracle pins (inputs only)."""
import numpy as np

from synth.scene import Scene, render
from synth.trajectory import rotvec_to_matrix


def tilted_plane_pair(W=160, H=120, seed=0, ramp=(0.75, 0.5, 10.0)):
    """One tilted plane filling the view, a 2 deg / 2 cm ground-truth offset,
    a linear-ramp reference intensity I0 and the current intensity
    I1(u) = I0(warp_gt(u)) computed in float64 from the current depth.

    With this construction every ICP and photometric residual vanishes at the
    ground truth up to float32 rounding, so Gauss-Newton must recover it.
    """
    rng = np.random.default_rng(seed)
    f = 130.0 * W / 160.0
    cx, cy = W / 2.0, H / 2.0
    n = np.array([0.3, -0.4, -1.0])
    n /= np.linalg.norm(n)
    sc = Scene(planes=[(n, -2.0)], spheres=[], seed=seed)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    td = rng.normal(size=3)
    td /= np.linalg.norm(td)
    R1 = rotvec_to_matrix(np.deg2rad(2.0) * ax)
    r1 = 0.02 * td
    z0, _ = render(sc, np.eye(3), np.zeros(3), W, H, f, f, cx, cy)
    z1, _ = render(sc, R1, r1, W, H, f, f, cx, cy)
    z0, z1 = z0.numpy(), z1.numpy()
    jj, ii = np.mgrid[0:H, 0:W].astype(np.float64)
    a, b, c = ramp
    I0 = (a * ii + b * jj + c).astype(np.float32)
    z = z1.astype(np.float64)
    P = np.stack([(ii - cx) * z / f, (jj - cy) * z / f, z], -1)
    Q = P @ R1.T + r1
    u = f * Q[..., 0] / Q[..., 2] + cx
    v = f * Q[..., 1] / Q[..., 2] + cy
    I1 = (a * u + b * v + c).astype(np.float32)
    return {"z0": z0, "I0": I0, "z1": z1, "I1": I1, "R1": R1, "r1": r1, "f": f, "cx": cx, "cy": cy, "W": W, "H": H}


def identity_state():
    return {"r": np.zeros(3), "q": np.array([1.0, 0, 0, 0]), "v": np.zeros(3), "bg": np.zeros(3), "ba": np.zeros(3)}


def imu_plane_pair(W=160, H=120, seed=11):
    """A frame pair whose every residual of the joint cost vanishes at one known state: the IMU reads a
    constant body rate (2 deg over 15 ms) and specific force (about hover), for which the zero-order hold
    is exact, so the oracle's IMU prediction is the true x1; frame 1 is the tilted-plane, linear-ramp scene
    rendered at that pose (ICP and photometric residuals vanish there); the prior is centred on x0.  The
    intensities are float32; I0_u8 / I1_u8 are them rounded to the grey levels the device boundary takes
    (exact no longer: the rounding moves the solution by about 3e-5 m in x1's position and 2e-4 rad in the
    gravity direction)."""
    from oracle import imu as imu_mod
    from oracle import lie
    from oracle import track
    from synth.configs import Camera, initial_prior, quat_from_matrix
    f = 130.0 * W / 160.0
    cx, cy = W / 2.0, H / 2.0
    rng = np.random.default_rng(seed)
    p = track.default_params(levels=2, iters=(6, 6), mode="rgbdi")
    x0 = {"r": np.zeros(3), "q": np.array([1.0, 0.0, 0.0, 0.0]), "v": np.array([0.9, -0.4, 0.6]),
          "bg": np.zeros(3), "ba": np.zeros(3)}
    q_IW = quat_from_matrix(lie.exp_so3(np.array([0.3, -0.2, 0.0])))
    w = rng.normal(size=3)
    w *= np.deg2rad(2.0) / 0.015 / np.linalg.norm(w)
    R_IW = lie.quat_to_rot(q_IW)
    fsp = R_IW.T @ np.array([0.0, 0.0, p["gravity"]]) + rng.normal(size=3) * 0.5
    imu = {"t": np.array([0.0, 0.005, 0.010]), "gyro": np.tile(w, (3, 1)), "acc": np.tile(fsp, (3, 1))}
    pre = imu_mod.preintegrate(imu["t"], imu["gyro"], imu["acc"], 0.0, 0.015, x0["bg"], x0["ba"],
                               p["sigma_g"], p["sigma_a"])
    x1 = imu_mod.predict_state(x0, q_IW, pre, p)
    R1 = lie.quat_to_rot(x1["q"])
    n = np.array([0.3, -0.4, -1.0])
    n /= np.linalg.norm(n)
    sc = Scene(planes=[(n, -2.0)], spheres=[], seed=0)
    z0, _ = render(sc, np.eye(3), np.zeros(3), W, H, f, f, cx, cy)
    z1, _ = render(sc, R1, x1["r"], W, H, f, f, cx, cy)
    z0, z1 = z0.numpy(), z1.numpy()
    jj, ii = np.mgrid[0:H, 0:W].astype(np.float64)
    a, b, c = 0.75, 0.5, 10.0
    I0 = (a * ii + b * jj + c).astype(np.float32)
    z = z1.astype(np.float64)
    P = np.stack([(ii - cx) * z / f, (jj - cy) * z / f, z], -1)
    Q = P @ R1.T + x1["r"]
    I1 = (a * (f * Q[..., 0] / Q[..., 2] + cx) + b * (f * Q[..., 1] / Q[..., 2] + cy) + c).astype(np.float32)
    u8 = lambda a: np.clip(np.rint(a), 0, 255).astype(np.uint8)  # noqa: E731
    return {"z0": z0, "I0": I0, "z1": z1, "I1": I1, "I0_u8": u8(I0), "I1_u8": u8(I1),
            "camera": Camera(W, H, f, f, cx, cy), "imu": imu,
            "x0": x0, "x1": x1, "q_IW": q_IW, "prior": initial_prior(x0, q_IW), "params": p}
