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
