"""Projective data association and validity masks, FP32 mirror (mask layer).

The ICP term pairs each current point with "a corresponding point in the
global model" (Section IV-B, eq. (4)) without stating the rule; the
photometric term samples the reference image at the warped pixel (eq. (3)).
Readings taken here:

* ICP: transform the current vertex into the model-view camera,
  q = R_a p + t_a, project it with the pinhole model, round to the nearest
  pixel (half-even), and accept the pair when the pixel is in the image, the
  current depth, the model depth and the model normal are valid and
  |q - v0|^2 <= d_max^2 (d_max = 0.10 m).  Eq. (4) involves only the model
  normal; an optional compatibility gate (rotated current normal within an
  angle of the model normal, given as a cosine) is off by default: with the
  configured depth noise at full resolution the forward-difference normals of
  the raw current depth are dominated by noise, and such a gate discards most
  correct pairs;
* RGB: transform into the reference camera, q' = R_b p + t_b, project without
  rounding, and accept when q'.z > 0 and 1 <= u' < W-2, 1 <= v' < H-2, so
  that every bilinear tap has a central-difference gradient.

Inputs are float32 transforms given as D = R - I (row-major 3x3, the
rotation's offset from the identity, rounded once to float32 from its float64
value) and t.  Keeping the offset instead of R makes the rounding of the
transform about as small as the rotation angle times one ulp, which matters
because every pixel sees the same rounding.  Every operation is a single
float32 operation with no contraction: a point maps as
q_x = x + (((D00 x + D01 y) + D02 z) + t0) (likewise y, z), the projection is
inv = 1/z; u = ((fx x) inv) + cx.
"""
from __future__ import annotations

import numpy as np

F = np.float32
DIST_THRESHOLD = 0.10              # metres


def _xform(D, t, x, y, z):
    """q = p + (D p + t), D = R - I, all float32."""
    D = np.asarray(D, dtype=np.float32).reshape(3, 3)
    t = np.asarray(t, dtype=np.float32).reshape(3)
    p = (x, y, z)
    return [(p[r] + (((D[r, 0] * x + D[r, 1] * y) + D[r, 2] * z) + t[r])).astype(np.float32) for r in range(3)]


def _rotate(D, x, y, z):
    """n' = n + D n."""
    D = np.asarray(D, dtype=np.float32).reshape(3, 3)
    p = (x, y, z)
    return [(p[r] + ((D[r, 0] * x + D[r, 1] * y) + D[r, 2] * z)).astype(np.float32) for r in range(3)]


def _project(qx, qy, qz, K):
    fx, fy, cx, cy = (F(k) for k in K)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = (F(1) / qz).astype(np.float32)
        u = ((fx * qx) * inv + cx).astype(np.float32)
        v = ((fy * qy) * inv + cy).astype(np.float32)
    return u, v


def icp_association(cur: dict, ref: dict, Da, ta, dist=DIST_THRESHOLD, cos_min=None):
    """Returns (valid mask, ui, vi) over the current level's pixels.

    dist: association distance gate (m); the squared gate is dist^2 rounded to
    float32.  cos_min: optional normal-compatibility gate (None: off)."""
    V1, N1, D1 = cur["V"], cur["N"], cur["D"]
    V0, N0, D0 = ref["V"], ref["N"], ref["D"]
    H0, W0 = D0.shape
    x, y, z = V1[..., 0], V1[..., 1], V1[..., 2]
    qx, qy, qz = _xform(Da, ta, x, y, z)
    u, v = _project(qx, qy, qz, ref["K"])
    ui = np.rint(u).astype(np.float32)
    vi = np.rint(v).astype(np.float32)
    with np.errstate(invalid="ignore"):
        inb = (ui >= F(0)) & (ui <= F(W0 - 1)) & (vi >= F(0)) & (vi <= F(H0 - 1))
    ok = (D1 > F(0)) & (qz > F(0)) & inb
    iu = np.where(ok, ui, 0).astype(np.int64)
    iv = np.where(ok, vi, 0).astype(np.int64)
    d0 = D0[iv, iu]
    v0 = V0[iv, iu]
    n0 = N0[iv, iu]
    n0_ok = (n0[..., 0] != 0) | (n0[..., 1] != 0) | (n0[..., 2] != 0)
    ex = (qx - v0[..., 0]).astype(np.float32)
    ey = (qy - v0[..., 1]).astype(np.float32)
    ez = (qz - v0[..., 2]).astype(np.float32)
    dist2 = ((ex * ex + ey * ey) + ez * ez).astype(np.float32)
    ok = ok & (d0 > F(0)) & n0_ok & (dist2 <= F(dist * dist))
    if cos_min is not None:
        n1_ok = (N1[..., 0] != 0) | (N1[..., 1] != 0) | (N1[..., 2] != 0)
        nx, ny, nz = _rotate(Da, N1[..., 0], N1[..., 1], N1[..., 2])
        cosang = ((nx * n0[..., 0] + ny * n0[..., 1]) + nz * n0[..., 2]).astype(np.float32)
        ok = ok & n1_ok & (cosang >= F(cos_min))
    return ok, iu, iv


def rgb_validity(cur: dict, ref: dict, Db, tb):
    """Returns (valid mask, u', v') with u', v' the float32 warped coordinates."""
    V1, D1 = cur["V"], cur["D"]
    H0, W0 = ref["D"].shape
    x, y, z = V1[..., 0], V1[..., 1], V1[..., 2]
    qx, qy, qz = _xform(Db, tb, x, y, z)
    u, v = _project(qx, qy, qz, ref["K"])
    with np.errstate(invalid="ignore"):
        inside = (u >= F(1)) & (u < F(W0 - 2)) & (v >= F(1)) & (v < F(H0 - 2))
    ok = (D1 > F(0)) & (qz > F(0)) & inside
    return ok, u, v
