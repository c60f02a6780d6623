"""Photometric and point-to-plane ICP terms, value layer in float64.

Photometric residual, eq. (3): for current pixel u with depth d,
``e = I0(pi(K T_WC0^-1 T_WC1 rho(u, d))) - I1(u)``; the warp uses the previous
*state* pose T_WC0, so the term couples x0 and x1.  I0 is the reference
(model-view) intensity, sampled bilinearly; its gradient is sampled bilinearly
from the central-difference gradient map.

ICP residual, eq. (4): ``e = n_W^T (T_WC1 p_C1 - p_W)`` with (p_W, n_W) the
associated model-view vertex and normal, mapped to W by the model-view pose.

The paper omits the Jacobians (Section IV-D).  With the left perturbations of
Section IV-A (R <- exp(da) R, r <- r + dr) they are, per pixel:

* ICP, with respect to (dr1, da1): ``[n_W, (R1 p) x n_W]``;
* RGB, with w = R1 p + r1 - r0, x' = R0^T w, g = grad I0 . d pi / d x' and
  h = R0 g^T, with respect to (dr0, da0, dr1, da1):
  ``[-h, h x w, h, (R1 p) x h]``.

Weights are the inverse measurement variances the paper uses in place of a
tuning factor (Sections III, IV-D): W_RGB = 1/sigma_I^2 and
W_ICP,k = 1/(k_z z_k^2)^2 at the current depth z_k.  A Huber multiplier
psi(s)/s on the whitened residual s = |e| sqrt(W) is applied on top
(huber_k = 0 switches it off).
"""
from __future__ import annotations

import numpy as np

from .association import icp_association, rgb_validity
from .lie import quat_to_rot


def huber_weight(s, k):
    """psi(s)/s of the Huber loss: 1 for s <= k, k/s beyond (k <= 0: no robust weight)."""
    s = np.asarray(s, dtype=np.float64)
    if k <= 0:
        return np.ones_like(s)
    return np.where(s <= k, 1.0, k / np.maximum(s, 1e-300))


def bilinear(img, u, v):
    """Bilinear sample of a 2-D map at float64 coordinates (caller ensures interior)."""
    x0 = np.floor(u).astype(np.int64)
    y0 = np.floor(v).astype(np.int64)
    a = u - x0
    b = v - y0
    im = np.asarray(img, dtype=np.float64)
    return ((1 - a) * (1 - b) * im[y0, x0] + a * (1 - b) * im[y0, x0 + 1]
            + (1 - a) * b * im[y0 + 1, x0] + a * b * im[y0 + 1, x0 + 1])


def icp_terms(cur, ref, T_WM, x1, Ra, ta, params):
    """Per-pixel ICP residuals, Jacobians (w.r.t. x1's dr, da) and weights.

    Returns a dict with mask (H, W), e (n,), J (n, 6), w (n,) for the valid pixels.
    """
    mask, iu, iv = icp_association(cur, ref, Ra, ta, params.get("icp_dist", 0.10), params.get("icp_cos"))
    p = cur["V"][mask].astype(np.float64)
    v0 = ref["V"][iv[mask], iu[mask]].astype(np.float64)
    n0 = ref["N"][iv[mask], iu[mask]].astype(np.float64)
    R_WM, t_WM = T_WM[:3, :3], T_WM[:3, 3]
    pW = v0 @ R_WM.T + t_WM
    nW = n0 @ R_WM.T
    R1 = quat_to_rot(x1["q"])
    R1p = p @ R1.T
    e = np.einsum("ij,ij->i", nW, R1p + x1["r"] - pW)
    J = np.concatenate([nW, np.cross(R1p, nW)], axis=1)
    sigma = params["depth_k"] * p[:, 2] ** 2
    W = 1.0 / sigma**2
    w = W * huber_weight(np.abs(e) / sigma, params["huber_k"])
    return {"mask": mask, "e": e, "J": J, "w": w}


def rgb_terms(cur, ref, x0, x1, Rb, tb, params):
    """Per-pixel photometric residuals, Jacobians (w.r.t. x0 and x1 poses) and weights.

    Returns a dict with mask (H, W), e (n,), J (n, 12), w (n,).
    """
    mask, _, _ = rgb_validity(cur, ref, Rb, tb)
    p = cur["V"][mask].astype(np.float64)
    I1 = cur["I"][mask].astype(np.float64)
    fx, fy, cx, cy = (float(k) for k in ref["K"])
    R0 = quat_to_rot(x0["q"])
    R1 = quat_to_rot(x1["q"])
    R1p = p @ R1.T
    wv = R1p + x1["r"] - x0["r"]
    xp = wv @ R0  # R0^T w, row-wise
    z = xp[:, 2]
    u = fx * xp[:, 0] / z + cx
    v = fy * xp[:, 1] / z + cy
    I0 = bilinear(ref["I"], u, v)
    gx = bilinear(ref["G"][..., 0], u, v)
    gy = bilinear(ref["G"][..., 1], u, v)
    e = I0 - I1
    g = np.stack([gx * fx / z, gy * fy / z, -(gx * fx * xp[:, 0] + gy * fy * xp[:, 1]) / z**2], axis=1)
    h = g @ R0.T  # R0 g^T, row-wise
    J = np.concatenate([-h, np.cross(h, wv), h, np.cross(R1p, h)], axis=1)
    sig = params["sigma_I"]
    W = 1.0 / sig**2
    w = W * huber_weight(np.abs(e) / sig, params["huber_k"])
    return {"mask": mask, "e": e, "J": J, "w": w}


def normal_equations(terms, cols, dim):
    """Sum w J^T J and -w J^T e into a dim-sized system over the given columns.

    Returns (H, b, cost, count) with b = -sum w J^T e (the Gauss-Newton right-hand side).
    """
    H = np.zeros((dim, dim))
    b = np.zeros(dim)
    J, e, w = terms["J"], terms["e"], terms["w"]
    if J.shape[0]:
        Jw = J * w[:, None]
        H[np.ix_(cols, cols)] = Jw.T @ J
        b[cols] = -(Jw.T @ e)
    return H, b, float(np.sum(w * e * e)), int(J.shape[0])
