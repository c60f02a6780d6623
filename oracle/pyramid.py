"""Image pyramid, FP32 mirror (mask layer).

The paper minimises its cost over a three-level coarse-to-fine pyramid
(Section IV-D) but does not say how the levels are built.  Reading taken here:

* level 0: depth = input where finite and > 0, else 0; intensity = float(uint8);
* level l+1 depth: mean of the valid depths of the 2x2 block, visited in the
  order (2x,2y), (2x+1,2y), (2x,2y+1), (2x+1,2y+1), summed left to right, then
  divided by their count (0 if none is valid);
* level l+1 intensity: ((a + b) + (c + d)) * 0.25 over the same block;
* intrinsics: fx_l = fx 2^-l, cx_l = (cx + 0.5) 2^-l - 0.5 (pixel centres);
* vertex map: back-projection rho(u, d) of Section IV-B,
  x = ((i - cx) d) / fx, y = ((j - cy) d) / fy, z = d;
* normal map: cross product of forward differences, a = V(i+1,j) - V(i,j),
  b = V(i,j+1) - V(i,j), n = (a x b) / |a x b|, zero where any of the three
  depths is invalid, on the last row/column, or where |a x b| = 0;
* intensity gradient (reference image only): central differences
  ((I(i+1) - I(i-1)) * 0.5), zero on the border.

Every operation is one IEEE float32 operation with round-to-nearest-even and no
contraction into fused multiply-adds; NumPy float32 ufuncs behave exactly so.
"""
from __future__ import annotations

import numpy as np

F = np.float32


def level0(depth, intensity):
    d = np.asarray(depth, dtype=np.float32)
    d = np.where(np.isfinite(d) & (d > F(0)), d, F(0)).astype(np.float32)
    i = np.asarray(intensity).astype(np.float32)
    return d, i


def downsample(D, I):
    """One 2x2 reduction step of depth (valid mean) and intensity (mean)."""
    H, W = D.shape
    h, w = H // 2, W // 2
    taps = [D[0:2 * h:2, 0:2 * w:2], D[0:2 * h:2, 1:2 * w:2], D[1:2 * h:2, 0:2 * w:2], D[1:2 * h:2, 1:2 * w:2]]
    s = np.zeros((h, w), np.float32)
    n = np.zeros((h, w), np.float32)
    for t in taps:
        v = t > F(0)
        s = np.where(v, s + t, s).astype(np.float32)
        n = np.where(v, n + F(1), n).astype(np.float32)
    Dn = np.where(n > F(0), s / np.where(n > F(0), n, F(1)), F(0)).astype(np.float32)
    a, b = I[0:2 * h:2, 0:2 * w:2], I[0:2 * h:2, 1:2 * w:2]
    c, d = I[1:2 * h:2, 0:2 * w:2], I[1:2 * h:2, 1:2 * w:2]
    In = (((a + b) + (c + d)) * F(0.25)).astype(np.float32)
    return Dn, In


def intrinsics(fx, fy, cx, cy, level):
    """Level-l intrinsics, computed in float64 and rounded once to float32."""
    s = 2.0 ** (-level)
    return (F(fx * s), F(fy * s), F((cx + 0.5) * s - 0.5), F((cy + 0.5) * s - 0.5))


def vertex_map(D, fx, fy, cx, cy):
    H, W = D.shape
    ii = np.arange(W, dtype=np.float32)[None, :].repeat(H, 0)
    jj = np.arange(H, dtype=np.float32)[:, None].repeat(W, 1)
    x = (((ii - F(cx)) * D) / F(fx)).astype(np.float32)
    y = (((jj - F(cy)) * D) / F(fy)).astype(np.float32)
    return np.stack([x, y, D.astype(np.float32)], axis=-1)


def normal_map(V, D):
    H, W = D.shape
    N = np.zeros((H, W, 3), np.float32)
    p = V[:-1, :-1]
    a = (V[:-1, 1:] - p).astype(np.float32)
    b = (V[1:, :-1] - p).astype(np.float32)
    cx_ = (a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1]).astype(np.float32)
    cy_ = (a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2]).astype(np.float32)
    cz_ = (a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]).astype(np.float32)
    L = np.sqrt(((cx_ * cx_ + cy_ * cy_) + cz_ * cz_).astype(np.float32)).astype(np.float32)
    ok = (D[:-1, :-1] > F(0)) & (D[:-1, 1:] > F(0)) & (D[1:, :-1] > F(0)) & (L > F(0))
    Ls = np.where(ok, L, F(1))
    for k, c in enumerate((cx_, cy_, cz_)):
        N[:-1, :-1, k] = np.where(ok, c / Ls, F(0))
    return N


def gradient_map(I):
    H, W = I.shape
    G = np.zeros((H, W, 2), np.float32)
    G[:, 1:-1, 0] = (I[:, 2:] - I[:, :-2]) * F(0.5)
    G[1:-1, :, 1] = (I[2:, :] - I[:-2, :]) * F(0.5)
    G[:, 0, :] = 0
    G[:, -1, :] = 0
    G[0, :, :] = 0
    G[-1, :, :] = 0
    return G


def build(depth, intensity, fx, fy, cx, cy, levels, with_gradient=False):
    """Pyramid as a list of dicts with keys D, I, V, N (and G), plus intrinsics K."""
    D, I = level0(depth, intensity)
    out = []
    for l in range(levels):
        if l > 0:
            D, I = downsample(D, I)
        K = intrinsics(fx, fy, cx, cy, l)
        V = vertex_map(D, *K)
        lev = {"D": D, "I": I, "V": V, "N": normal_map(V, D), "K": K}
        if with_gradient:
            lev["G"] = gradient_map(I)
        out.append(lev)
    return out
