"""Surfel map: fusion of tracked frames and model-view prediction (TEST INFRASTRUCTURE).

The paper tracks each frame against a view predicted from its fused dense
surfel map and fuses the frame into that map with the estimated pose
(Section III, the mapping step of Section V); it keeps ElasticFusion's map and
states neither the fusion rule nor the rendering.  Readings taken here (all
values float32, one IEEE rounding per operation, no fused multiply-adds; NumPy
float32 ufuncs behave exactly so, and the device kernels perform the same
operations in the same order):

* a surfel holds a world position p, a unit world normal n, an intensity I,
  a radius r and a confidence c;
* transforms are given as float32 (D = R - I, t), each rounded once from its
  float64 value: camera to world (R_WC - I, r_WC) and world to camera
  (R_WC^T - I, -R_WC^T r_WC, the latter summed as -((R00 r0 + R10 r1) + R20 r2)
  per component in float64); a point maps as q = p + (((D00 x + D01 y) + D02 z)
  + t0) per component and a direction as n' = n + ((D00 x + D01 y) + D02 z);
* projection as in the tracker's association: inv = 1/q_z,
  u = ((fx q_x) inv) + cx, rounded half-even, inside the image as a float
  compare;
* index map (fusion): every surfel in front of the camera marks the pixel of
  its projected centre with the key (bits(q_z) << 32) | index; the smallest
  key wins (the nearest surfel, then the lowest index);
* fusion of pixel u with a valid depth and normal: the measurement
  p_m = camera-to-world(V(u)) from the frame's level-0 vertex, n_m = the
  rotated normal of its parent pixel (u >> 1) at level 1 of the frame's
  pyramid (level 0 for a one-level pyramid: forward differences of the raw
  depth are dominated by its noise at full resolution, while the level-1
  normal averages 2x2 depths over twice the baseline), I_m = I(u), weight
  alpha = 1 / (1 + g2) with g2 = ((i - cx)^2 + (j - cy)^2) / (cx^2 + cy^2)
  (down-weighting the image periphery), radius
  r_m = (z sqrt2) / (fx max(|N_z|, 0.5)).  It updates the surfel of its index
  map cell when |z_s - z| <= dist and n_s . n_m >= cos_min: c' = c + alpha,
  p' = ((c p) + (alpha p_m)) / c' per component, n' = the normalised
  (c n) + (alpha n_m), I' = ((c I) + (alpha I_m)) / c', r' = min(r, r_m).
  Every surfel marks one cell, so it is updated by at most one pixel.  A valid
  pixel that updates no surfel becomes a new surfel (p_m, n_m, I_m, r_m,
  alpha) unless one of the 8 neighbouring cells holds a surfel within dist of
  its depth (the surface is already mapped there: a moving camera leaves
  cells between projected surfel centres empty); new surfels are appended in
  pixel order after the existing ones while the capacity lasts;
* prediction (splat rendering) at the model pose: each surfel in front of the
  camera covers the pixels within h = min(ceil((r fx) / q_z), HMAX) of its
  rounded centre; a pixel's ray d = ((i - cx) / fx, (j - cy) / fy, 1) meets the
  surfel's plane at depth t = (n_c . q) / (n_c . d) (dot products summed as
  (x + y) + z, n_c the camera-frame normal, |n_c . d| > 1e-6); the pixel is
  covered when t > 0 and |t d - q|^2 <= r^2.  Of the surfels covering a
  pixel, those within `band` metres of the nearest one (t <= t_min + band)
  form its front surface, and the one whose projected centre (u, v) is
  closest to the pixel, d2 = (i - u)^2 + (j - v)^2, wins (then the lowest
  index): taking the nearest depth alone would pick, of several noisy
  observations of one surface, the one nearest the camera.  The rendered
  depth is the winner's t, the intensity the winner's, rounded half-even and
  clamped to [0, 255], and the normal the winner's camera-frame normal n_c
  (zero where no surfel covers the pixel).  The model view's level-0 normals
  are these surfel normals, averaged over the frames fused into each surfel,
  rather than forward differences of the rendered depth, which carry the
  depth noise of the frames the surfels came from.
"""
from __future__ import annotations

import numpy as np

F = np.float32
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
HMAX = 4
FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "inten", "radius", "conf")
SQRT2 = F(1.41421356)


def fusion_normals(levels: list) -> np.ndarray:
    """(H, W, 3) normals the fusion uses: level 1's normal of each level-0 pixel's parent (u >> 1), or
    level 0's own for a one-level pyramid (levels: the frame's pyramid, oracle.pyramid.build)."""
    if len(levels) < 2:
        return levels[0]["N"]
    N1 = levels[1]["N"]
    H, W = levels[0]["V"].shape[:2]
    jj, ii = np.meshgrid(np.arange(H) >> 1, np.arange(W) >> 1, indexing="ij")
    return N1[jj, ii]


def empty_map() -> dict:
    return {k: np.zeros(0, dtype=np.float32) for k in FIELDS}


def transforms(T_WC):
    """(D_wc, t_wc, D_cw, t_cw): float32 camera-to-world and world-to-camera transforms of the float64
    pose T_WC (4x4), as the header describes."""
    T = np.asarray(T_WC, dtype=np.float64)
    R, r = T[:3, :3], T[:3, 3]
    D_wc = (R - np.eye(3)).astype(np.float32)
    t_wc = r.astype(np.float32)
    D_cw = (R.T - np.eye(3)).astype(np.float32)
    t_cw = np.array([-((float(R[0, i]) * float(r[0]) + float(R[1, i]) * float(r[1])) + float(R[2, i]) * float(r[2]))
                     for i in range(3)], dtype=np.float64).astype(np.float32)
    return D_wc, t_wc, D_cw, t_cw


def _xform(D, t, x, y, z):
    p = (x, y, z)
    return [(p[k] + (((D[k, 0] * x + D[k, 1] * y) + D[k, 2] * z) + t[k])).astype(np.float32) for k in range(3)]


def _rotate(D, x, y, z):
    p = (x, y, z)
    return [(p[k] + ((D[k, 0] * x + D[k, 1] * y) + D[k, 2] * z)).astype(np.float32) for k in range(3)]


def _project(qx, qy, qz, cam):
    fx, fy, cx, cy = F(cam[0]), F(cam[1]), F(cam[2]), F(cam[3])
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        inv = (F(1) / qz).astype(np.float32)
        u = ((fx * qx) * inv + cx).astype(np.float32)
        v = ((fy * qy) * inv + cy).astype(np.float32)
    return u, v


def _keys(z, idx):
    return (z.astype(np.float32).view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)


def index_map(m: dict, D_cw, t_cw, cam, W: int, H: int) -> np.ndarray:
    """(H, W) uint64 keys of the nearest surfel whose centre projects to each pixel (EMPTY if none)."""
    out = np.full(H * W, EMPTY, dtype=np.uint64)
    n = len(m["px"])
    if n == 0:
        return out.reshape(H, W)
    qx, qy, qz = _xform(D_cw, t_cw, m["px"], m["py"], m["pz"])
    u, v = _project(qx, qy, qz, cam)
    ur, vr = np.rint(u), np.rint(v)
    with np.errstate(invalid="ignore"):
        ok = (qz > 0) & (ur >= 0) & (ur <= F(W - 1)) & (vr >= 0) & (vr <= F(H - 1))
    s = np.nonzero(ok)[0]
    pix = vr[s].astype(np.int64) * W + ur[s].astype(np.int64)
    np.minimum.at(out, pix, _keys(qz[s], s))
    return out.reshape(H, W)


def fuse(m: dict, V, N, I16, T_WC, cam, W: int, H: int, capacity: int, dist=0.05, cos_min=0.8):
    """The map after fusing one frame: V (H, W, 3) camera-frame vertices of the frame's level 0, N its
    fusion normals (fusion_normals), I16 its fixed-point intensity plane (value * 64, uint16), T_WC the
    frame's pose,
    cam (fx, fy, cx, cy).  Returns (new map, number of new surfels dropped for lack of capacity)."""
    D_wc, t_wc, D_cw, t_cw = transforms(T_WC)
    key = index_map(m, D_cw, t_cw, cam, W, H).ravel()
    Vx, Vy, Vz = (np.asarray(V[..., k], dtype=np.float32).ravel() for k in range(3))
    Nx, Ny, Nz = (np.asarray(N[..., k], dtype=np.float32).ravel() for k in range(3))
    Im = (np.asarray(I16).ravel().astype(np.float32) * F(1.0 / 64.0)).astype(np.float32)
    valid = (Vz > 0) & ((Nx != 0) | (Ny != 0) | (Nz != 0))
    pmx, pmy, pmz = _xform(D_wc, t_wc, Vx, Vy, Vz)
    nmx, nmy, nmz = _rotate(D_wc, Nx, Ny, Nz)
    fx, cx, cy = F(cam[0]), F(cam[2]), F(cam[3])
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    dx = (ii.ravel().astype(np.float32) - cx).astype(np.float32)
    dy = (jj.ravel().astype(np.float32) - cy).astype(np.float32)
    g2 = ((dx * dx + dy * dy) / (cx * cx + cy * cy)).astype(np.float32)
    alpha = (F(1) / (F(1) + g2)).astype(np.float32)
    rm = ((Vz * SQRT2) / (fx * np.maximum(np.abs(Nz), F(0.5)))).astype(np.float32)
    out = {k: m[k].copy() for k in FIELDS}
    has = key != EMPTY
    s_idx = (key & np.uint64(0xFFFFFFFF)).astype(np.int64)
    zs = (key >> np.uint64(32)).astype(np.uint32).view(np.float32)
    assoc = valid & has
    a = np.nonzero(assoc)[0]
    sa = s_idx[a]
    ndot = ((m["nx"][sa] * nmx[a] + m["ny"][sa] * nmy[a]) + m["nz"][sa] * nmz[a]).astype(np.float32)
    ok = (np.abs((zs[a] - Vz[a]).astype(np.float32)) <= F(dist)) & (ndot >= F(cos_min))
    assoc[a[~ok]] = False
    a, sa = a[ok], sa[ok]
    al = alpha[a]
    c = m["conf"][sa]
    c1 = (c + al).astype(np.float32)
    for f, meas in (("px", pmx), ("py", pmy), ("pz", pmz), ("inten", Im)):
        out[f][sa] = (((c * m[f][sa]) + (al * meas[a])) / c1).astype(np.float32)
    nn = [((c * m[f][sa]) + (al * meas[a])).astype(np.float32) for f, meas in (("nx", nmx), ("ny", nmy), ("nz", nmz))]
    ln = np.sqrt(((nn[0] * nn[0] + nn[1] * nn[1]) + nn[2] * nn[2]).astype(np.float32)).astype(np.float32)
    pos = ln > 0
    for k, f in enumerate(("nx", "ny", "nz")):
        out[f][sa[pos]] = (nn[k][pos] / ln[pos]).astype(np.float32)
    out["radius"][sa] = np.minimum(m["radius"][sa], rm[a])
    out["conf"][sa] = c1
    covered = np.zeros(H * W, dtype=bool)
    zk = (key >> np.uint64(32)).astype(np.uint32).view(np.float32)
    jj2, ii2 = jj.ravel(), ii.ravel()
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            i2, j2 = ii2 + di, jj2 + dj
            inimg = (i2 >= 0) & (i2 < W) & (j2 >= 0) & (j2 < H)
            q = np.where(inimg, j2 * W + i2, 0)
            near = inimg & (key[q] != EMPTY) & (np.abs((zk[q] - Vz).astype(np.float32)) <= F(dist))
            covered |= near
    new = np.nonzero(valid & ~assoc & ~covered)[0]
    room = max(0, capacity - len(m["px"]))
    dropped = max(0, len(new) - room)
    new = new[:room]
    for f, meas in (("px", pmx), ("py", pmy), ("pz", pmz), ("nx", nmx), ("ny", nmy), ("nz", nmz), ("inten", Im),
                    ("radius", rm), ("conf", alpha)):
        out[f] = np.concatenate([out[f], meas[new].astype(np.float32)])
    return out, dropped


def render(m: dict, T_WM, cam, W: int, H: int, band=0.03, with_normals=False):
    """Predicted model view at pose T_WM: (depth float32 (H, W), intensity uint8 (H, W)), and with
    with_normals the (H, W, 3) float32 camera-frame normals as a third element."""
    _, _, D_cw, t_cw = transforms(T_WM)
    npx = H * W
    zmin = np.full(npx, np.inf, dtype=np.float32)
    best = np.full(npx, EMPTY, dtype=np.uint64)
    depth = np.zeros(npx, dtype=np.float32)
    inten = np.zeros(npx, dtype=np.uint8)
    nrm = np.zeros((npx, 3), dtype=np.float32)
    if len(m["px"]) == 0:
        out = (depth.reshape(H, W), inten.reshape(H, W))
        return out + (nrm.reshape(H, W, 3),) if with_normals else out
    cands = list(_splat_candidates(m, D_cw, t_cw, cam, W, H))
    for pix, s, t, d2c in cands:  # pass 1: the nearest depth of each pixel
        np.minimum.at(zmin, pix, t)
    bandf = F(band)
    for pix, s, t, d2c in cands:  # pass 2: the front surface's most central surfel
        front = t <= (zmin[pix] + bandf).astype(np.float32)
        np.minimum.at(best, pix[front], _keys(d2c[front], s[front]))
    for pix, s, t, d2c in cands:  # the winner's own depth
        win = best[pix] == _keys(d2c, s)
        depth[pix[win]] = t[win]
    has = best != EMPTY
    si = (best[has] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    inten[has] = np.clip(np.rint(m["inten"][si]), F(0), F(255)).astype(np.uint8)
    if not with_normals:
        return depth.reshape(H, W), inten.reshape(H, W)
    ncx, ncy, ncz = _rotate(D_cw, m["nx"][si], m["ny"][si], m["nz"][si])
    nrm[has] = np.stack([ncx, ncy, ncz], axis=1)
    return depth.reshape(H, W), inten.reshape(H, W), nrm.reshape(H, W, 3)


def _splat_candidates(m, D_cw, t_cw, cam, W, H):
    """(pixel, surfel, depth t, squared centre distance) of every pixel a surfel's disk covers, in
    batches by footprint offset."""
    fx, fy, cx, cy = F(cam[0]), F(cam[1]), F(cam[2]), F(cam[3])
    qx, qy, qz = _xform(D_cw, t_cw, m["px"], m["py"], m["pz"])
    ncx, ncy, ncz = _rotate(D_cw, m["nx"], m["ny"], m["nz"])
    u, v = _project(qx, qy, qz, cam)
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        front = qz > 0
        u0 = np.where(front, np.rint(u), F(-1e9)).astype(np.float32)
        v0 = np.where(front, np.rint(v), F(-1e9)).astype(np.float32)
        rp = ((m["radius"] * fx) / qz).astype(np.float32)
        h = np.where(front, np.minimum(np.ceil(rp), F(HMAX)), F(-1)).astype(np.float32)
    r2 = (m["radius"] * m["radius"]).astype(np.float32)
    # centres far outside the image cover nothing: keep the integer pixel arithmetic in range
    inb = front & (u0 >= F(-HMAX)) & (u0 <= F(W - 1 + HMAX)) & (v0 >= F(-HMAX)) & (v0 <= F(H - 1 + HMAX))
    s_all = np.nonzero(inb)[0]
    ui, vi, hi = u0[s_all].astype(np.int64), v0[s_all].astype(np.int64), h[s_all].astype(np.int64)
    for dv in range(-HMAX, HMAX + 1):
        for du in range(-HMAX, HMAX + 1):
            sel = (np.abs(du) <= hi) & (np.abs(dv) <= hi)
            i, j = ui[sel] + du, vi[sel] + dv
            inimg = (i >= 0) & (i < W) & (j >= 0) & (j < H)
            s = s_all[sel][inimg]
            i, j = i[inimg], j[inimg]
            fi, fj = i.astype(np.float32), j.astype(np.float32)
            dxr = ((fi - cx) / fx).astype(np.float32)
            dyr = ((fj - cy) / fy).astype(np.float32)
            den = ((ncx[s] * dxr + ncy[s] * dyr) + ncz[s]).astype(np.float32)
            num = ((ncx[s] * qx[s] + ncy[s] * qy[s]) + ncz[s] * qz[s]).astype(np.float32)
            with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
                t = (num / den).astype(np.float32)
                ex = ((t * dxr) - qx[s]).astype(np.float32)
                ey = ((t * dyr) - qy[s]).astype(np.float32)
                ez = (t - qz[s]).astype(np.float32)
                d2 = ((ex * ex + ey * ey) + ez * ez).astype(np.float32)
                hit = (np.abs(den) > F(1e-6)) & (t > 0) & (d2 <= r2[s])
            eu = (fi - u[s]).astype(np.float32)
            ev = (fj - v[s]).astype(np.float32)
            d2c = (eu * eu + ev * ev).astype(np.float32)
            yield (j[hit] * W + i[hit]), s[hit], t[hit], d2c[hit]
