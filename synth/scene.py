"""Procedural RGB-D scene: three planes and four spheres with value-noise albedo.

Depth is the camera-frame z of the first hit (metres, FP32, 0 = invalid, valid
on [0.5, 4] m) with additive noise N(0, (k z^2)^2); intensity is the uint8
Lambertian shade ``round_half_even(255 * albedo * (0.3 + 0.7 max(0, n.l)))``.
The albedo is seeded 3-D value noise (integer lattice hash, smoothstep
trilinear interpolation, three octaves) mapped to [0.2, 0.9].

Written against torch so that the same generator runs on the CPU for tests and
on the GPU for the long sequences of the benchmark; it holds none of the
tracking method's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

_M32 = 0xFFFFFFFF
LIGHT_I = np.array([0.4, -0.3, 0.85]) / np.linalg.norm([0.4, -0.3, 0.85])
BACKGROUND_INTENSITY = 20


@dataclass
class Scene:
    planes: list = field(default_factory=list)   # (normal facing the room, offset d): n.x = d
    spheres: list = field(default_factory=list)  # (centre, radius)
    seed: int = 0


def make_scene(rng: np.random.Generator, seed: int, layout: str = "room") -> Scene:
    """Room corner (floor, back wall, left wall) with four spheres in view; with
    layout "wall", the back wall alone (a geometrically degenerate view: the
    same random draws, so the rest of a seeded sequence is unchanged)."""
    h = rng.uniform(1.1, 1.5)
    yb = rng.uniform(3.0, 3.6)
    xs = rng.uniform(1.6, 2.2)
    planes = [(np.array([0.0, 0.0, 1.0]), -h), (np.array([0.0, -1.0, 0.0]), -yb), (np.array([1.0, 0.0, 0.0]), -xs)]
    spheres = []
    for _ in range(4):
        r = rng.uniform(0.2, 0.5)
        c = np.array([rng.uniform(-1.2, 1.2), rng.uniform(1.5, 2.8), rng.uniform(-h + r, 0.5)])
        spheres.append((c, r))
    if layout == "wall":
        return Scene(planes=[planes[1]], spheres=[], seed=int(seed))
    if layout != "room":
        raise ValueError(f"unknown scene layout {layout!r}")
    return Scene(planes=planes, spheres=spheres, seed=int(seed))


def _hash01(ix, iy, iz, seed: int):
    h = (ix * 0x8DA6B343) ^ (iy * 0xD8163841) ^ (iz * 0xCB1AB31F) ^ (seed * 0x9E3779B1)
    h = h & _M32
    h = (((h >> 16) ^ h) * 0x45D9F3B) & _M32
    h = (((h >> 16) ^ h) * 0x45D9F3B) & _M32
    h = (h >> 16) ^ h
    return h.to(torch.float64) / 4294967296.0


def value_noise3(p: torch.Tensor, seed: int, octaves: int = 3, base_freq: float = 2.0) -> torch.Tensor:
    """Sum of octaves of smoothstep-trilinear lattice noise, normalised to [0, 1]."""
    total = torch.zeros(p.shape[:-1], dtype=torch.float64, device=p.device)
    amp, norm, freq = 1.0, 0.0, base_freq
    for o in range(octaves):
        q = p * freq
        q0 = torch.floor(q)
        f = q - q0
        w = f * f * (3.0 - 2.0 * f)
        i0 = q0.to(torch.int64)
        acc = torch.zeros_like(total)
        for dx in (0, 1):
            wx = w[..., 0] if dx else 1.0 - w[..., 0]
            for dy in (0, 1):
                wy = w[..., 1] if dy else 1.0 - w[..., 1]
                for dz in (0, 1):
                    wz = w[..., 2] if dz else 1.0 - w[..., 2]
                    acc = acc + wx * wy * wz * _hash01(i0[..., 0] + dx, i0[..., 1] + dy, i0[..., 2] + dz, seed * 8 + o)
        total = total + amp * acc
        norm += amp
        amp *= 0.5
        freq *= 2.0
    return total / norm


def value_noise2(x: torch.Tensor, y: torch.Tensor, seed: int, scale: float) -> torch.Tensor:
    p = torch.stack([x * scale, y * scale, torch.zeros_like(x)], dim=-1)
    return value_noise3(p, seed, octaves=2, base_freq=1.0)


def render(scene: Scene, R_IC, p_IC, W: int, H: int, fx: float, fy: float, cx: float, cy: float, *,
           depth_noise_k: float = 1e-3, generator: torch.Generator | None = None, low_texture: bool = False,
           hole_fraction: float = 0.0, hole_seed: int = 0, device="cpu", float_intensity: bool = False):
    """Ray-cast the scene from camera pose (R_IC, p_IC).

    Returns ``(depth float32 (H, W), intensity uint8 (H, W))`` on ``device``
    (intensity float64 before rounding with ``float_intensity``); depth noise
    is drawn from ``generator`` when it is given.
    """
    dev = torch.device(device)
    f64 = torch.float64
    R = torch.as_tensor(np.asarray(R_IC, dtype=np.float64), device=dev)
    o = torch.as_tensor(np.asarray(p_IC, dtype=np.float64), device=dev)
    jj, ii = torch.meshgrid(torch.arange(H, dtype=f64, device=dev), torch.arange(W, dtype=f64, device=dev),
                            indexing="ij")
    dC = torch.stack([(ii - cx) / fx, (jj - cy) / fy, torch.ones_like(ii)], dim=-1)  # z = 1: ray param == depth
    dI = dC @ R.T
    inf = torch.full((H, W), float("inf"), dtype=f64, device=dev)
    best = inf.clone()
    nrm = torch.zeros((H, W, 3), dtype=f64, device=dev)
    obj = torch.full((H, W), -1, dtype=torch.int64, device=dev)
    for k, (n, d) in enumerate(scene.planes):
        nt = torch.as_tensor(n, device=dev)
        den = dI @ nt
        s = (d - torch.dot(nt, o)) / den
        hit = (s > 1e-6) & (s < best) & (den.abs() > 1e-12)
        best = torch.where(hit, s, best)
        nrm = torch.where(hit[..., None], nt.expand(H, W, 3), nrm)
        obj = torch.where(hit, torch.full_like(obj, k), obj)
    for k, (c, r) in enumerate(scene.spheres):
        ct = torch.as_tensor(c, device=dev)
        oc = o - ct
        a = (dI * dI).sum(-1)
        b = dI @ oc
        c0 = torch.dot(oc, oc) - r * r
        disc = b * b - a * c0
        sq = torch.sqrt(torch.clamp(disc, min=0.0))
        s = (-b - sq) / a
        hit = (disc > 0) & (s > 1e-6) & (s < best)
        best = torch.where(hit, s, best)
        pts = o + s[..., None] * dI
        nrm = torch.where(hit[..., None], (pts - ct) / r, nrm)
        obj = torch.where(hit, torch.full_like(obj, 16 + k), obj)
    found = torch.isfinite(best)
    s = torch.where(found, best, torch.zeros_like(best))
    pts = o + s[..., None] * dI
    alb = torch.zeros((H, W), dtype=f64, device=dev)
    for k in torch.unique(obj[found]).tolist():
        m = obj == k
        alb = torch.where(m, 0.2 + 0.7 * value_noise3(pts, scene.seed * 64 + int(k)), alb)
    if low_texture:
        alb = 0.55 + 0.1 * (alb - 0.55)
    light = torch.as_tensor(LIGHT_I, device=dev)
    shade = 0.3 + 0.7 * torch.clamp(nrm @ light, min=0.0)
    inten = 255.0 * alb * shade
    if not float_intensity:
        inten = torch.round(inten).clamp(0, 255)
    inten = torch.where(found, inten, torch.full_like(inten, float(BACKGROUND_INTENSITY)))
    if not float_intensity:
        inten = inten.to(torch.uint8)
    valid = found & (s >= 0.5) & (s <= 4.0)
    z = torch.where(valid, s, torch.zeros_like(s))
    if depth_noise_k > 0 and generator is not None:
        noise = torch.randn((H, W), generator=generator, dtype=f64, device=generator.device).to(dev)
        z = torch.where(valid, z + noise * depth_noise_k * z * z, z)
    if hole_fraction > 0:
        hv = value_noise2(ii, jj, hole_seed, scale=1.0 / 24.0)
        thr = torch.quantile(hv.flatten().float(), hole_fraction).to(f64)
        z = torch.where(hv < thr, torch.zeros_like(z), z)
    return z.to(torch.float32), inten
