"""Helpers for the GPU parity tests (inputs and comparisons only)."""
import contextlib

import numpy as np

import paper_2207_10940_amd as P
import synth
from oracle import lie


def cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda")


@contextlib.contextmanager
def session(W, H, levels, iters, mode="rgbdi", x0=None, q_IW=None, prior=None, budget=0, **kw):
    ctx = P.Context(0, budget)
    cam = synth.configs.camera_for(W, H)
    tp = P.track_params(levels=levels, iters=iters, mode=mode, **kw)
    if x0 is None:
        x0 = {"r": np.zeros(3), "q": np.array([1.0, 0, 0, 0]), "v": np.zeros(3), "bg": np.zeros(3), "ba": np.zeros(3)}
    if q_IW is None:
        q_IW = np.array([1.0, 0, 0, 0])
    if prior is None and mode != "rgbd":
        prior = synth.configs.initial_prior(x0, q_IW)
    s = P.Session(ctx, cam, tp, P.imu_params(), x0, q_IW, prior)
    try:
        yield s
    finally:
        s.close()
        ctx.close()


def rel_fro(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def jtr_scale(terms, cols, dim):
    """| |J|^T |w e| |: the normwise scale of a cancelling J^T r sum."""
    s = np.zeros(dim)
    if terms["J"].shape[0]:
        s[cols] = np.abs(terms["J"]).T @ np.abs(terms["w"] * terms["e"])
    return np.linalg.norm(s)


def pose_err(xa, xb):
    return np.linalg.norm(xa["r"] - xb["r"]), np.linalg.norm(lie.quat_boxminus(xa["q"], xb["q"]))
