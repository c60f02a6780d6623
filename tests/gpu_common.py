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


def seq_frame(seq, j):
    """Inputs of tracking frame j of a synthetic sequence (frame dict of the batch and server APIs)."""
    md, mi, T = synth.configs.model_view(seq, j)
    t0, t1 = seq["times"][j - 1], seq["times"][j]
    a, b = synth.configs.imu_window(seq["imu"]["t"], t0, t1)
    imu = {k: v[a:b] for k, v in seq["imu"].items()}
    return {"depth": seq["depth"][j].contiguous(), "intensity": seq["intensity"][j].contiguous(),
            "model_depth": md.contiguous(), "model_intensity": mi.contiguous(), "T_WM": T,
            "imu": imu, "t0": t0, "t1": t1}


def open_seq_session(ctx, seq, mode, iters=(4, 3, 2), jac="fp32"):
    tp = P.track_params(levels=len(iters), iters=iters, mode=mode, jac=jac)
    prior = seq["prior"] if mode != "rgbd" else None
    return P.Session(ctx, seq["camera"], tp, P.imu_params(), seq["x0"], seq["q_IW"], prior)


def same_result(a, b, what):
    """Bit-for-bit equality of two result dicts."""
    assert a["status"] == b["status"] == 0, what
    for k in ("x0", "x1"):
        for f in ("r", "q", "v", "bg", "ba"):
            assert np.array_equal(a[k][f], b[k][f]), (what, k, f, a[k][f] - b[k][f])
    assert np.array_equal(a["q_IW"], b["q_IW"]), what
    assert a["health"] == b["health"] and a["tracking_lost"] == b["tracking_lost"], what
    assert a["n_icp"] == b["n_icp"] and a["n_rgb"] == b["n_rgb"], what
    for f in ("cost_icp", "cost_rgb", "cost_imu", "last_step_norm"):
        assert a[f] == b[f], (what, f)
    assert np.array_equal(a["prior"]["H"], b["prior"]["H"]) and np.array_equal(a["prior"]["b"], b["prior"]["b"]), what
