"""Parity at the serving workloads' large resolutions (1280x720, 1920x1080),
where the residual pass runs 4 pixels per thread and launches its largest
grids: the association masks bit-exact and the normal equations against the
float64 oracle for every pyramid level; a tracked frame pair within
1e-6 m / 1e-6 rad of the oracle, tracked alone and inside a batched step of
mixed resolutions."""
import numpy as np
import pytest

import paper_2207_10940_amd as P
import synth
from oracle import lie, track
from tests.gpu_common import cuda, jtr_scale, pose_err, rel_fro, session

pytestmark = pytest.mark.gpu


def _pair(seed, W, H):
    d = synth.configs.frame_pair(seed=seed, width=W, height=H, device="cuda")
    for k in ("depth", "intensity", "model_depth", "model_intensity"):
        d[k] = d[k].contiguous()
    return d


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("W,H,seed", [(1280, 720, 4101), (1920, 1080, 4102)])
def test_linearize_large(W, H, seed):
    import torch
    d = _pair(seed, W, H)
    rng = np.random.default_rng(seed)
    x0 = lie.state_boxplus(d["x0"], np.r_[rng.normal(size=6) * 1e-3, np.zeros(9)])
    x1 = lie.state_boxplus(d["gt1"], np.r_[rng.normal(size=6) * 2e-3, np.zeros(9)])
    T_WM = d["T_WM"]
    cam = d["camera"]
    levels = 3
    params = track.default_params(levels=levels, iters=[1] * levels, mode="rgbdi")
    cur, ref = track.build_pyramids(_np(d["depth"]), _np(d["intensity"]), _np(d["model_depth"]),
                                    _np(d["model_intensity"]), cam, levels)
    Ra, ta, Rb, tb = track.fp32_transforms(T_WM, x0, x1)
    print(f"linearize {W}x{H}", flush=True)
    with session(W, H, levels, [1] * levels) as s:
        s.set_model(d["model_depth"], d["model_intensity"], T_WM)
        s.build_pyramid(P.PYR_CURRENT, d["depth"], d["intensity"])
        for l in range(levels):
            vis = track.linearise_visual(cur[l], ref[l], T_WM, x0, x1, Ra, ta, Rb, tb, params)
            mask = torch.zeros((H >> l, W >> l), dtype=torch.uint8, device="cuda")
            g = s.linearize(l, Ra, ta, Rb, tb, x0, x1, mask=mask)
            m = mask.cpu().numpy()
            assert np.array_equal((m & 1) != 0, vis["mask_icp"]), l
            assert np.array_equal((m & 2) != 0, vis["mask_rgb"]), l
            assert g["n_icp"] == vis["n_icp"] and g["n_rgb"] == vis["n_rgb"]
            for term, cols in (("icp", np.r_[6:12]), ("rgb", np.r_[0:12])):
                eH = rel_fro(g["H_" + term], vis["H_" + term])
                eb = np.linalg.norm(g["b_" + term] - vis["b_" + term]) / jtr_scale(vis[term], cols, 12)
                eb_plain = rel_fro(g["b_" + term], vis["b_" + term])
                print(f"  level {l} {term}: n {g['n_' + term]}  JtJ {eH:.2e}  Jtr {eb:.2e} (plain {eb_plain:.2e})",
                      flush=True)
                assert eH < 1e-5 and eb < 1e-5, (l, term, eH, eb)


SCHED = (2, 2, 2)


def _oracle_pair(d, mode="rgbdi"):
    params = track.default_params(levels=len(SCHED), iters=SCHED, mode=mode)
    return track.track_frame(_np(d["depth"]), _np(d["intensity"]), _np(d["model_depth"]), _np(d["model_intensity"]),
                             d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"], d["q_IW"], d["prior"],
                             params)


def _frame(d):
    return {"depth": d["depth"], "intensity": d["intensity"], "model_depth": d["model_depth"],
            "model_intensity": d["model_intensity"], "T_WM": d["T_WM"], "imu": d["imu"], "t0": d["t0"], "t1": d["t1"]}


def test_track_pair_large_alone_and_batched():
    import torch
    pairs = [_pair(4201, 1920, 1080), _pair(4202, 1280, 720), _pair(4203, 640, 480)]
    oracle = []
    for d in pairs:
        print(f"oracle {d['camera'].width}x{d['camera'].height}", flush=True)
        oracle.append(_oracle_pair(d))
    stream = torch.cuda.current_stream()
    ctx = P.Context(0)
    try:
        def open_s(d):
            tp = P.track_params(levels=len(SCHED), iters=SCHED, mode="rgbdi")
            return P.Session(ctx, d["camera"], tp, P.imu_params(), d["x0"], d["q_IW"], d["prior"])
        alone = []
        for d in pairs:
            s = open_s(d)
            alone.append(s.track_frame_sync(_frame(d)))
            s.close()
        sess = [open_s(d) for d in pairs]
        batch = P.Batch(ctx, len(pairs))
        batch.track(sess, [_frame(d) for d in pairs], stream)
        batched = batch.results()
        batch.close()
        for s in sess:
            s.close()
    finally:
        ctx.close()
    for d, o, a, b in zip(pairs, oracle, alone, batched):
        name = f"{d['camera'].width}x{d['camera'].height}"
        assert o["status"] == "ok" and a["status"] == 0 and b["status"] == 0, name
        for what, g in (("alone", a), ("batched", b)):
            dr, da = pose_err(g["x1"], o["x1"])
            print(f"{name} {what}: |dr| {dr:.2e} m |da| {da:.2e} rad", flush=True)
            assert dr < 1e-6 and da < 1e-6, (name, what, dr, da)
        for f in ("r", "q", "v", "bg", "ba"):  # alone and batched: the same arithmetic
            assert np.array_equal(a["x1"][f], b["x1"][f]), (name, f)
