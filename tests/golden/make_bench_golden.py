"""Writes the oracle values the benchmark reports its errors against
(tests/golden/bench_oracle.json), so that the benchmark itself never runs the
oracle.  Inputs come from synth/ on the CPU; every stored value is computed
here by oracle/ (float64 value layer, float32 mask layer); nothing here
touches the HIP library.

* "precision": the 160x120 frame pair (seed 1001), 2 levels.  Per level the
  visual normal equations (J^T J, J^T r, cost, inlier counts of the ICP and
  photometric terms, Section IV-B eqs. (2)-(3)) at a fixed linearisation point
  near the truth, with the float32 transforms the kernels take; and the pose
  the oracle's Gauss-Newton reaches over 4/4 iterations (Section IV-E).
* "stress_first_frame": the first tracked frame of session 0 of each
  resolution of the 256-session stress mix (synth.configs.session_sequence,
  seed 5000 + 1000 * class), 3 levels 10/5/4 iterations, RGB-D-inertial.

Usage (from the repository root): python tests/golden/make_bench_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import lie, track  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_oracle.json")
PAIR_SEED, PAIR_W, PAIR_H, PAIR_LEVELS, PAIR_ITERS = 1001, 160, 120, 2, (4, 4)
STRESS_RES = ((1920, 1080), (1280, 720), (640, 480), (320, 240))
STRESS_FRAMES = 8  # tracked frames per stress session (sequences of STRESS_FRAMES + 1 frames)


def state_json(x):
    return {k: [float(v) for v in np.asarray(x[k], dtype=np.float64)] for k in ("r", "q", "v", "bg", "ba")}


def linearisation_point(d, seed):
    """A pose pair near the truth (previous state 1e-3, current 2e-3 off) and a slightly moved model pose."""
    rng = np.random.default_rng(seed)
    x0 = lie.state_boxplus(d["x0"], np.r_[rng.normal(size=6) * 1e-3, np.zeros(9)])
    x1 = lie.state_boxplus(d["gt1"], np.r_[rng.normal(size=6) * 2e-3, np.zeros(9)])
    T_WM = np.eye(4)
    T_WM[:3, :3] = lie.exp_so3(rng.normal(size=3) * 1e-3)
    T_WM[:3, 3] = rng.normal(size=3) * 1e-3
    return x0, x1, T_WM


def precision_case():
    d = synth.configs.frame_pair(seed=PAIR_SEED, width=PAIR_W, height=PAIR_H)
    x0, x1, T_WM = linearisation_point(d, PAIR_SEED)
    params = track.default_params(levels=PAIR_LEVELS, iters=[1] * PAIR_LEVELS, mode="rgbdi")
    cur, ref = track.build_pyramids(d["depth"].numpy(), d["intensity"].numpy(), d["model_depth"].numpy(),
                                    d["model_intensity"].numpy(), d["camera"], PAIR_LEVELS)
    Ra, ta, Rb, tb = track.fp32_transforms(T_WM, x0, x1)
    levels = []
    for l in range(PAIR_LEVELS):
        vis = track.linearise_visual(cur[l], ref[l], T_WM, x0, x1, Ra, ta, Rb, tb, params)
        levels.append({f"{k}_{t}": (np.asarray(vis[f"{k}_{t}"], dtype=np.float64).ravel().tolist()
                                    if k in ("H", "b") else float(vis[f"{k}_{t}"]) if k == "cost"
                                    else int(vis[f"{k}_{t}"]))
                       for t in ("icp", "rgb") for k in ("H", "b", "cost", "n")})
    tp = track.default_params(levels=PAIR_LEVELS, iters=PAIR_ITERS, mode="rgbdi")
    o = track.track_frame(d["depth"].numpy(), d["intensity"].numpy(), d["model_depth"].numpy(),
                          d["model_intensity"].numpy(), d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"],
                          d["q_IW"], d["prior"], tp)
    assert o["status"] == "ok", o["status"]
    f32 = lambda a: [float(v) for v in np.asarray(a, dtype=np.float32).ravel()]  # noqa: E731
    return {"seed": PAIR_SEED, "width": PAIR_W, "height": PAIR_H, "levels": PAIR_LEVELS,
            "iters": list(PAIR_ITERS), "mode": "rgbdi",
            "linearize": {"x0": state_json(x0), "x1": state_json(x1), "T_WM": T_WM.ravel().tolist(),
                          "Ra": f32(Ra), "ta": f32(ta), "Rb": f32(Rb), "tb": f32(tb), "levels": levels},
            "track_x1": state_json(o["x1"])}


def stress_case(ci, w, h):
    seed = 5000 + 1000 * ci
    t = time.time()
    seq = synth.configs.session_sequence(seed, STRESS_FRAMES + 1, w, h, hole_rate=0.05, low_texture_rate=0.10)
    md, mi, T = synth.configs.model_view(seq, 1)
    t0, t1 = seq["times"][0], seq["times"][1]
    a, b = synth.configs.imu_window(seq["imu"]["t"], t0, t1)
    imu = {k: v[a:b] for k, v in seq["imu"].items()}
    params = track.default_params(levels=3, iters=(10, 5, 4), mode="rgbdi")
    o = track.track_frame(seq["depth"][1].numpy(), seq["intensity"][1].numpy(), md.numpy(), mi.numpy(), T,
                          seq["camera"], imu, t0, t1, seq["x0"], seq["q_IW"], seq["prior"], params)
    assert o["status"] == "ok", o["status"]
    print(f"stress {w}x{h} seed {seed}: {time.time() - t:.0f} s", flush=True)
    return {"width": w, "height": h, "seed": seed, "session": 0, "n_frames": STRESS_FRAMES + 1,
            "x1": state_json(o["x1"]), "q_IW": [float(v) for v in o["q_IW"]]}


def main():
    t = time.time()
    doc = {"description": "oracle values the benchmark compares with; written by tests/golden/make_bench_golden.py",
           "precision": precision_case()}
    print(f"precision case: {time.time() - t:.0f} s", flush=True)
    doc["stress_first_frame"] = [stress_case(ci, w, h) for ci, (w, h) in enumerate(STRESS_RES)]
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
