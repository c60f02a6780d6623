"""Writes the expected per-frame states of the 640x480 sequence workload.

The oracle (float64 Gauss-Newton over the paper's cost, Section IV) tracks
every frame of the seeded 300-frame sequence (3 levels, 10/5/4 iterations,
RGB-D-inertial), chained: each frame starts from the oracle's own previous
estimate and marginal prior.  Inputs come from synth/ only (CPU rendering);
nothing here touches the HIP library.

Usage (from the repository root): python tests/golden/make_sequence_golden.py [n_frames]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import track  # noqa: E402

SEED, WIDTH, HEIGHT, LEVELS, ITERS = 2001, 640, 480, 3, (10, 5, 4)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sequence_640x480_rgbdi.json")


def frame_inputs(seq, j):
    md, mi, T = synth.configs.model_view(seq, j)
    t0, t1 = seq["times"][j - 1], seq["times"][j]
    a, b = synth.configs.imu_window(seq["imu"]["t"], t0, t1)
    imu = {k: v[a:b] for k, v in seq["imu"].items()}
    return md.numpy(), mi.numpy(), T, seq["depth"][j].numpy(), seq["intensity"][j].numpy(), imu, t0, t1


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 300
    t = time.time()
    seq = synth.configs.sequence(seed=SEED, n_frames=n, width=WIDTH, height=HEIGHT)
    print(f"inputs {time.time() - t:.0f} s", flush=True)
    params = track.default_params(levels=LEVELS, iters=ITERS, mode="rgbdi")
    x0, q, prior = seq["x0"], seq["q_IW"], seq["prior"]
    frames = []
    for j in range(1, n):
        md, mi, T, d, i, imu, t0, t1 = frame_inputs(seq, j)
        o = track.track_frame(d, i, md, mi, T, seq["camera"], imu, t0, t1, x0, q, prior, params)
        assert o["status"] == "ok", (j, o["status"])
        x0, q, prior = o["x1"], o["q_IW"], o["prior"]
        frames.append({"frame": j, "x1": {k: [float(v) for v in o["x1"][k]] for k in ("r", "q", "v", "bg", "ba")},
                       "q_IW": [float(v) for v in o["q_IW"]]})
        if j % 10 == 0:
            print(f"frame {j} ({time.time() - t:.0f} s)", flush=True)
    doc = {"description": "oracle states of the 640x480 RGB-D-inertial sequence (3 levels, 10/5/4 iterations), "
                          "chained frame by frame; written by tests/golden/make_sequence_golden.py",
           "seed": SEED, "width": WIDTH, "height": HEIGHT, "levels": LEVELS, "iters": list(ITERS),
           "n_frames": n, "frames": frames}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {OUT}: {len(frames)} frames", flush=True)


if __name__ == "__main__":
    main()
