"""Tile-shape autotuner through the C ABI: it times the residual pass per
resolution, level and format, and sessions opened afterwards track with the
chosen shapes to the same oracle bar as with the default shapes."""
import numpy as np
import pytest

import paper_2207_10940_amd as P
import synth
from oracle import track
from tests.gpu_common import cuda, pose_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("jac", ["fp32", "bf16"])
def test_autotune_then_track_pair(jac):
    W, H, levels, iters = 160, 120, 2, (4, 4)
    d = synth.configs.frame_pair(seed=1001, width=W, height=H)
    ctx = P.Context(0)
    tuned = ctx.autotune([d["camera"], synth.configs.camera_for(320, 240)], levels=levels, jac=jac)
    print(tuned, flush=True)
    assert len(tuned) == 2 * levels
    assert all(e["ppt"] in (1, 2, 4) and e["us"] > 0 for e in tuned)
    assert ctx.used_bytes() == 0  # temporary memory released
    params = track.default_params(levels=levels, iters=iters, mode="rgbdi")
    o = track.track_frame(d["depth"].numpy(), d["intensity"].numpy(), d["model_depth"].numpy(),
                          d["model_intensity"].numpy(), d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"],
                          d["q_IW"], d["prior"], params)
    tp = P.track_params(levels=levels, iters=iters, mode="rgbdi", jac=jac)
    s = P.Session(ctx, d["camera"], tp, P.imu_params(), d["x0"], d["q_IW"], d["prior"])
    s.set_model(cuda(d["model_depth"].numpy()), cuda(d["model_intensity"].numpy()), d["T_WM"])
    s.track_frame(cuda(d["depth"].numpy()), cuda(d["intensity"].numpy()), d["imu"], d["t0"], d["t1"])
    g = s.result()
    s.close()
    ctx.close()
    dr, da = pose_err(g["x1"], o["x1"])
    bar = 1e-6 if jac == "fp32" else 1e-4
    assert g["status"] == 0 and dr < bar and da < bar, (dr, da)


def test_autotune_rejects_bad_input():
    ctx = P.Context(0)
    with pytest.raises(P.DslamError):
        ctx.autotune([synth.configs.camera_for(160, 120)], levels=5)
    with pytest.raises(P.DslamError):
        ctx.autotune([synth.configs.camera_for(162, 120)], levels=3)  # width not divisible by 4
    ctx.close()
