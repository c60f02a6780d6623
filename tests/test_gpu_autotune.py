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
    assert all(e["ppt"] in (1, 2, 4) and e["xcd_banded"] in (0, 1) and e["us"] > 0 for e in tuned)
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


@pytest.mark.parametrize("ppt", [1, 2, 4])
def test_tile_order_changes_no_result(ppt):
    """Launch shapes pinned with dslam_context_set_tune: the XCD-banded tile order gives the same results,
    bit for bit, as the round-robin order (each tile's sums land in the same place), alone and batched,
    on a ragged 200x152 sequence; the pose meets the oracle bar."""
    import torch
    from tests.gpu_common import open_seq_session, same_result, seq_frame
    seq = synth.configs.sequence(seed=3301, n_frames=4, width=200, height=152, device="cuda")
    stream = torch.cuda.current_stream()
    ctx = P.Context(0)
    out = {}
    for banded in (0, 1):
        ctx.set_tune([{"width": 200, "height": 152, "level": l, "jac_format": "fp32", "ppt": ppt,
                       "xcd_banded": banded} for l in range(3)])
        s = open_seq_session(ctx, seq, "rgbdi")
        out[banded] = [s.track_frame_sync(seq_frame(seq, j), stream) for j in range(1, 4)]
        s.close()
    for j in range(3):
        same_result(out[1][j], out[0][j], f"ppt {ppt} frame {j + 1}")
    # batched: a round-robin and a banded session in one step, in each of the batch's tile orders
    batch = P.Batch(ctx, 2)
    for order in (-1, 0, 1):
        ctx.set_tune([{"width": 200, "height": 152, "level": l, "jac_format": "fp32", "ppt": ppt, "xcd_banded": 0}
                      for l in range(3)])
        a = open_seq_session(ctx, seq, "rgbdi")
        ctx.set_tune([{"width": 200, "height": 152, "level": l, "jac_format": "fp32", "ppt": ppt, "xcd_banded": 1}
                      for l in range(3)])
        b = open_seq_session(ctx, seq, "rgbdi")
        batch.set_tile_order(order)
        batch.track([b, a], [seq_frame(seq, 1), seq_frame(seq, 1)], stream)
        rb, ra = batch.results()
        same_result(ra, out[0][0], f"batched round-robin session, batch order {order}")
        same_result(rb, out[0][0], f"batched banded session, batch order {order}")
        a.close()
        b.close()
    with pytest.raises(P.DslamError):
        batch.set_tile_order(2)
    batch.close()
    with pytest.raises(P.DslamError):
        ctx.set_tune([{"width": 200, "height": 152, "level": 0, "jac_format": "fp32", "ppt": 3}])
    with pytest.raises(P.DslamError):
        ctx.set_tune([{"width": 200, "height": 152, "level": 0, "jac_format": "fp32", "ppt": 2, "xcd_banded": 2}])
    ctx.close()
