"""Batched tracking (serving form) through the C ABI: every session's result
in a batch must equal, bit for bit, the result of tracking it alone, whatever
the other sessions of the batch and the batch composition of each step."""
import numpy as np
import pytest

import paper_2207_10940_amd as P
import synth
from tests.gpu_common import open_seq_session as _open, same_result as _same, seq_frame as _frame

pytestmark = pytest.mark.gpu

# (seed, width, height, mode): mixed resolutions, a ragged one (200x152: tiles
# and blocks do not divide the image), one RGB-D-only and one gyro-only session
SESSIONS = [(3101, 160, 120, "rgbdi"), (3102, 320, 240, "rgbdi"), (3103, 160, 120, "rgbdi"),
            (3104, 200, 152, "rgbdi"), (3105, 160, 120, "rgbd"), (3106, 160, 120, "gyro")]
# batch composition per step: indices of the sessions that get their next frame
STEPS = [[0, 1, 2, 3, 4, 5], [1, 3, 5], [0, 2, 3, 4], [4, 0, 1, 5], [2, 1, 0, 3, 4, 5]]


@pytest.mark.parametrize("jac", ["fp32", "bf16"])
def test_batched_results_equal_alone_results(jac):
    import torch
    seqs = [synth.configs.sequence(seed=s, n_frames=8, width=w, height=h, device="cuda") for s, w, h, _ in SESSIONS]
    stream = torch.cuda.current_stream()
    # alone: each session tracks its frames 1, 2, ... one at a time
    ctx = P.Context(0)
    alone = []
    for idx, (seq, (_, _, _, mode)) in enumerate(zip(seqs, SESSIONS)):
        s = _open(ctx, seq, mode, jac=jac)
        res = []
        count = sum(1 for st in STEPS if idx in st)
        for j in range(1, count + 1):
            f = _frame(seq, j)
            s.set_model(f["model_depth"], f["model_intensity"], f["T_WM"], stream)
            s.track_frame(f["depth"], f["intensity"], f["imu"] if mode != "rgbd" else None, f["t0"], f["t1"], stream)
            res.append(s.result())
        alone.append(res)
        s.close()
    # batched: the composition changes from step to step
    sess = [_open(ctx, seq, mode, jac=jac) for seq, (_, _, _, mode) in zip(seqs, SESSIONS)]
    batch = P.Batch(ctx, len(SESSIONS))
    nxt = [1] * len(SESSIONS)
    for step, members in enumerate(STEPS):
        frames = [_frame(seqs[i], nxt[i]) for i in members]
        for i, f in zip(members, frames):
            if SESSIONS[i][3] == "rgbd":
                f["imu"] = None
        batch.track([sess[i] for i in members], frames, stream)
        out = batch.results()
        for i, r in zip(members, out):
            _same(r, alone[i][nxt[i] - 1], f"step {step} session {i} frame {nxt[i]}")
            # the session's own result call sees the same record
            _same(sess[i].result(), r, f"session result {i}")
            nxt[i] += 1
        print(f"step {step}: sessions {members} equal to alone", flush=True)
    batch.close()
    for s in sess:
        s.close()
    ctx.close()


# compositions repeat, so later steps replay graphs captured by earlier ones
GRAPH_STEPS = [[0, 1, 2, 3, 4, 5], [1, 3, 5], [5, 4, 3, 2, 1, 0], [0, 2, 3, 4], [0, 1, 2, 3, 4, 5], [3, 1, 5],
               [2, 0, 4, 3], [1, 0, 2, 3, 4, 5]]


def test_batch_graph_replays_equal_alone_results():
    """With the batch's launches replayed from graphs (one per composition), every step equals the
    sessions tracked alone, bit for bit, also when eager work of the program (another session's
    frames, library and torch kernels, synchronisations) runs between the replays."""
    import torch
    seqs = [synth.configs.sequence(seed=s, n_frames=10, width=w, height=h, device="cuda") for s, w, h, _ in SESSIONS]
    stream = torch.cuda.current_stream()
    ctx = P.Context(0)
    alone = []
    for idx, (seq, (_, _, _, mode)) in enumerate(zip(seqs, SESSIONS)):
        s = _open(ctx, seq, mode)
        res = []
        for j in range(1, sum(1 for st in GRAPH_STEPS if idx in st) + 1):
            f = _frame(seq, j)
            if mode == "rgbd":
                f["imu"] = None
            res.append(s.track_frame_sync(f, stream))
        alone.append(res)
        s.close()
    sess = [_open(ctx, seq, mode) for seq, (_, _, _, mode) in zip(seqs, SESSIONS)]
    other = _open(ctx, seqs[0], "rgbdi")
    batch = P.Batch(ctx, len(SESSIONS))
    batch.set_graphs(True)
    nxt = [1] * len(SESSIONS)
    scratch = torch.zeros(1 << 20, device="cuda")
    for step, members in enumerate(GRAPH_STEPS):
        frames = [_frame(seqs[i], nxt[i]) for i in members]
        for i, f in zip(members, frames):
            if SESSIONS[i][3] == "rgbd":
                f["imu"] = None
        batch.track([sess[i] for i in members], frames, stream)
        out = batch.results()
        for i, r in zip(members, out):
            _same(r, alone[i][nxt[i] - 1], f"graph step {step} session {i} frame {nxt[i]}")
            nxt[i] += 1
        print(f"graph step {step}: sessions {members} equal to alone", flush=True)
        # the program's own eager work between replays
        other.track_frame_sync(_frame(seqs[0], 1 + step % 8), stream)
        scratch.mul_(0.5).add_(float(step))
        torch.cuda.synchronize()
    batch.set_graphs(False)  # frees the graphs; the eager launches continue the same sessions
    members = [0, 1, 2, 3, 4, 5]
    frames = [_frame(seqs[i], nxt[i]) for i in members]
    frames[4]["imu"] = None
    batch.track([sess[i] for i in members], frames, stream)
    assert all(r["status"] == 0 for r in batch.results())
    batch.close()
    other.close()
    for s in sess:
        s.close()
    ctx.close()


def test_batch_rejects_inconsistent_sessions():
    import torch
    seq = synth.configs.sequence(seed=3201, n_frames=3, width=160, height=120, device="cuda")
    ctx = P.Context(0)
    a = _open(ctx, seq, "rgbdi")
    tp = P.track_params(levels=2, iters=(4, 3), mode="rgbdi")
    b = P.Session(ctx, seq["camera"], tp, P.imu_params(), seq["x0"], seq["q_IW"], seq["prior"])
    batch = P.Batch(ctx, 4)
    f = _frame(seq, 1)
    stream = torch.cuda.current_stream()
    with pytest.raises(P.DslamError):   # different pyramid depth
        batch.track([a, b], [f, f], stream)
    with pytest.raises(P.DslamError):   # the same session twice
        batch.track([a, a], [f, f], stream)
    bad = dict(f)
    bad["imu"] = {k: v[::-1].copy() for k, v in f["imu"].items()}
    with pytest.raises(P.DslamError):   # unsorted IMU samples
        batch.track([a], [bad], stream)
    batch.track([a], [f], stream)
    assert batch.results()[0]["status"] == 0
    with pytest.raises(P.DslamError):   # more sessions than the batch holds
        P.Batch(ctx, 0)
    batch.close()
    a.close()
    b.close()
    ctx.close()


def test_batched_step_leaves_current_normals_to_demand():
    """Without the normal gate a batched step does not write the current
    pyramid's normals; reading them (dslam_copy_pyramid) or fusing the frame
    into a map fills them first, with the values a single-session frame
    writes, bit for bit.  A session with the gate keeps them in the step."""
    import math
    import torch
    stream = torch.cuda.current_stream()
    specs = [(3121, 160, 120, None), (3122, 200, 152, None), (3123, 160, 120, math.cos(math.radians(20.0)))]
    seqs = [synth.configs.sequence(seed=sd, n_frames=4, width=w, height=h, device="cuda") for sd, w, h, _ in specs]
    ctx = P.Context(0)

    def open_session(seq, gate):
        tp = P.track_params(levels=3, iters=(4, 3, 2), mode="rgbdi", icp_cos=gate)
        return P.Session(ctx, seq["camera"], tp, P.imu_params(), seq["x0"], seq["q_IW"], seq["prior"])

    def planes(s):
        return [[s.copy_pyramid(P.PYR_CURRENT, l, ch) for ch in range(P.CH_VX, P.CH_NZ + 1)] for l in range(3)]

    def fused(s, seq, f):
        m = P.Map(ctx, seq["camera"], capacity=40000)
        m.fuse(s, f["T_WM"], stream)
        torch.cuda.synchronize()
        out = m.arrays()
        m.close()
        return out

    alone = []
    for seq, (_, _, _, gate) in zip(seqs, specs):
        s = open_session(seq, gate)
        for j in (1, 2):
            f = _frame(seq, j)
            s.set_model(f["model_depth"], f["model_intensity"], f["T_WM"], stream)
            s.track_frame(f["depth"], f["intensity"], f["imu"], f["t0"], f["t1"], stream)
        alone.append((s.result(), planes(s), fused(s, seq, f)))
        s.close()
    sess = [open_session(seq, gate) for seq, (_, _, _, gate) in zip(seqs, specs)]
    batch = P.Batch(ctx, len(sess))
    for j in (1, 2):
        frames = [_frame(seq, j) for seq in seqs]
        batch.track(sess, frames, stream)
        out = batch.results()
    for i, (s, seq) in enumerate(zip(sess, seqs)):
        r, pl, mp = alone[i]
        _same(out[i], r, f"session {i}")
        if i == 0:  # normals filled from the stored depths by the map fusion, then read back
            got_map = fused(s, seq, frames[i])
            got = planes(s)
        else:  # filled by the read (session 1); written by the gated session's step (session 2)
            got = planes(s)
            got_map = fused(s, seq, frames[i])
        for l in range(3):
            for ch in range(len(pl[l])):
                assert np.array_equal(got[l][ch], pl[l][ch]), (i, l, ch)
        assert mp.keys() == got_map.keys()
        for k in mp:
            assert np.array_equal(mp[k], got_map[k]), (i, k)
        print(f"session {i}: current planes and fused map equal to alone ({len(mp['px'])} surfels)", flush=True)
    batch.close()
    for s in sess:
        s.close()
    ctx.close()
