"""Serving loop (continuous batching) through the C ABI: every request's
result equals the result of tracking its session alone, frames of a session
come back in order, steps overlap, and sessions are admitted by the context's
HBM budget."""
import numpy as np
import pytest

import paper_2207_10940_amd as P
import synth
from tests.gpu_common import open_seq_session, same_result, seq_frame

pytestmark = pytest.mark.gpu

SESSIONS = [(3301, 160, 120, "rgbdi"), (3302, 320, 240, "rgbdi"), (3303, 200, 152, "rgbdi"),
            (3304, 160, 120, "rgbd"), (3305, 160, 120, "rgbdi")]
FRAMES = 4


def _alone(ctx, seq, mode, stream):
    s = open_seq_session(ctx, seq, mode)
    out = []
    for j in range(1, FRAMES + 1):
        f = seq_frame(seq, j)
        s.set_model(f["model_depth"], f["model_intensity"], f["T_WM"], stream)
        s.track_frame(f["depth"], f["intensity"], f["imu"] if mode != "rgbd" else None, f["t0"], f["t1"], stream)
        out.append(s.result())
    s.close()
    return out


@pytest.mark.parametrize("graphs", [False, True])
def test_server_results_equal_alone_results(graphs):
    import torch
    stream = torch.cuda.current_stream()
    seqs = [synth.configs.sequence(seed=sd, n_frames=FRAMES + 2, width=w, height=h, device="cuda")
            for sd, w, h, _ in SESSIONS]
    ctx = P.Context(0)
    alone = [_alone(ctx, seq, mode, stream) for seq, (_, _, _, mode) in zip(seqs, SESSIONS)]
    torch.cuda.synchronize()
    sess = [open_seq_session(ctx, seq, mode) for seq, (_, _, _, mode) in zip(seqs, SESSIONS)]
    server = P.Server(ctx, max_batch=3, pipeline_depth=2, graphs=graphs)
    inputs, owner = [], {}
    # frames interleaved across sessions (each session's in order); the last two sessions start late
    order = sorted(((i, j) for j in range(1, FRAMES + 1) for i in range(len(SESSIONS))),
                   key=lambda ij: (ij[1] + (2 if ij[0] >= 3 else 0), ij[0]))
    for i, j in order:
        f = seq_frame(seqs[i], j)
        if SESSIONS[i][3] == "rgbd":
            f["imu"] = None
        fi, keep = P.frame_input(f)
        inputs.append((fi, keep))
        rid = server.submit(sess[i], fi)
        owner[rid] = (i, j)
    got = {i: [] for i in range(len(SESSIONS))}
    sizes = set()
    while sum(len(v) for v in got.values()) < len(order):
        for rid, _h, t_sub, t_launch, t_done, dev_ms, bsize, res in server.poll(wait=True):
            i, j = owner[rid]
            got[i].append((j, P.result_dict(res)))
            sizes.add(bsize)
            assert t_sub <= t_launch <= t_done and dev_ms > 0
    assert server.counts() == (0, 0)
    for i in range(len(SESSIONS)):
        js = [j for j, _ in got[i]]
        assert js == sorted(js) == list(range(1, FRAMES + 1)), (i, js)  # in order, none lost
        for j, r in got[i]:
            same_result(r, alone[i][j - 1], f"session {i} frame {j}")
    assert max(sizes) == 3 and min(sizes) >= 1
    print(f"batch sizes seen: {sorted(sizes)}", flush=True)
    server.close()
    for s in sess:
        s.close()
    ctx.close()


def test_server_pipelines_a_sessions_frames_across_steps():
    """Every session in every step (a saturated mix): the next step is staged and
    launched while the previous one runs, and the device orders each session's
    frames across the two step streams.  Results equal tracking alone."""
    import torch
    stream = torch.cuda.current_stream()
    specs = [(3601, 320, 240, "rgbdi"), (3602, 160, 120, "rgbdi"), (3603, 200, 152, "rgbd")]
    seqs = [synth.configs.sequence(seed=sd, n_frames=FRAMES + 2, width=w, height=h, device="cuda")
            for sd, w, h, _ in specs]
    ctx = P.Context(0)
    alone = [_alone(ctx, seq, mode, stream) for seq, (_, _, _, mode) in zip(seqs, specs)]
    torch.cuda.synchronize()
    sess = [open_seq_session(ctx, seq, mode) for seq, (_, _, _, mode) in zip(seqs, specs)]
    server = P.Server(ctx, max_batch=len(specs), pipeline_depth=2)
    inputs, owner = [], {}
    for j in range(1, FRAMES + 1):
        for i in range(len(specs)):
            f = seq_frame(seqs[i], j)
            if specs[i][3] == "rgbd":
                f["imu"] = None
            fi, keep = P.frame_input(f)
            inputs.append((fi, keep))
            owner[server.submit(sess[i], fi)] = (i, j)
    got = {i: {} for i in range(len(specs))}
    while sum(len(v) for v in got.values()) < len(specs) * FRAMES:
        for rid, _h, t_sub, t_launch, t_done, dev_ms, bsize, res in server.poll(wait=True):
            i, j = owner[rid]
            got[i][j] = (t_launch, t_done, bsize, P.result_dict(res))
            assert dev_ms > 0
    assert server.counts() == (0, 0)
    overlapped = 0
    for i in range(len(specs)):
        assert sorted(got[i]) == list(range(1, FRAMES + 1)), i
        for j in range(1, FRAMES + 1):
            assert got[i][j][2] == len(specs)
            same_result(got[i][j][3], alone[i][j - 1], f"session {i} frame {j}")
            if j > 1 and got[i][j][0] < got[i][j - 1][1]:
                overlapped += 1  # launched before the previous frame was returned
    assert overlapped > 0
    print(f"frames launched before their predecessor returned: {overlapped}", flush=True)
    server.close()
    for s in sess:
        s.close()
    ctx.close()


def test_server_rejects_bad_requests():
    seq = synth.configs.sequence(seed=3401, n_frames=3, width=160, height=120, device="cuda")
    ctx = P.Context(0)
    s = open_seq_session(ctx, seq, "rgbdi")
    server = P.Server(ctx, max_batch=2)
    f = seq_frame(seq, 1)
    bad = dict(f)
    bad["imu"] = {k: v[::-1].copy() for k, v in f["imu"].items()}
    fi, keep = P.frame_input(bad)
    with pytest.raises(P.DslamError):
        server.submit(s, fi)
    with pytest.raises(P.DslamError):
        P.Server(ctx, max_batch=0)
    fi, keep = P.frame_input(f)
    server.submit(s, fi)
    done = []
    while not done:
        done = server.poll(wait=True)
    assert done[0][-1].status == 0
    server.close()
    s.close()
    ctx.close()


def test_admission_by_hbm_budget():
    cam = synth.configs.camera_for(320, 240)
    per = P.session_bytes(cam, 3)
    probe = P.Context(0)
    server = P.Server(probe, max_batch=4)
    staging = probe.used_bytes()
    server.close()
    probe.close()
    seq = synth.configs.sequence(seed=3501, n_frames=3, width=320, height=240, device="cuda")
    ctx = P.Context(0, staging + 2 * per + per // 2)
    server = P.Server(ctx, max_batch=4)
    a = open_seq_session(ctx, seq, "rgbdi")
    b = open_seq_session(ctx, seq, "rgbdi")
    with pytest.raises(P.DslamError) as e:
        open_seq_session(ctx, seq, "rgbdi")
    assert e.value.code == 2  # NO_CAPACITY
    a.close()
    c = open_seq_session(ctx, seq, "rgbdi")  # admitted once memory frees up
    fi, keep = P.frame_input(seq_frame(seq, 1))
    server.submit(c, fi)
    done = []
    while not done:
        done = server.poll(wait=True)
    assert done[0][-1].status == 0
    assert ctx.used_bytes() == staging + 2 * per
    server.close()
    b.close()
    c.close()
    ctx.close()
