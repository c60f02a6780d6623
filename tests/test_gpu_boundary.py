"""The boundary's calls beyond the hot path itself, through the C ABI:
asynchronous results into caller memory, the synchronous variant, the
tracking-lost flag, session checkpoints (bitwise resume), closing a session
that a server still references, and ordering across streams."""
import ctypes as C

import numpy as np
import pytest

import paper_2207_10940_amd as P
import synth
from tests.gpu_common import cuda, open_seq_session, same_result, seq_frame, session

pytestmark = pytest.mark.gpu


def _pair_frame(d, model=True):
    f = {"depth": cuda(d["depth"].numpy()), "intensity": cuda(d["intensity"].numpy()), "imu": d["imu"],
         "t0": d["t0"], "t1": d["t1"], "model_depth": None}
    if model:
        f.update(model_depth=cuda(d["model_depth"].numpy()), model_intensity=cuda(d["model_intensity"].numpy()),
                 T_WM=d["T_WM"])
    return f


def test_result_into_pinned_memory_and_sync_variant():
    import torch
    d = synth.configs.frame_pair()
    print("track_frame out / sync", flush=True)
    pinned = torch.empty(C.sizeof(P._abi.TrackResult), dtype=torch.uint8, pin_memory=True)
    out = P._abi.TrackResult.from_address(pinned.data_ptr())
    with session(160, 120, 2, [4, 4], x0=d["x0"], q_IW=d["q_IW"], prior=d["prior"]) as s:
        s.track_frame_input(_pair_frame(d), out=out)
        torch.cuda.current_stream().synchronize()
        a = P.result_dict(out)
        b = s.result()
    with session(160, 120, 2, [4, 4], x0=d["x0"], q_IW=d["q_IW"], prior=d["prior"]) as s:
        c = s.track_frame_sync(_pair_frame(d))
    same_result(a, b, "async out vs session result")
    same_result(a, c, "async vs sync")
    assert a["health"] == 0 and not a["tracking_lost"] and a["frame_index"] == 1


def test_tracking_lost_flags():
    d = synth.configs.frame_pair()
    zero = np.zeros((120, 160), np.float32)
    print("tracking lost", flush=True)
    with session(160, 120, 2, [3, 3], x0=d["x0"], q_IW=d["q_IW"], prior=d["prior"]) as s:
        f = _pair_frame(d)
        f["depth"] = cuda(zero)  # no depth: no visual term, the IMU and the prior alone
        r = s.track_frame_sync(f)
        assert r["status"] == 0 and r["n_icp"][0] == 0 and r["n_rgb"][0] == 0
        assert r["health"] & P.HEALTH_LOW_INLIERS and r["tracking_lost"]
    with session(160, 120, 2, [3, 3], mode="rgbd") as s:  # RGB-D only, no depth: singular
        f = _pair_frame(d)
        f["depth"] = cuda(zero)
        r = s.track_frame_sync(f)
        assert r["status"] == P._abi.ERR_SINGULAR
        assert r["health"] & P.HEALTH_SINGULAR and r["tracking_lost"]
    # the inlier threshold is a fraction of 2 x pixels: 0.99 flags an ordinary frame, 0 never does
    for frac, lost in ((0.99, True), (0.0, False)):
        with session(160, 120, 2, [3, 3], x0=d["x0"], q_IW=d["q_IW"], prior=d["prior"],
                     min_inlier_frac=frac) as s:
            r = s.track_frame_sync(_pair_frame(d))
            assert r["status"] == 0 and r["tracking_lost"] == lost, (frac, r["health"])


def _seq_session(ctx, seq):
    return open_seq_session(ctx, seq, "rgbdi", iters=(4, 3, 2))


def test_checkpoint_resume_is_bitwise():
    """Resuming from a checkpoint taken after frame k gives frames k+1..k+5
    bit for bit, including a frame tracked against the checkpointed model
    view (no model view given with it)."""
    seq = synth.configs.sequence(seed=2301, n_frames=10, width=320, height=240, device="cuda")
    k = 3
    ctx = P.Context(0)
    try:
        a = _seq_session(ctx, seq)
        for j in range(1, k + 1):
            a.track_frame_sync(seq_frame(seq, j))
        blob = a.checkpoint()
        print(f"checkpoint {len(blob)} bytes", flush=True)

        def frames(j):
            f = seq_frame(seq, j)
            if j == k + 1:
                f["model_depth"] = None  # against the model view of frame k
            return f
        want = [a.track_frame_sync(frames(j)) for j in range(k + 1, k + 6)]
        b = _seq_session(ctx, seq)
        b.restore(blob)
        got = [b.track_frame_sync(frames(j)) for j in range(k + 1, k + 6)]
        for j, (x, y) in enumerate(zip(want, got)):
            same_result(x, y, f"frame {k + 1 + j}")
            assert x["frame_index"] == y["frame_index"] == k + 1 + j
        # foreign, corrupted and truncated blobs are rejected, leaving the session as it was
        bad = bytearray(blob)
        bad[len(bad) // 2] ^= 0x40
        for junk in (bytes(bad), blob[:-8], b"\0" * 64):
            with pytest.raises(P.DslamError) as ei:
                b.restore(junk)
            assert ei.value.code == P._abi.ERR_INVALID
        other = open_seq_session(ctx, seq, "rgbdi", iters=(4, 3, 3))  # different schedule
        with pytest.raises(P.DslamError) as ei:
            other.restore(blob)
        assert ei.value.code == P._abi.ERR_INVALID
        other.close()
        a.close()
        b.close()
    finally:
        ctx.close()


def test_close_is_busy_while_a_server_holds_requests():
    seq = synth.configs.sequence(seed=2302, n_frames=3, width=160, height=120, device="cuda")
    ctx = P.Context(0)
    try:
        s = _seq_session(ctx, seq)
        sv = P.Server(ctx, max_batch=4)
        fi, keep = P.frame_input(seq_frame(seq, 1))
        sv.submit(s, fi)
        print("close with a queued request", flush=True)
        with pytest.raises(P.DslamError) as ei:
            s.close()
        assert ei.value.code == P._abi.ERR_BUSY
        done = []
        while not done:
            done = sv.poll(wait=True)
        assert done[0][7].status == 0
        s2 = _seq_session(ctx, seq)
        fi2, keep2 = P.frame_input(seq_frame(seq, 1))
        sv.submit(s2, fi2)
        sv.close()  # drops the request: the session closes afterwards
        s.close()
        s2.close()
    finally:
        ctx.close()


def test_frames_on_different_streams_are_ordered():
    import torch
    seq = synth.configs.sequence(seed=2303, n_frames=4, width=320, height=240, device="cuda")
    ctx = P.Context(0)
    try:
        a = _seq_session(ctx, seq)
        ref = [a.track_frame_sync(seq_frame(seq, j)) for j in (1, 2, 3)]
        b = _seq_session(ctx, seq)
        streams = [torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.current_stream()]
        frames = [seq_frame(seq, j) for j in (1, 2, 3)]
        for f, st in zip(frames, streams):  # enqueued back to back, each on its own stream
            b.track_frame_input(f, st)
        got = b.result()
        same_result(ref[-1], got, "three streams")
        a.close()
        b.close()
    finally:
        ctx.close()
