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


def _lost_pair(seed, patch):
    d = synth.configs.frame_pair(seed=seed, width=160, height=120)
    z = d["depth"].numpy().copy()
    keep = np.zeros_like(z, dtype=bool)
    keep[patch[0]:patch[0] + 6, patch[1]:patch[1] + 6] = True
    z[~keep] = 0.0
    return d, z


@pytest.mark.parametrize("graphs", [False, True])
def test_inertial_fallback_matches_oracle(graphs):
    """A frame with too few valid pixels to track (LOW_INLIERS) in RGB-D-inertial mode: with imu_fallback
    the result is the oracle's inertial-only re-estimate (one Gauss-Newton step of the prior and the IMU
    factor from the frame's start and its IMU prediction, marginalised there) and carries IMU_ONLY;
    without it, the oracle's joint estimate.  A frame that tracks is unaffected by the option."""
    from oracle import lie, track
    d, z = _lost_pair(1001, (60, 80))
    print(f"inertial fallback, graphs {graphs}", flush=True)
    for fallback in (True, False):
        p = track.default_params(levels=2, iters=(4, 4), mode="rgbdi")
        p["imu_fallback"] = fallback
        o = track.track_frame(z, d["intensity"].numpy(), d["model_depth"].numpy(), d["model_intensity"].numpy(),
                              d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"], d["q_IW"], d["prior"], p)
        with session(160, 120, 2, [4, 4], x0=d["x0"], q_IW=d["q_IW"], prior=d["prior"],
                     imu_fallback=fallback) as s:
            s.set_graphs(graphs)
            f = _pair_frame(d)
            f["depth"] = cuda(z)
            g = s.track_frame_sync(f)
            st = s.get_state()
        assert g["status"] == 0 and g["tracking_lost"] and g["health"] & P.HEALTH_LOW_INLIERS
        assert bool(g["health"] & P.HEALTH_IMU_ONLY) == fallback == ("imu_only" in o["health"])
        dr = np.linalg.norm(g["x1"]["r"] - o["x1"]["r"])
        da = np.linalg.norm(lie.quat_boxminus(g["x1"]["q"], o["x1"]["q"]))
        dv = np.linalg.norm(g["x1"]["v"] - o["x1"]["v"])
        eH = np.linalg.norm(g["prior"]["H"] - o["prior"]["H"]) / np.linalg.norm(o["prior"]["H"])
        print(f"  fallback {fallback}: |dr| {dr:.2e} |da| {da:.2e} |dv| {dv:.2e} prior H {eH:.2e}", flush=True)
        assert dr < 1e-6 and da < 1e-6 and dv < 1e-6 and eH < 1e-4
        # the next frame starts from the published estimate
        for k in ("r", "q", "v", "bg", "ba"):
            assert np.array_equal(st[0][k], g["x1"][k]), k
    # a frame that tracks: the option changes nothing, bit for bit
    d = synth.configs.frame_pair(seed=1001, width=160, height=120)
    res = []
    for fallback in (False, True):
        with session(160, 120, 2, [4, 4], x0=d["x0"], q_IW=d["q_IW"], prior=d["prior"],
                     imu_fallback=fallback) as s:
            s.set_graphs(graphs)
            res.append(s.track_frame_sync(_pair_frame(d)))
    same_result(res[1], res[0], "clean frame with and without the fallback")
    assert res[1]["health"] == 0


def test_inertial_fallback_batched_equals_alone():
    import torch
    stream = torch.cuda.current_stream()
    d, z = _lost_pair(1001, (60, 80))
    e = synth.configs.frame_pair(seed=1002, width=160, height=120)
    print("inertial fallback batched", flush=True)
    lost = _pair_frame(d)
    lost["depth"] = cuda(z)
    clean = _pair_frame(e)
    ctx = P.Context(0)
    cam = synth.configs.camera_for(160, 120)
    tp = P.track_params(levels=2, iters=(4, 4), mode="rgbdi", imu_fallback=True)

    def open_(x):
        return P.Session(ctx, cam, tp, P.imu_params(), x["x0"], x["q_IW"], x["prior"])
    alone = []
    for x, f in ((d, lost), (e, clean)):
        s = open_(x)
        alone.append(s.track_frame_sync(f, stream))
        s.close()
    ss = [open_(d), open_(e)]
    batch = P.Batch(ctx, 2)
    batch.track(ss, [lost, clean], stream)
    out = batch.results()
    same_result(out[0], alone[0], "lost session batched")
    same_result(out[1], alone[1], "clean session batched")
    assert out[0]["health"] & P.HEALTH_IMU_ONLY and out[1]["health"] == 0
    batch.close()
    for s in ss:
        s.close()
    ctx.close()
