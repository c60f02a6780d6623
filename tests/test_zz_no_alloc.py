"""The allocation-free batched step (dslam_batch_track_noalloc) through the C
ABI: its results equal those of dslam_batch_track + dslam_batch_results bit
for bit, on two calls in a row, the second with fewer (and smaller) sessions
than the first."""
import numpy as np
import pytest

import paper_2207_10940_amd as P
import synth
from tests.gpu_common import open_seq_session as _open, same_result as _same, seq_frame as _frame

pytestmark = pytest.mark.gpu

SESSIONS = [(3401, 320, 240, "rgbdi"), (3402, 160, 120, "rgbdi"), (3403, 200, 152, "rgbdi"), (3404, 160, 120, "rgbd")]
CALLS = [[0, 1, 2, 3], [1, 3]]  # the second call: two sessions, the smallest images


def _frames(seqs, members, nxt):
    frames = [_frame(seqs[i], nxt[i]) for i in members]
    for i, f in zip(members, frames):
        if SESSIONS[i][3] == "rgbd":
            f["imu"] = None
    return frames


def test_noalloc_batch_equals_batch():
    import torch
    seqs = [synth.configs.sequence(seed=s, n_frames=4, width=w, height=h, device="cuda") for s, w, h, _ in SESSIONS]
    stream = torch.cuda.current_stream()
    ctx = P.Context(0)
    ref = [_open(ctx, seq, mode) for seq, (_, _, _, mode) in zip(seqs, SESSIONS)]
    got = [_open(ctx, seq, mode) for seq, (_, _, _, mode) in zip(seqs, SESSIONS)]
    batch = P.Batch(ctx, len(SESSIONS))
    nxt = [1] * len(SESSIONS)
    for call, members in enumerate(CALLS):
        print(f"no-alloc call {call}: sessions {members}", flush=True)
        batch.track([ref[i] for i in members], _frames(seqs, members, nxt), stream)
        want = batch.results()
        out = P.batch_track_noalloc([got[i] for i in members], _frames(seqs, members, nxt), stream)
        assert len(out) == len(members)
        for i, a, b in zip(members, want, out):
            _same(a, b, f"call {call} session {i}")
            assert a["health"] == b["health"] and a["frame_index"] == b["frame_index"] == nxt[i]
            _same(got[i].result(), b, f"session record {i}")
            nxt[i] += 1
    with pytest.raises(P.DslamError) as ei:  # the same session twice
        P.batch_track_noalloc([got[0], got[0]], _frames(seqs, [0, 0], nxt), stream)
    assert ei.value.code == P._abi.ERR_INVALID
    batch.close()
    for s in ref + got:
        s.close()
    ctx.close()
