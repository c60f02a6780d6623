"""HIP-graph replay of a frame's Gauss-Newton launches (each level's residual
passes and steps, captured at the first frame) against the same launches
issued one by one (the default): over a 640x480 sequence every result is equal
bit for bit at every frame, with other sessions' eager launches and host
synchronisations between the replays, and a session that switches between
the two in the middle of the sequence gives the same results too."""
import numpy as np
import pytest

import paper_2207_10940_amd as P
import synth
from tests.gpu_common import cuda

pytestmark = pytest.mark.gpu


def _same(a, b, where):
    if isinstance(a, dict):
        assert a.keys() == b.keys(), where
        for k in a:
            _same(a[k], b[k], f"{where}.{k}")
    else:
        x, y = np.asarray(a), np.asarray(b)
        assert x.shape == y.shape and x.tobytes() == y.tobytes(), where


def test_graph_replays_equal_eager_launches():
    import bench
    W, H = 640, 480
    seq = synth.configs.sequence(n_frames=7, width=W, height=H)
    cam = synth.configs.camera_for(W, H)
    tp = P.track_params(levels=3, iters=[10, 5, 4], mode="rgbdi")
    ctx = P.Context(0)
    sessions = []
    try:
        for _ in range(3):
            sessions.append(P.Session(ctx, cam, tp, P.imu_params(), seq["x0"], seq["q_IW"], seq["prior"]))
        graph, eager, mixed = sessions
        assert not graph.graphs  # launches one by one unless asked
        graph.set_graphs(True)
        eager.set_graphs(False)
        for j in range(1, 7):
            mixed.set_graphs(j % 2 == 1)
            md, mi, T, d, i, imu, t0, t1 = bench.frame_inputs(seq, j)
            frame = {"depth": cuda(d.numpy()), "intensity": cuda(i.numpy()), "model_depth": cuda(md.numpy()),
                     "model_intensity": cuda(mi.numpy()), "T_WM": T, "imu": imu, "t0": t0, "t1": t1}
            print(f"frame {j}: graph / eager / {'graph' if j % 2 == 1 else 'eager'}", flush=True)
            res = []
            for s in sessions:
                s.track_frame_input(frame)
                res.append(s.result())
            assert res[0]["status"] == 0
            _same(res[1], res[0], f"eager, frame {j}")
            _same(res[2], res[0], f"mixed, frame {j}")
        assert P.lib().dslam_session_set_graphs(graph.handle, 2) == P._abi.ERR_INVALID
    finally:
        for s in sessions:
            s.close()
        ctx.close()
