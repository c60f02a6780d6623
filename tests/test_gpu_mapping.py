"""GPU parity of the surfel map (dslam_map_*) against the oracle's float32
mirror: after every fusion the surfel arrays (count, positions, normals,
intensities, radii, confidences, in index order) and every rendered model
view (depth and intensity) are equal bit for bit; a closed tracking loop
(predict from the map, track, fuse) stays on the ground truth."""
import numpy as np
import pytest
import torch

import paper_2207_10940_amd as P
import synth
from oracle import mapping as M
from oracle import pyramid as pyr
from tests.gpu_common import cuda, session

pytestmark = pytest.mark.gpu


def _pose(g):
    T = np.eye(4)
    T[:3, :3] = synth.configs._rot_from_quat(g["q"])
    T[:3, 3] = g["r"]
    return T


def _oracle_frame(depth, inten, cam, levels):
    lev = pyr.build(depth, inten, cam.fx, cam.fy, cam.cx, cam.cy, levels)
    return lev[0]["V"], M.fusion_normals(lev), (lev[0]["I"] * np.float32(64.0)).astype(np.uint16)


def _assert_same_map(gm, om):
    assert len(gm["px"]) == len(om["px"])
    for k in M.FIELDS:
        assert np.array_equal(gm[k].view(np.uint32), om[k].view(np.uint32)), k


@pytest.mark.parametrize("W,H,levels,capacity", [(160, 120, 2, 10**6), (200, 152, 3, 10**6), (160, 120, 1, 25000),
                                                 (640, 480, 3, 2 * 10**6)])
def test_fuse_and_render_match_oracle(W, H, levels, capacity):
    print(f"map {W}x{H} levels {levels} capacity {capacity}", flush=True)
    seq = synth.configs.sequence(seed=3001, n_frames=4, width=W, height=H)
    cam = seq["camera"]
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    rng = np.random.default_rng(7)
    with session(W, H, levels, [1] * levels, mode="rgbd") as s:
        mp = P.Map(s.ctx, cam, capacity)
        om = M.empty_map()
        odrop = 0
        for j in range(4):
            depth, inten = seq["depth"][j].numpy(), seq["intensity"][j].numpy()
            s.build_pyramid(P.PYR_CURRENT, cuda(depth), cuda(inten))
            T = _pose(seq["gt"][j])
            if j == 3:  # a pose off the truth: the map is fused wherever the tracker puts it
                T[:3, 3] += rng.normal(size=3) * 0.01
            mp.fuse(s, T)
            V, N, I16 = _oracle_frame(depth, inten, cam, levels)
            om, d = M.fuse(om, V, N, I16, T, K, W, H, capacity=capacity)
            odrop += d
            n, gdrop = mp.count()
            assert (n, gdrop) == (len(om["px"]), odrop), j
            _assert_same_map(mp.arrays(), om)
            # render at the next frame's pose
            Tn = _pose(seq["gt"][min(j + 1, 3)])
            dg = torch.zeros((H, W), dtype=torch.float32, device="cuda")
            ig = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
            mp.render(Tn, dg, ig)
            torch.cuda.synchronize()
            do, io = M.render(om, Tn, K, W, H)
            assert np.array_equal(dg.cpu().numpy().view(np.uint32), do.view(np.uint32)), j
            assert np.array_equal(ig.cpu().numpy(), io), j
            assert (do > 0).mean() > 0.5
        # prediction: the session's model pyramid is built from the rendered view
        Tn = _pose(seq["gt"][3])
        mp.predict(s, Tn)
        do, io, no = M.render(om, Tn, K, W, H, with_normals=True)
        got = s.copy_pyramid(P.PYR_MODEL, 0, P.CH_VZ)
        assert np.array_equal(got.view(np.uint32), do.view(np.uint32))
        for k, ch in enumerate((P.CH_NX, P.CH_NY, P.CH_NZ)):
            got = s.copy_pyramid(P.PYR_MODEL, 0, ch)
            assert np.array_equal(got.view(np.uint32), no[..., k].view(np.uint32)), k
        mp.close()


def test_empty_map_and_all_hole_frames():
    """Degenerate inputs: rendering a map with no surfels, and fusing a frame
    whose depth is all holes, into an empty and into a filled map."""
    W, H = 160, 120
    seq = synth.configs.sequence(seed=3003, n_frames=2, width=W, height=H)
    cam = seq["camera"]
    K = (cam.fx, cam.fy, cam.cx, cam.cy)
    holes = np.zeros((H, W), dtype=np.float32)
    with session(W, H, 2, [1, 1], mode="rgbd") as s:
        mp = P.Map(s.ctx, cam, 10**5)
        om = M.empty_map()
        T0 = _pose(seq["gt"][0])
        dg = torch.full((H, W), 7.0, dtype=torch.float32, device="cuda")
        ig = torch.full((H, W), 9, dtype=torch.uint8, device="cuda")
        mp.render(T0, dg, ig)
        torch.cuda.synchronize()
        do, io = M.render(om, T0, K, W, H)
        assert np.array_equal(dg.cpu().numpy().view(np.uint32), do.view(np.uint32))
        assert np.array_equal(ig.cpu().numpy(), io)
        assert not do.any()
        inten = seq["intensity"][0].numpy()
        for j, depth in enumerate((holes, seq["depth"][0].numpy(), holes)):
            s.build_pyramid(P.PYR_CURRENT, cuda(depth), cuda(inten))
            mp.fuse(s, T0)
            V, N, I16 = _oracle_frame(depth, inten, cam, 2)
            om, d = M.fuse(om, V, N, I16, T0, K, W, H, capacity=10**5)
            assert mp.count() == (len(om["px"]), d), j
            _assert_same_map(mp.arrays(), om)
        assert len(om["px"]) > 0
        mp.close()


def test_reset_and_errors():
    seq = synth.configs.sequence(seed=3002, n_frames=1, width=160, height=120)
    cam = seq["camera"]
    with session(160, 120, 1, [1], mode="rgbd") as s:
        mp = P.Map(s.ctx, cam, 10**5)
        s.build_pyramid(P.PYR_CURRENT, cuda(seq["depth"][0].numpy()), cuda(seq["intensity"][0].numpy()))
        mp.fuse(s, _pose(seq["gt"][0]))
        assert mp.count()[0] > 0
        mp.reset()
        assert mp.count() == (0, 0)
        bad = np.eye(4)
        bad[0, 3] = np.nan
        with pytest.raises(P.DslamError):
            mp.fuse(s, bad)
        mp.close()
        other = synth.configs.camera_for(200, 152)
        mp2 = P.Map(s.ctx, other, 10**4)
        with pytest.raises(P.DslamError):  # camera mismatch
            mp2.fuse(s, _pose(seq["gt"][0]))
        mp2.close()
    ctx = P.Context(0, 1 << 20)
    with pytest.raises(P.DslamError) as ei:  # 10^6 surfels do not fit in 1 MiB
        P.Map(ctx, cam, 10**6)
    assert ei.value.code == P._abi.ERR_NO_CAPACITY
    ctx.close()


def test_tracking_against_the_fused_map():
    """Closed loop on the 320x240 sequence: the model view of each frame is
    predicted from the map at the previous estimate, the frame is tracked and
    then fused at its estimate.  Every frame stays within 2 cm / 1 degree of
    the ground truth."""
    W, H, n = 320, 240, 16
    seq = synth.configs.sequence(seed=2001, n_frames=n, width=W, height=H)
    cam = seq["camera"]
    with session(W, H, 3, [10, 5, 4], x0=seq["x0"], q_IW=seq["q_IW"], prior=seq["prior"]) as s:
        mp = P.Map(s.ctx, cam, 4 * 10**6)
        try:
            _closed_loop(s, mp, seq, n)
        finally:
            mp.close()


def _closed_loop(s, mp, seq, n):
    s.build_pyramid(P.PYR_CURRENT, cuda(seq["depth"][0].numpy()), cuda(seq["intensity"][0].numpy()))
    prev = _pose(seq["gt"][0])
    mp.fuse(s, prev)
    for j in range(1, n):
        mp.predict(s, prev)
        a, b = synth.configs.imu_window(seq["imu"]["t"], seq["times"][j - 1], seq["times"][j])
        imu = {k: v[a:b] for k, v in seq["imu"].items()}
        s.track_frame(cuda(seq["depth"][j].numpy()), cuda(seq["intensity"][j].numpy()), imu,
                      seq["times"][j - 1], seq["times"][j])
        r = s.result()
        assert r["status"] == 0
        prev = _pose(r["x1"])
        g = seq["gt"][j]
        dr = np.linalg.norm(r["x1"]["r"] - g["r"])
        Rg, Re = synth.configs._rot_from_quat(g["q"]), synth.configs._rot_from_quat(r["x1"]["q"])
        da = np.degrees(np.arccos(np.clip((np.trace(Rg.T @ Re) - 1) / 2, -1, 1)))
        print(f"frame {j}: |dr| {dr * 100:.3f} cm, |da| {da:.4f} deg, surfels {mp.count()[0]}", flush=True)
        assert dr < 0.02 and da < 1.0, (j, dr, da)
        mp.fuse(s, prev)
