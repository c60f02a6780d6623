"""Precision form through the C ABI: Jacobian rows in FP16 / BF16 contracted
into J^T J on MFMA with float32 accumulation.  Association masks and inlier
counts stay bit-exact (they are decided in float32 before any rounding to 16
bits); J^T J, J^T r and the cost are compared with the float64 oracle and with
the plain float32 form; Gauss-Newton recovers the pose to 1e-4 rad / 0.1 mm."""
import numpy as np
import pytest

import paper_2207_10940_amd as P
import synth
from oracle import track
from tests.gpu_common import cuda, jtr_scale, pose_err, rel_fro, session
from tests.test_gpu_parity import _linearize_case

pytestmark = pytest.mark.gpu

# relative bounds on J^T J (Frobenius), J^T r (against its normwise scale) and
# the cost: the unit roundoff of the 16-bit format (FP16 4.9e-4, BF16 3.9e-3)
# scaled by 0.6 -- rounding errors of many pixels average out
BOUND = {"fp16": 3e-4, "bf16": 2.4e-3,
         "fp32_mfma": 1e-5}  # float32 rows on v_mfma_f32_16x16x4_f32: the plain form's bar


@pytest.mark.parametrize("jac", ["fp16", "bf16", "fp32_mfma"])
@pytest.mark.parametrize("W,H,levels,seed", [(160, 120, 2, 1001), (200, 152, 3, 7), (640, 480, 3, 1002)])
def test_precision_linearize(jac, W, H, levels, seed):
    import torch
    d, x0, x1, T_WM = _linearize_case(W, H, seed)
    cam = d["camera"]
    params = track.default_params(levels=levels, iters=[1] * levels, mode="rgbdi")
    cur, ref = track.build_pyramids(d["depth"].numpy(), d["intensity"].numpy(), d["model_depth"].numpy(),
                                    d["model_intensity"].numpy(), cam, levels)
    Ra, ta, Rb, tb = track.fp32_transforms(T_WM, x0, x1)
    print(f"precision {jac} {W}x{H} seed {seed}", flush=True)
    with session(W, H, levels, [1] * levels, jac=jac) as s, session(W, H, levels, [1] * levels) as s32:
        for ss in (s, s32):
            ss.set_model(cuda(d["model_depth"].numpy()), cuda(d["model_intensity"].numpy()), T_WM)
            ss.build_pyramid(P.PYR_CURRENT, cuda(d["depth"].numpy()), cuda(d["intensity"].numpy()))
        for l in range(levels):
            vis = track.linearise_visual(cur[l], ref[l], T_WM, x0, x1, Ra, ta, Rb, tb, params)
            mask = torch.zeros((H >> l, W >> l), dtype=torch.uint8, device="cuda")
            g = s.linearize(l, Ra, ta, Rb, tb, x0, x1, mask=mask)
            f = s32.linearize(l, Ra, ta, Rb, tb, x0, x1)
            m = mask.cpu().numpy()
            assert np.array_equal((m & 1) != 0, vis["mask_icp"]) and np.array_equal((m & 2) != 0, vis["mask_rgb"])
            assert g["n_icp"] == vis["n_icp"] and g["n_rgb"] == vis["n_rgb"]
            for term, cols in (("icp", np.r_[6:12]), ("rgb", np.r_[0:12])):
                eH = rel_fro(g["H_" + term], vis["H_" + term])
                eH32 = rel_fro(g["H_" + term], f["H_" + term])
                scale = jtr_scale(vis[term], cols, 12)
                eb = np.linalg.norm(g["b_" + term] - vis["b_" + term]) / scale
                ec = abs(g["cost_" + term] - vis["cost_" + term]) / vis["cost_" + term]
                print(f"  level {l} {term}: JtJ vs oracle {eH:.2e} vs fp32 {eH32:.2e}  Jtr {eb:.2e}  cost {ec:.2e}",
                      flush=True)
                assert eH < BOUND[jac] and eb < BOUND[jac] and ec < max(BOUND[jac], 1e-4), (l, term, eH, eb, ec)


@pytest.mark.parametrize("jac", ["fp16", "bf16", "fp32_mfma"])
@pytest.mark.parametrize("mode", ["rgbdi", "rgbd"])
def test_precision_track_pair_recovers_pose(jac, mode):
    """Gauss-Newton iteration recovers what the 16-bit rows lose: the tracked
    pose matches the float64 oracle within 1e-4 rad / 0.1 mm."""
    W, H, levels, iters = 160, 120, 2, (4, 4)
    d = synth.configs.frame_pair(seed=1001, width=W, height=H)
    params = track.default_params(levels=levels, iters=iters, mode=mode)
    o = track.track_frame(d["depth"].numpy(), d["intensity"].numpy(), d["model_depth"].numpy(),
                          d["model_intensity"].numpy(), d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"], d["x0"],
                          d["q_IW"], d["prior"], params)
    prior = d["prior"] if mode != "rgbd" else None
    res = {}
    for fmt in ("fp32", jac):
        with session(W, H, levels, list(iters), mode=mode, x0=d["x0"], q_IW=d["q_IW"], prior=prior, jac=fmt) as s:
            s.set_model(cuda(d["model_depth"].numpy()), cuda(d["model_intensity"].numpy()), d["T_WM"])
            s.track_frame(cuda(d["depth"].numpy()), cuda(d["intensity"].numpy()), d["imu"], d["t0"], d["t1"])
            res[fmt] = s.result()
    g = res[jac]
    assert g["status"] == 0
    dr, da = pose_err(g["x1"], o["x1"])
    dr32, da32 = pose_err(g["x1"], res["fp32"]["x1"])
    print(f"track pair {mode} {jac}: vs oracle {dr:.2e} m {da:.2e} rad; vs fp32 {dr32:.2e} m {da32:.2e} rad",
          flush=True)
    assert dr < 1e-4 and da < 1e-4, (dr, da)


@pytest.mark.parametrize("nearest,within_bound", [(0.27, True), (0.06, False)])
def test_fp16_rows_near_range(nearest, within_bound):
    """FP16 rows are scaled for depths of at least 0.25 m.  The frame pair's scene and poses shrunk so
    that the nearest depth is 0.27 m stays within the FP16 bound of the oracle; shrunk to 0.06 m, the
    nearest pixels' entries saturate at the FP16 maximum instead of overflowing: the sums stay finite
    (the error is then the saturation's, not bounded) and the masks and counts stay exact."""
    import torch
    W, H, levels = 160, 120, 2
    d, x0, x1, T_WM = _linearize_case(W, H, 1001)
    z = d["depth"].numpy()
    scale = nearest / float(z[z > 0].min())
    depth, mdepth = z * scale, d["model_depth"].numpy() * scale
    x0 = dict(x0, r=x0["r"] * scale)
    x1 = dict(x1, r=x1["r"] * scale)
    T_WM = T_WM.copy()
    T_WM[:3, 3] *= scale
    valid = depth[depth > 0]
    print(f"fp16 near range: nearest depth {valid.min():.3f} m", flush=True)
    cam = d["camera"]
    params = track.default_params(levels=levels, iters=[1] * levels, mode="rgbdi")
    cur, ref = track.build_pyramids(depth, d["intensity"].numpy(), mdepth, d["model_intensity"].numpy(), cam,
                                    levels)
    Ra, ta, Rb, tb = track.fp32_transforms(T_WM, x0, x1)
    with session(W, H, levels, [1] * levels, jac="fp16") as s:
        s.set_model(cuda(mdepth.astype(np.float32)), cuda(d["model_intensity"].numpy()), T_WM)
        s.build_pyramid(P.PYR_CURRENT, cuda(depth.astype(np.float32)), cuda(d["intensity"].numpy()))
        for l in range(levels):
            vis = track.linearise_visual(cur[l], ref[l], T_WM, x0, x1, Ra, ta, Rb, tb, params)
            mask = torch.zeros((H >> l, W >> l), dtype=torch.uint8, device="cuda")
            g = s.linearize(l, Ra, ta, Rb, tb, x0, x1, mask=mask)
            m = mask.cpu().numpy()
            assert np.array_equal((m & 1) != 0, vis["mask_icp"]) and np.array_equal((m & 2) != 0, vis["mask_rgb"])
            assert g["n_icp"] == vis["n_icp"] and g["n_rgb"] == vis["n_rgb"]
            for term in ("icp", "rgb"):
                assert np.all(np.isfinite(g["H_" + term])) and np.all(np.isfinite(g["b_" + term]))
                eH = rel_fro(g["H_" + term], vis["H_" + term])
                print(f"  level {l} {term}: JtJ vs oracle {eH:.2e}", flush=True)
                if within_bound:
                    assert eH < BOUND["fp16"], (l, term, eH)
