"""Pins of the oracle's association, residuals and Jacobians (Section IV-B, eqs. (3)-(4))."""
import numpy as np

from oracle import association as assoc
from oracle import lie, track
from oracle import pyramid as pyr
from oracle import residuals as res
from synth.configs import Camera, quat_from_matrix
from synth.scene import Scene, render
from tests.oracle_cases import identity_state, tilted_plane_pair


def _params(**kw):
    p = track.default_params(levels=1, iters=(1,), mode="rgbd")
    p.update(kw)
    return p


def _frames_8x6(seed=3):
    rng = np.random.default_rng(seed)
    sc = Scene(planes=[(np.array([0.2, -0.1, -1.0]) / np.linalg.norm([0.2, -0.1, -1.0]), -2.0)],
               spheres=[(np.array([0.1, 0.05, 1.6]), 0.25)], seed=seed)
    z0, i0 = render(sc, np.eye(3), np.zeros(3), 8, 6, 6.5, 6.5, 4.0, 3.0)
    R1 = lie.exp_so3(rng.normal(size=3) * 0.05)
    t1 = rng.normal(size=3) * 0.05
    z1, i1 = render(sc, R1, t1, 8, 6, 6.5, 6.5, 4.0, 3.0)
    return z0.numpy(), i0.numpy(), z1.numpy(), i1.numpy(), R1, t1


def test_association_brute_force_8x6():
    """Every accepted pair links the current pixel to the model pixel whose
    centre is nearest to the projection, found by exhaustive search in float64."""
    z0, i0, z1, i1, R1, t1 = _frames_8x6()
    cur = pyr.build(z1, i1, 6.5, 6.5, 4.0, 3.0, 1)[0]
    ref = pyr.build(z0, i0, 6.5, 6.5, 4.0, 3.0, 1, with_gradient=True)[0]
    Da, ta = (R1 - np.eye(3)).astype(np.float32), t1.astype(np.float32)
    ok, iu, iv = assoc.icp_association(cur, ref, Da, ta)
    cells = np.stack(np.meshgrid(np.arange(8), np.arange(6)), -1).reshape(-1, 2).astype(np.float64)
    checked = 0
    for j in range(6):
        for i in range(8):
            p = cur["V"][j, i].astype(np.float64)
            if p[2] <= 0:
                assert not ok[j, i]
                continue
            q = R1 @ p + t1
            uv = np.array([6.5 * q[0] / q[2] + 4.0, 6.5 * q[1] / q[2] + 3.0])
            dist = np.abs(cells - uv).max(axis=1)
            best = int(np.argmin(dist))
            frac = np.abs(uv - np.round(uv))
            if np.any(np.abs(frac - 0.5) < 1e-4):
                continue  # too close to a tie to decide in float64 vs float32
            inside = np.all(uv > -0.5) and uv[0] < 7.5 and uv[1] < 5.5
            if ok[j, i]:
                assert inside and (iu[j, i], iv[j, i]) == tuple(cells[best].astype(int))
                checked += 1
    assert checked >= 10


def test_identical_frames_at_identity():
    """Same frame as model and current view, identity transforms: every ICP
    residual is exactly zero and the photometric ones vanish to float32
    round-trip accuracy."""
    d = tilted_plane_pair()
    cam = Camera(d["W"], d["H"], d["f"], d["f"], d["cx"], d["cy"])
    cur, ref = track.build_pyramids(d["z0"], d["I0"], d["z0"], d["I0"], cam, 1)
    x = identity_state()
    Ra, ta, Rb, tb = track.fp32_transforms(np.eye(4), x, x)
    assert not np.any(Ra) and not np.any(ta)  # R - I = 0 at identity
    p = _params()
    icp = res.icp_terms(cur[0], ref[0], np.eye(4), x, Ra, ta, p)
    ok, iu, iv = assoc.icp_association(cur[0], ref[0], Ra, ta)
    jj, ii = np.nonzero(ok)
    assert np.array_equal(iu[ok], ii) and np.array_equal(iv[ok], jj)
    assert icp["J"].shape[0] > 0.9 * (d["W"] - 1) * (d["H"] - 1)
    assert np.all(icp["e"] == 0.0)
    rgb = res.rgb_terms(cur[0], ref[0], x, x, Rb, tb, p)
    assert rgb["J"].shape[0] > 0.9 * (d["W"] - 3) * (d["H"] - 3)
    # back-projection to float32 vertices and re-projection in float64 moves a
    # pixel by at most a few float32 ulps of its coordinate: |e| <= |grad I|_1 4 ulp(W)
    bound = (0.75 + 0.5) * 4 * 2.0**-23 * max(d["W"], d["H"])
    assert np.abs(rgb["e"]).max() <= bound
    _, b, _, _ = res.normal_equations(rgb, np.r_[0:12], 12)
    assert np.all(np.abs(b) <= bound * (rgb["w"][:, None] * np.abs(rgb["J"])).sum(0))


def _fd_jacobians(cur, ref, x0, x1, rgb, icp, Ra, ta, T_WM, h=1e-6):
    mask = rgb["mask"]
    P = cur["V"][mask].astype(np.float64)
    I1 = cur["I"][mask].astype(np.float64)
    fx, fy, cx, cy = (float(k) for k in ref["K"])

    def e_rgb(a, b):
        R0, R1 = lie.quat_to_rot(a["q"]), lie.quat_to_rot(b["q"])
        x = (P @ R1.T + b["r"] - a["r"]) @ R0
        return res.bilinear(ref["I"], fx * x[:, 0] / x[:, 2] + cx, fy * x[:, 1] / x[:, 2] + cy) - I1

    ok, iu, iv = assoc.icp_association(cur, ref, Ra, ta)
    Pi = cur["V"][ok].astype(np.float64)
    v0 = ref["V"][iv[ok], iu[ok]].astype(np.float64) @ T_WM[:3, :3].T + T_WM[:3, 3]
    n0 = ref["N"][iv[ok], iu[ok]].astype(np.float64) @ T_WM[:3, :3].T

    def e_icp(b):
        return np.einsum("ij,ij->i", n0, Pi @ lie.quat_to_rot(b["q"]).T + b["r"] - v0)

    Jr, Ji = [], []
    for k in range(12):
        d = np.zeros(15)
        d[k % 6] = h
        if k < 6:
            Jr.append((e_rgb(lie.state_boxplus(x0, d), x1) - e_rgb(lie.state_boxplus(x0, -d), x1)) / (2 * h))
        else:
            Jr.append((e_rgb(x0, lie.state_boxplus(x1, d)) - e_rgb(x0, lie.state_boxplus(x1, -d))) / (2 * h))
            Ji.append((e_icp(lie.state_boxplus(x1, d)) - e_icp(lie.state_boxplus(x1, -d))) / (2 * h))
    return np.stack(Jr, 1), np.stack(Ji, 1)


def test_jacobians_match_central_differences():
    """On a linear-ramp reference image bilinear sampling and central-difference
    gradients are exact, so the analytic photometric Jacobian must equal the
    finite-difference derivative of the residual; likewise for ICP."""
    d = tilted_plane_pair()
    cam = Camera(d["W"], d["H"], d["f"], d["f"], d["cx"], d["cy"])
    cur, ref = track.build_pyramids(d["z1"], d["I1"], d["z0"], d["I0"], cam, 1)
    x0 = lie.state_boxplus(identity_state(), np.r_[2e-3, 1e-3, -1e-3, -1e-3, 2e-3, 1e-3, np.zeros(9)])
    x1 = {"r": d["r1"] + 1e-3, "q": quat_from_matrix(lie.exp_so3([1e-3, -2e-3, 1e-3]) @ d["R1"]),
          "v": np.zeros(3), "bg": np.zeros(3), "ba": np.zeros(3)}
    T_WM = np.eye(4)
    T_WM[:3, :3] = lie.exp_so3([0.002, -0.001, 0.003])
    T_WM[:3, 3] = [0.004, -0.002, 0.001]
    Ra, ta, Rb, tb = track.fp32_transforms(T_WM, x0, x1)
    p = _params()
    rgb = res.rgb_terms(cur[0], ref[0], x0, x1, Rb, tb, p)
    icp = res.icp_terms(cur[0], ref[0], T_WM, x1, Ra, ta, p)
    Jr, Ji = _fd_jacobians(cur[0], ref[0], x0, x1, rgb, icp, Ra, ta, T_WM)
    scale = np.abs(rgb["J"]).max(axis=1, keepdims=True)
    assert (np.abs(Jr - rgb["J"]) / scale).max() < 1e-4
    assert np.median(np.abs(Jr - rgb["J"]) / scale) < 1e-7
    assert np.abs(Ji - icp["J"]).max() < 1e-8


def test_normal_equations_symmetric_psd():
    d = tilted_plane_pair()
    cam = Camera(d["W"], d["H"], d["f"], d["f"], d["cx"], d["cy"])
    cur, ref = track.build_pyramids(d["z1"], d["I1"], d["z0"], d["I0"], cam, 1)
    x = identity_state()
    Ra, ta, Rb, tb = track.fp32_transforms(np.eye(4), x, x)
    vis = track.linearise_visual(cur[0], ref[0], np.eye(4), x, x, Ra, ta, Rb, tb, _params())
    for H in (vis["H_icp"], vis["H_rgb"]):
        assert np.allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())
        assert np.linalg.eigvalsh(H).min() >= -1e-12 * np.trace(H)
    # dense check: stacking the per-pixel rows gives the same system
    rgb = vis["rgb"]
    Jd = rgb["J"] * np.sqrt(rgb["w"])[:, None]
    assert np.allclose(Jd.T @ Jd, vis["H_rgb"], rtol=1e-12, atol=0)


def test_recovers_known_se3_offset():
    """Plane + ramp construction: the ground truth is an exact fixed point, and
    Gauss-Newton from identity must land on it (RGB-D-only mode, x0 fixed)."""
    d = tilted_plane_pair()
    cam = Camera(d["W"], d["H"], d["f"], d["f"], d["cx"], d["cy"])
    for huber in (1.345, 0.0):
        p = track.default_params(levels=2, iters=(10, 10), mode="rgbd")
        p["huber_k"] = huber
        out = track.track_frame(d["z1"], d["I1"], d["z0"], d["I0"], np.eye(4), cam, None, 0.0, 0.015,
                                identity_state(), None, None, p)
        assert out["status"] == "ok"
        assert np.linalg.norm(out["x1"]["r"] - d["r1"]) < 1e-6
        assert np.linalg.norm(lie.quat_boxminus(out["x1"]["q"], quat_from_matrix(d["R1"]))) < 1e-6


def test_huber_weight():
    s = np.array([0.0, 1.0, 1.345, 2.69, 13.45])
    assert np.allclose(res.huber_weight(s, 1.345), [1, 1, 1, 0.5, 0.1])
    assert np.all(res.huber_weight(s, 0.0) == 1)


def test_photometric_taps_lie_where_the_gradient_is_defined():
    """Every pixel the photometric term accepts (eq. (3)) samples I0 and its
    central-difference gradient at four taps that all have both neighbours
    in the image: on a linear ramp those taps carry the exact ramp slope,
    while the border pixels, whose central difference is undefined, carry
    the pyramid's 0.  Conversely, every pixel with valid depth in front of
    the reference camera whose four taps are interior is accepted (the rule
    is no stricter than the taps require).  Random warps push projections
    across all four borders."""
    d = tilted_plane_pair(W=48, H=36, seed=4, ramp=(0.75, 0.5, 10.0))
    cam = Camera(d["W"], d["H"], d["f"], d["f"], d["cx"], d["cy"])
    cur, ref = track.build_pyramids(d["z1"], d["I1"], d["z0"], d["I0"], cam, 1)
    G = ref[0]["G"]
    W, H = d["W"], d["H"]
    slope = np.array([0.75, 0.5], dtype=np.float32)
    interior = np.zeros((H, W), bool)
    interior[1:H - 1, 1:W - 1] = True
    assert np.all(G[interior] == slope) and np.all(G[~interior] == 0.0)
    rng = np.random.default_rng(8)
    x = identity_state()
    seen_reject = 0
    for trial in range(12):
        x1 = lie.state_boxplus(x, np.r_[rng.normal(size=3) * 0.08, rng.normal(size=3) * 0.06, np.zeros(9)])
        _, _, Rb, tb = track.fp32_transforms(np.eye(4), x, x1)
        ok, u, v = assoc.rgb_validity(cur[0], ref[0], Rb, tb)
        assert ok.sum() > 0
        fu, fv = np.floor(u[ok]).astype(np.int64), np.floor(v[ok]).astype(np.int64)
        for du in (0, 1):
            for dv in (0, 1):
                taps = G[fv + dv, fu + du]
                assert np.all(taps == slope), trial
        # converse: valid depth, point in front, all four taps interior
        qz = cur[0]["V"][..., 2] + (((Rb.reshape(3, 3)[2, 0] * cur[0]["V"][..., 0]
                                      + Rb.reshape(3, 3)[2, 1] * cur[0]["V"][..., 1])
                                     + Rb.reshape(3, 3)[2, 2] * cur[0]["V"][..., 2]) + tb[2])
        with np.errstate(invalid="ignore"):
            cand = (cur[0]["D"] > 0) & (qz > 0) & np.isfinite(u) & np.isfinite(v)
        fu_all = np.where(cand, np.floor(np.nan_to_num(u)), -10).astype(np.int64)
        fv_all = np.where(cand, np.floor(np.nan_to_num(v)), -10).astype(np.int64)
        taps_in = cand & (fu_all >= 1) & (fu_all + 1 <= W - 2) & (fv_all >= 1) & (fv_all + 1 <= H - 2)
        assert np.array_equal(ok, taps_in), trial
        seen_reject += int((cand & ~ok).sum())
    assert seen_reject > 0  # the warps did push pixels onto the border
