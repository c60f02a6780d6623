"""The C-ABI library loads, exports every declared entry point, and its host
float64 entry points (preintegration, Gauss-Newton step) match the oracle.
These run without a GPU: no device call is made."""
import os
import re

import numpy as np
import pytest

from oracle import imu, lie, solve
from synth.configs import initial_prior
from tests.test_oracle_imu import _rigid_motion_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dslam.h")

P = pytest.importorskip("paper_2207_10940_amd")


def _lib_or_skip():
    try:
        return P.lib()
    except RuntimeError as e:  # library not built in this checkout
        pytest.skip(str(e))


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dslam_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dslam_build_pyramid", "dslam_preintegrate_imu", "dslam_solve_step", "dslam_track_frame",
                     "dslam_track_frame_sync", "dslam_session_checkpoint", "dslam_session_restore",
                     "dslam_context_create", "dslam_session_open", "dslam_session_close", "dslam_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib_or_skip()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.dslam_build_info()


def test_status_strings():
    lib = _lib_or_skip()
    assert lib.dslam_status_string(0) == b"ok"
    assert lib.dslam_status_string(3) == b"singular system"
    assert lib.dslam_status_string(99) == b"unknown status"


def _noisy_case():
    c = _rigid_motion_case()
    rng = np.random.default_rng(0)
    c["gyro"] = c["gyro"] + rng.normal(size=c["gyro"].shape) * 0.05
    c["acc"] = c["acc"] + rng.normal(size=c["acc"].shape) * 0.2
    return c, rng


def test_host_preintegration_matches_oracle():
    _lib_or_skip()
    c, _ = _noisy_case()
    t0, t1 = 0.002, c["T"]
    bg, ba = c["x0"]["bg"] + 0.003, c["x0"]["ba"] - 0.01
    ip = P.imu_params(sigma_g=1e-3, sigma_a=1e-2, R_CS=c["params"]["R_CS"], t_CS=c["params"]["t_CS"])
    pc = P.preintegrate_imu(c["stamps"], c["gyro"], c["acc"], t0, t1, bg, ba, ip)
    po = imu.preintegrate(c["stamps"], c["gyro"], c["acc"], t0, t1, bg, ba, 1e-3, 1e-2)
    assert np.abs(pc["dR"] - po["dR"]).max() < 1e-14
    assert np.abs(pc["dv"] - po["dv"]).max() < 1e-14
    assert np.abs(pc["dp"] - po["dp"]).max() < 1e-15
    assert np.abs(pc["J"] - po["J"]).max() < 1e-10 * np.abs(po["J"]).max()
    assert np.abs(pc["Sigma"] - po["Sigma"]).max() < 1e-8 * np.abs(po["Sigma"]).max()


def test_host_preintegration_rejects_bad_samples():
    _lib_or_skip()
    ip = P.imu_params()
    st = np.array([0.0, 0.005, 0.004])
    with pytest.raises(P.DslamError):
        P.preintegrate_imu(st, np.zeros((3, 3)), np.zeros((3, 3)), 0.0, 0.01, np.zeros(3), np.zeros(3), ip)
    with pytest.raises(P.DslamError):  # first sample after t0
        P.preintegrate_imu(np.array([0.001]), np.zeros((1, 3)), np.zeros((1, 3)), 0.0, 0.01, np.zeros(3),
                           np.zeros(3), ip)


def test_host_solve_step_imu_and_prior_match_oracle():
    """Visual sums zero: the step is the IMU factor plus the prior.  The
    library's analytic IMU Jacobians and noise map must reproduce the
    oracle's finite-difference ones through the whole Gauss-Newton step and
    the Schur-complement prior."""
    _lib_or_skip()
    c, rng = _noisy_case()
    t0, t1 = 0.002, c["T"]
    params = {"gravity": 9.81, "R_CS": c["params"]["R_CS"], "t_CS": c["params"]["t_CS"], "sigma_bg_rw": 4e-6,
              "sigma_ba_rw": 2e-5}
    ip = P.imu_params(sigma_g=1e-3, sigma_a=1e-2, R_CS=c["params"]["R_CS"], t_CS=c["params"]["t_CS"])
    x0 = lie.state_boxplus(c["x0"], rng.normal(size=15) * 1e-3)
    x1 = lie.state_boxplus(c["x1"], rng.normal(size=15) * 1e-3)
    q = lie.quat_boxplus(c["q_IW"], rng.normal(size=3) * 1e-3)
    prior = initial_prior(c["x0"], c["q_IW"])
    prior["b"] = rng.normal(size=18) * 10
    po = imu.preintegrate(c["stamps"], c["gyro"], c["acc"], t0, t1, x0["bg"], x0["ba"], 1e-3, 1e-2)
    pc = P.preintegrate_imu(c["stamps"], c["gyro"], c["acc"], t0, t1, x0["bg"], x0["ba"], ip)
    e, J, W = imu.factor(x0, x1, q, po, params)
    H = J.T @ W @ J
    b = -J.T @ W @ e
    Hp, bp = solve.prior_terms(x0, q, prior)
    H += Hp
    b += bp
    dz_o = np.linalg.solve(H, b)
    tp = P.track_params(levels=1, iters=(1,), mode="rgbdi")
    a0, a1, qn, dz_c, mp = P.solve_step(np.zeros(58), np.eye(4), pc, ip, tp, prior, x0, x1, q, marginalise=True)
    # H has condition ~1e11 here (prior weights 1e8, IMU weights up to 1e10):
    # the oracle's own increment moves by ~3e-7 relative between finite-
    # difference steps 1e-4 and 1e-5, so that is the scale of agreement.
    tol = 1e-6 * np.abs(dz_o).max()
    assert np.abs(dz_c - dz_o).max() <= tol
    x0o, x1o, qo = solve.apply_update(x0, x1, q, dz_o)
    for k in ("r", "v", "bg", "ba"):
        assert np.abs(a1[k] - x1o[k]).max() < tol and np.abs(a0[k] - x0o[k]).max() < tol
    assert np.linalg.norm(lie.quat_boxminus(a1["q"], x1o["q"])) < tol
    mo = solve.marginalise(H, b, dz_o, x1o, qo)
    assert np.abs(mp["H"] - mo["H"]).max() < 1e-7 * np.abs(mo["H"]).max()
    # b* is rounding noise around zero at the updated point: compare on that scale
    assert np.abs(mp["b"] - mo["b"]).max() < 1e-12 * np.abs(H).max() * np.abs(dz_o).max()


def test_host_solve_step_rejects_bad_input():
    _lib_or_skip()
    x = {"r": np.zeros(3), "q": np.array([1.0, 0, 0, 0.1]), "v": np.zeros(3), "bg": np.zeros(3), "ba": np.zeros(3)}
    tp = P.track_params(levels=1, iters=(1,), mode="rgbd")
    with pytest.raises(P.DslamError):  # non-unit quaternion
        P.solve_step(np.zeros(58), np.eye(4), None, P.imu_params(), tp, None, x, x, np.array([1.0, 0, 0, 0]))


def test_host_solve_step_singular_without_information():
    _lib_or_skip()
    x = {"r": np.zeros(3), "q": np.array([1.0, 0, 0, 0]), "v": np.zeros(3), "bg": np.zeros(3), "ba": np.zeros(3)}
    tp = P.track_params(levels=1, iters=(1,), mode="rgbd")
    with pytest.raises(P.DslamError) as ei:
        P.solve_step(np.zeros(58), np.eye(4), None, P.imu_params(), tp, None, x, x, np.array([1.0, 0, 0, 0]))
    assert ei.value.code == 3


def test_binding_rejects_images_the_library_would_misread():
    """The C ABI takes plain device pointers (depth float32 metres, intensity uint8 grey levels, H x W with
    pitch = width); the binding refuses any other tensor before it reaches the library."""
    import torch
    z = torch.zeros((120, 160), dtype=torch.float32)
    i = torch.zeros((120, 160), dtype=torch.uint8)
    cases = [((z, i.float()), "dtype"), ((z.double(), i), "dtype"), ((z[:, :80], i), "contiguous"),
             ((z, i[:60]), "differ"), ((z.reshape(1, 120, 160), i), "H x W"), ((z.numpy(), i), "torch tensor")]
    for (a, b), what in cases:
        with pytest.raises(ValueError, match=what):
            P.check_images(a, b)
    with pytest.raises(ValueError, match="shape"):
        P.check_images(z, i, (200, 152))
    with pytest.raises(ValueError, match="CUDA"):  # right type and shape, host memory
        P.check_images(z, i, (160, 120))
    with pytest.raises(ValueError, match="dtype"):
        P.frame_input({"depth": z, "intensity": i.float(), "imu": None}, (160, 120))
