"""The per-frame tracking step (Sections IV-B to IV-E), oracle form.

At the arrival of frame 1 the step estimates x1 while refining x0 (Section
IV-A) by Gauss-Newton on the joint cost of eq. (6), coarse to fine over the
pyramid (Section IV-D), updating both states with box-plus after each
iteration, and finally marginalising x0 into the prior for the next frame
(Section IV-E).

Readings taken where the paper is silent:

* x1 starts at the IMU prediction from x0 (RGB-D-inertial mode) or at x0's
  pose with x0 held fixed (RGB-D-only mode, the paper's baseline system);
* gyro-only mode (the paper's variant without the accelerometer residuals):
  only the rotation residual and the gyro-bias random walk of the IMU factor
  remain; the entries no remaining term constrains (velocities, accelerometer
  biases, gravity direction) are held fixed, their rows and columns of the
  normal equations replaced by the identity with a zero right-hand side
  (the same solution as the system without them); x1 starts at x0 rotated by
  the gyro-integrated rotation;
* the IMU and prior terms are added at every iteration of every level;
* a fixed number of iterations per level, no damping, no early exit;
* the float32 transforms that drive association are the float64 compositions
  T_WM^-1 T_WC1 (ICP) and T_WC0^-1 T_WC1 (photometric), their rotations kept
  as R - I, rounded once to float32;
* health of the frame (not in the paper): tracking is lost when the finest
  level's last pass has fewer inliers of both terms than min_inlier_frac of
  twice its pixels, when its visual cost exceeds (1 + max_cost_rise) times
  its first pass's, or when a cost or state is not finite;
* with imu_fallback (RGB-D-inertial mode), a lost frame is re-estimated
  without its visual terms: one Gauss-Newton step of the prior and the IMU
  factor (Sections IV-C, IV-E) from the frame's start state x0, the IMU
  prediction of x1 and the start q_IW, marginalised at the result.
"""
from __future__ import annotations

import numpy as np

from . import imu as imu_mod
from . import pyramid as pyr
from . import residuals as res
from . import solve as slv
from .lie import copy_state, quat_to_rot, state_boxplus


def default_params(levels=3, iters=(10, 5, 4), mode="rgbdi"):
    return {
        "levels": levels, "iters": list(iters), "mode": mode,
        "min_inlier_frac": 0.05, "max_cost_rise": 0.5, "imu_fallback": False,
        "depth_k": 1e-3, "sigma_I": 4.0, "huber_k": 1.345, "icp_dist": 0.10, "icp_cos": None,
        "sigma_g": 1.7e-4, "sigma_a": 2.0e-3, "sigma_bg_rw": 4.0e-6, "sigma_ba_rw": 2.0e-5,
        "gravity": 9.81, "R_CS": np.eye(3), "t_CS": np.zeros(3),
    }


def fp32_transforms(T_WM, x0, x1):
    """(R_a - I, t_a) of T_WM^-1 T_WC1 and (R_b - I, t_b) of T_WC0^-1 T_WC1,
    formed in float64 and rounded once to float32."""
    R_WM, t_WM = T_WM[:3, :3], T_WM[:3, 3]
    R0, R1 = quat_to_rot(x0["q"]), quat_to_rot(x1["q"])
    Ra = R_WM.T @ R1
    ta = R_WM.T @ (x1["r"] - t_WM)
    Rb = R0.T @ R1
    tb = R0.T @ (x1["r"] - x0["r"])
    f = np.float32
    return (Ra - np.eye(3)).astype(f), ta.astype(f), (Rb - np.eye(3)).astype(f), tb.astype(f)


def linearise_visual(cur, ref, T_WM, x0, x1, Ra, ta, Rb, tb, params):
    """Visual normal equations over [pose0 (6), pose1 (6)], per term."""
    icp = res.icp_terms(cur, ref, T_WM, x1, Ra, ta, params)
    rgb = res.rgb_terms(cur, ref, x0, x1, Rb, tb, params)
    Hi, bi, ci, ni = res.normal_equations(icp, np.r_[6:12], 12)
    Hr, br, cr, nr = res.normal_equations(rgb, np.r_[0:12], 12)
    return {"H_icp": Hi, "b_icp": bi, "cost_icp": ci, "n_icp": ni, "mask_icp": icp["mask"],
            "H_rgb": Hr, "b_rgb": br, "cost_rgb": cr, "n_rgb": nr, "mask_rgb": rgb["mask"],
            "icp": icp, "rgb": rgb}


def build_pyramids(depth, intensity, model_depth, model_intensity, camera, levels):
    fx, fy, cx, cy = camera.fx, camera.fy, camera.cx, camera.cy
    cur = pyr.build(depth, intensity, fx, fy, cx, cy, levels)
    ref = pyr.build(model_depth, model_intensity, fx, fy, cx, cy, levels, with_gradient=True)
    return cur, ref


def track_frame(depth, intensity, model_depth, model_intensity, T_WM, camera, imu, t0, t1, x0, q_IW, prior,
                params, *, x1_init=None, record=False):
    """One tracking step.  Returns a dict with x0, x1, q_IW, prior (new), status and per-iteration logs."""
    levels = params["levels"]
    cur, ref = build_pyramids(depth, intensity, model_depth, model_intensity, camera, levels)
    mode = params["mode"]
    x0 = copy_state(x0)
    q_IW = np.array(q_IW, dtype=np.float64)
    pre = None
    if mode != "rgbd":
        pre = imu_mod.preintegrate(imu["t"], imu["gyro"], imu["acc"], t0, t1, x0["bg"], x0["ba"],
                                   params["sigma_g"], params["sigma_a"])
    if x1_init is not None:
        x1 = copy_state(x1_init)
    elif mode == "rgbd":
        x1 = copy_state(x0)
    elif mode == "gyro":
        x1 = imu_mod.predict_state_gyro(x0, pre, params)
    else:
        x1 = imu_mod.predict_state(x0, q_IW, pre, params)
    start = (copy_state(x0), copy_state(x1), q_IW.copy())  # the frame's start and the prediction of x1
    finest = min(l for l in range(levels) if params["iters"][l] > 0)
    cost_first = cost_last = None
    n_last = 0
    log = []
    H = b = dz = None
    status = "ok"
    for lvl in reversed(range(levels)):
        for it in range(params["iters"][lvl]):
            Ra, ta, Rb, tb = fp32_transforms(T_WM, x0, x1)
            vis = linearise_visual(cur[lvl], ref[lvl], T_WM, x0, x1, Ra, ta, Rb, tb, params)
            if lvl == finest:
                cost_last = vis["cost_icp"] + vis["cost_rgb"]
                cost_first = cost_last if it == 0 else cost_first
                n_last = vis["n_icp"] + vis["n_rgb"]
            if mode == "rgbd":
                Hv = vis["H_icp"] + vis["H_rgb"]
                bv = vis["b_icp"] + vis["b_rgb"]
                H6, b6 = Hv[6:12, 6:12], bv[6:12]
                if not slv.is_spd(H6):
                    status = "singular"
                    break
                d6 = np.linalg.solve(H6, b6)
                x1 = state_boxplus(x1, np.concatenate([d6, np.zeros(9)]))
                H = b = None
                dz = d6
            else:
                H = np.zeros((33, 33))
                b = np.zeros(33)
                idx = np.r_[0:6, 15:21]
                H[np.ix_(idx, idx)] += vis["H_icp"] + vis["H_rgb"]
                b[idx] += vis["b_icp"] + vis["b_rgb"]
                if mode == "gyro":
                    e, J, W = imu_mod.factor_gyro(x0, x1, q_IW, pre, params)
                else:
                    e, J, W = imu_mod.factor(x0, x1, q_IW, pre, params)
                H += J.T @ W @ J
                b += -(J.T @ W @ e)
                Hp, bp = slv.prior_terms(x0, q_IW, prior)
                H += Hp
                b += bp
                if mode == "gyro":
                    fixed = imu_mod.GYRO_FIXED
                    H[fixed, :] = 0.0
                    H[:, fixed] = 0.0
                    H[fixed, fixed] = 1.0
                    b[fixed] = 0.0
                if not slv.is_spd(H):
                    status = "singular"
                    break
                dz = slv.gn_step(H, b)
                x0, x1, q_IW = slv.apply_update(x0, x1, q_IW, dz)
            if record:
                log.append({"level": lvl, "iter": it, "Ra": Ra, "ta": ta, "Rb": Rb, "tb": tb,
                            "n_icp": vis["n_icp"], "n_rgb": vis["n_rgb"], "cost_icp": vis["cost_icp"],
                            "cost_rgb": vis["cost_rgb"], "H_icp": vis["H_icp"], "b_icp": vis["b_icp"],
                            "H_rgb": vis["H_rgb"], "b_rgb": vis["b_rgb"], "dz": dz.copy(),
                            "mask_icp": vis["mask_icp"], "mask_rgb": vis["mask_rgb"]})
        if status != "ok":
            break
    new_prior = None
    if status == "ok" and mode != "rgbd":
        new_prior = slv.marginalise(H, b, dz, x1, q_IW)
    health = []
    if status == "ok":
        npix = cur[finest]["D"].size
        if params.get("min_inlier_frac", 0.0) > 0.0 and n_last < params["min_inlier_frac"] * 2.0 * npix:
            health.append("low_inliers")
        states = np.concatenate([np.concatenate([np.ravel(x[k]) for k in ("r", "q", "v", "bg", "ba")])
                                 for x in (x0, x1)] + [np.ravel(q_IW)])
        if not (np.all(np.isfinite(states)) and np.isfinite(cost_last)):
            health.append("nonfinite")
        if params.get("max_cost_rise", 0.0) > 0.0 and cost_last > (1.0 + params["max_cost_rise"]) * cost_first:
            health.append("cost_up")
    if health and mode == "rgbdi" and params.get("imu_fallback"):
        x0f, x1f, qf = copy_state(start[0]), copy_state(start[1]), start[2].copy()
        e, J, W = imu_mod.factor(x0f, x1f, qf, pre, params)
        Hf = J.T @ W @ J
        bf = -(J.T @ W @ e)
        Hp, bp = slv.prior_terms(x0f, qf, prior)
        Hf = Hf + Hp
        bf = bf + bp
        if slv.is_spd(Hf):
            dzf = slv.gn_step(Hf, bf)
            x0, x1, q_IW = slv.apply_update(x0f, x1f, qf, dzf)
            new_prior = slv.marginalise(Hf, bf, dzf, x1, q_IW)
            health.append("imu_only")
        else:
            health.append("singular")
    return {"x0": x0, "x1": x1, "q_IW": q_IW, "prior": new_prior, "status": status, "preint": pre, "log": log,
            "health": health}
