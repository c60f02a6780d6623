"""ctypes mirror of include/dslam.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

MAX_LEVELS = 4
MAX_IMU_SAMPLES = 32

OK, ERR_INVALID, ERR_NO_CAPACITY, ERR_SINGULAR, ERR_DEVICE, ERR_BUSY, ERR_NOT_READY = range(7)
MODE_RGBDI, MODE_RGBD, MODE_GYRO = 0, 1, 2
JAC_FP32, JAC_FP32_MFMA, JAC_FP16, JAC_BF16 = 0, 1, 2, 3
PYR_CURRENT, PYR_MODEL = 0, 1
HEALTH_LOW_INLIERS, HEALTH_NONFINITE, HEALTH_COST_UP, HEALTH_SINGULAR, HEALTH_IMU_ONLY = 1, 2, 4, 8, 16
CH_VX, CH_VY, CH_VZ, CH_NX, CH_NY, CH_NZ, CH_I, CH_GX, CH_GY = range(9)


class FrameState(C.Structure):
    _fields_ = [("r", C.c_double * 3), ("q", C.c_double * 4), ("v", C.c_double * 3), ("bg", C.c_double * 3),
                ("ba", C.c_double * 3)]


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


class ImuParams(C.Structure):
    _fields_ = [("sigma_g", C.c_double), ("sigma_a", C.c_double), ("sigma_bg_rw", C.c_double),
                ("sigma_ba_rw", C.c_double), ("gravity", C.c_double), ("R_CS", C.c_double * 9),
                ("t_CS", C.c_double * 3)]


class TrackParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("iters", C.c_int32 * MAX_LEVELS), ("icp_dist", C.c_double),
                ("icp_cos", C.c_double), ("sigma_I", C.c_double), ("depth_k", C.c_double), ("huber_k", C.c_double),
                ("jac_format", C.c_int32), ("mode", C.c_int32), ("min_inlier_frac", C.c_double),
                ("max_cost_rise", C.c_double), ("imu_fallback", C.c_int32)]


class ImuSample(C.Structure):
    _fields_ = [("t", C.c_double), ("gyro", C.c_double * 3), ("acc", C.c_double * 3)]


class Preint(C.Structure):
    _fields_ = [("dR", C.c_double * 9), ("dv", C.c_double * 3), ("dp", C.c_double * 3), ("dt", C.c_double),
                ("bg", C.c_double * 3), ("ba", C.c_double * 3), ("J", C.c_double * 54), ("Sigma", C.c_double * 81)]


class Prior(C.Structure):
    _fields_ = [("H", C.c_double * 324), ("b", C.c_double * 18), ("xbar", FrameState), ("q_IW_bar", C.c_double * 4)]


class TrackResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("frame_index", C.c_int32), ("health", C.c_int32),
                ("tracking_lost", C.c_int32), ("x0", FrameState), ("x1", FrameState),
                ("q_IW", C.c_double * 4), ("cost_icp", C.c_double), ("cost_rgb", C.c_double),
                ("cost_imu", C.c_double), ("cost_prior", C.c_double), ("n_icp", C.c_int64 * MAX_LEVELS),
                ("n_rgb", C.c_int64 * MAX_LEVELS), ("last_step_norm", C.c_double), ("prior", Prior)]


class LinearSystem(C.Structure):
    _fields_ = [("H_icp", C.c_double * 144), ("b_icp", C.c_double * 12), ("cost_icp", C.c_double),
                ("n_icp", C.c_int64), ("H_rgb", C.c_double * 144), ("b_rgb", C.c_double * 12),
                ("cost_rgb", C.c_double), ("n_rgb", C.c_int64), ("raw", C.c_double * 58)]


class TuneEntry(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("level", C.c_int32), ("jac_format", C.c_int32),
                ("ppt", C.c_int32), ("us", C.c_float), ("xcd_banded", C.c_int32)]


class FrameInput(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("intensity", C.c_void_p), ("pitch", C.c_int32),
                ("model_depth", C.c_void_p), ("model_intensity", C.c_void_p), ("model_pitch", C.c_int32),
                ("T_WM", C.c_double * 16), ("imu", C.POINTER(ImuSample)), ("n_imu", C.c_int32),
                ("t0", C.c_double), ("t1", C.c_double)]


class ServerParams(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("pipeline_depth", C.c_int32), ("use_graphs", C.c_int32)]


class RequestDone(C.Structure):
    _fields_ = [("request_id", C.c_uint64), ("session", C.c_void_p), ("submit_s", C.c_double),
                ("launch_s", C.c_double), ("done_s", C.c_double), ("device_ms", C.c_float),
                ("batch_size", C.c_int32), ("result", TrackResult)]


MAX_BATCH = 256
MAX_BATCH_RESOLUTIONS = 16

P = C.POINTER
vp = C.c_void_p
dp = P(C.c_double)
fp = P(C.c_float)

class MapParams(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("assoc_dist", C.c_float), ("assoc_cos", C.c_float),
                ("render_band", C.c_float)]


class DeformProblem(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("nodes", C.POINTER(C.c_double)), ("n_con", C.c_int32),
                ("con", C.POINTER(C.c_double)), ("n_pin", C.c_int32), ("pin", C.POINTER(C.c_double)),
                ("n_rel", C.c_int32), ("rel", C.POINTER(C.c_double)), ("global_", C.c_int32),
                ("g_W", C.c_double * 3)]


SIGNATURES = {
    "dslam_status_string": (C.c_char_p, [C.c_int]),
    "dslam_build_info": (C.c_char_p, []),
    "dslam_context_create": (C.c_int, [C.c_int32, C.c_uint64, P(vp)]),
    "dslam_context_destroy": (C.c_int, [vp]),
    "dslam_context_used_bytes": (C.c_uint64, [vp]),
    "dslam_session_bytes": (C.c_uint64, [P(Camera), C.c_int32]),
    "dslam_session_open": (C.c_int, [vp, P(Camera), P(TrackParams), P(ImuParams), P(FrameState), dp, P(Prior),
                                     P(vp)]),
    "dslam_session_close": (C.c_int, [vp]),
    "dslam_build_pyramid": (C.c_int, [vp, C.c_int32, vp, vp, C.c_int32, dp, vp]),
    "dslam_preintegrate_imu": (C.c_int, [P(ImuSample), C.c_int32, C.c_double, C.c_double, dp, dp, P(ImuParams),
                                         P(Preint)]),
    "dslam_solve_step": (C.c_int, [dp, dp, P(Preint), P(ImuParams), P(TrackParams), P(Prior), P(FrameState),
                                   P(FrameState), dp, dp, P(Prior)]),
    "dslam_track_frame": (C.c_int, [vp, P(FrameInput), P(TrackResult), vp]),
    "dslam_track_frame_sync": (C.c_int, [vp, P(FrameInput), P(TrackResult), vp]),
    "dslam_session_checkpoint": (C.c_int, [vp, vp, C.c_uint64, P(C.c_uint64)]),
    "dslam_session_restore": (C.c_int, [vp, vp, C.c_uint64]),
    "dslam_session_result": (C.c_int, [vp, P(TrackResult)]),
    "dslam_linearize": (C.c_int, [vp, C.c_int32, fp, fp, fp, fp, P(FrameState), P(FrameState), vp,
                                  P(LinearSystem), vp]),
    "dslam_copy_pyramid": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32, fp]),
    "dslam_profile_residual": (C.c_int, [vp, C.c_int32, C.c_int32, vp]),
    "dslam_session_get_state": (C.c_int, [vp, P(FrameState), dp, P(Prior), P(C.c_int32)]),
    "dslam_session_set_state": (C.c_int, [vp, P(FrameState), dp, P(Prior), C.c_int32]),
    "dslam_context_autotune": (C.c_int, [vp, P(Camera), C.c_int32, C.c_int32, C.c_int32, vp, P(TuneEntry),
                                         C.c_int32, P(C.c_int32)]),
    "dslam_context_set_tune": (C.c_int, [vp, P(TuneEntry), C.c_int32]),
    "dslam_batch_create": (C.c_int, [vp, C.c_int32, P(vp)]),
    "dslam_batch_destroy": (C.c_int, [vp]),
    "dslam_batch_track": (C.c_int, [vp, C.c_int32, P(vp), P(FrameInput), vp]),
    "dslam_session_set_graphs": (C.c_int, [vp, C.c_int32]),
    "dslam_batch_results": (C.c_int, [vp, P(TrackResult)]),
    "dslam_batch_set_graphs": (C.c_int, [vp, C.c_int32]),
    "dslam_batch_set_tile_order": (C.c_int, [vp, C.c_int32]),
    "dslam_batch_track_noalloc": (C.c_int, [C.c_int32, P(vp), P(FrameInput), P(TrackResult), vp]),
    "dslam_batch_profile_residual": (C.c_int, [vp, C.c_int32, C.c_int32, vp, P(C.c_uint64)]),
    "dslam_server_create": (C.c_int, [vp, P(ServerParams), P(vp)]),
    "dslam_server_destroy": (C.c_int, [vp]),
    "dslam_server_submit": (C.c_int, [vp, vp, P(FrameInput), P(C.c_uint64)]),
    "dslam_server_poll": (C.c_int, [vp, C.c_int32, P(RequestDone), C.c_int32, P(C.c_int32)]),
    "dslam_server_counts": (C.c_int, [vp, P(C.c_int32), P(C.c_int32)]),
    "dslam_server_clock": (C.c_double, []),
    "dslam_map_create": (C.c_int, [vp, P(Camera), P(MapParams), P(vp)]),
    "dslam_map_destroy": (C.c_int, [vp]),
    "dslam_map_reset": (C.c_int, [vp, vp]),
    "dslam_map_fuse": (C.c_int, [vp, vp, dp, vp]),
    "dslam_map_predict": (C.c_int, [vp, vp, dp, vp]),
    "dslam_map_render": (C.c_int, [vp, dp, vp, vp, vp]),
    "dslam_map_count": (C.c_int, [vp, P(C.c_int32), P(C.c_int32)]),
    "dslam_map_copy": (C.c_int, [vp, C.c_int32, fp, C.c_int32]),
    "dslam_map_deform": (C.c_int, [vp, C.c_int32, dp, dp, vp]),
    "dslam_deform_create": (C.c_int, [vp, C.c_int32, C.c_int32, P(vp)]),
    "dslam_deform_destroy": (C.c_int, [vp]),
    "dslam_deform_solve": (C.c_int, [vp, P(DeformProblem), C.c_int32, dp, dp, vp]),
}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdslam.so")
_lib = None


def load():
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2207_10940_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
