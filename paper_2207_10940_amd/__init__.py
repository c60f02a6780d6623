"""MI355X (gfx950) dense RGB-D-inertial tracking: Python binding of libdslam.so.

Every step of the tracking path runs in the HIP library behind the C ABI of
include/dslam.h; this module only marshals arguments (torch CUDA tensors for
device images, numpy arrays and dicts for host-side states).  There is no
fallback: if the library is missing every call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import (CH_GX, CH_GY, CH_I, CH_NX, CH_NY, CH_NZ, CH_VX, CH_VY, CH_VZ, HEALTH_COST_UP, HEALTH_LOW_INLIERS,
                   HEALTH_IMU_ONLY, HEALTH_NONFINITE, HEALTH_SINGULAR, JAC_BF16, JAC_FP16, JAC_FP32, JAC_FP32_MFMA, MODE_GYRO, MODE_RGBD,
                   MODE_RGBDI, PYR_CURRENT, PYR_MODEL)

__all__ = ["DslamError", "Context", "Session", "Map", "Deform", "Batch", "Server", "check_images", "frame_input", "preintegrate_imu", "solve_step", "track_params", "imu_params",
           "camera", "state_struct", "state_dict", "prior_struct", "prior_dict", "lib"]

MODES = {"rgbdi": MODE_RGBDI, "rgbd": MODE_RGBD, "gyro": MODE_GYRO}
JAC = {"fp32": JAC_FP32, "fp32_mfma": JAC_FP32_MFMA, "fp16": JAC_FP16, "bf16": JAC_BF16}


class DslamError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().dslam_status_string(code).decode()} ({code})")


def lib():
    return _abi.load()


def _check(code, where):
    if code != _abi.OK:
        raise DslamError(code, where)


# --- struct conversion --------------------------------------------------------

def state_struct(x: dict) -> _abi.FrameState:
    s = _abi.FrameState()
    for k in ("r", "q", "v", "bg", "ba"):
        getattr(s, k)[:] = [float(v) for v in np.asarray(x[k], dtype=np.float64)]
    return s


def state_dict(s: _abi.FrameState) -> dict:
    return {k: np.array(getattr(s, k)[:], dtype=np.float64) for k in ("r", "q", "v", "bg", "ba")}


def prior_struct(p: dict) -> _abi.Prior:
    s = _abi.Prior()
    s.H[:] = [float(v) for v in np.asarray(p["H"], dtype=np.float64).ravel()]
    s.b[:] = [float(v) for v in np.asarray(p["b"], dtype=np.float64)]
    s.xbar = state_struct(p["xbar"])
    s.q_IW_bar[:] = [float(v) for v in p["qIW_bar"]]
    return s


def prior_dict(s: _abi.Prior) -> dict:
    return {"H": np.array(s.H[:]).reshape(18, 18), "b": np.array(s.b[:]), "xbar": state_dict(s.xbar),
            "qIW_bar": np.array(s.q_IW_bar[:])}


def camera(cam) -> _abi.Camera:
    return _abi.Camera(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy))


def track_params(levels=3, iters=(10, 5, 4), mode="rgbdi", jac="fp32", icp_dist=0.10, icp_cos=None,
                 sigma_I=4.0, depth_k=1e-3, huber_k=1.345, min_inlier_frac=0.05,
                 max_cost_rise=0.5, imu_fallback=False) -> _abi.TrackParams:
    p = _abi.TrackParams()
    p.levels = levels
    its = list(iters) + [0] * (_abi.MAX_LEVELS - len(iters))
    p.iters[:] = its[:_abi.MAX_LEVELS]
    p.icp_dist = icp_dist
    p.icp_cos = -2.0 if icp_cos is None else float(icp_cos)  # None: no normal-compatibility gate
    p.sigma_I = sigma_I
    p.depth_k = depth_k
    p.huber_k = huber_k
    p.jac_format = JAC[jac] if isinstance(jac, str) else int(jac)
    p.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    p.min_inlier_frac = min_inlier_frac
    p.max_cost_rise = max_cost_rise
    p.imu_fallback = int(bool(imu_fallback))
    return p


def imu_params(sigma_g=1.7e-4, sigma_a=2.0e-3, sigma_bg_rw=4.0e-6, sigma_ba_rw=2.0e-5, gravity=9.81,
               R_CS=np.eye(3), t_CS=np.zeros(3)) -> _abi.ImuParams:
    p = _abi.ImuParams()
    p.sigma_g, p.sigma_a, p.sigma_bg_rw, p.sigma_ba_rw, p.gravity = sigma_g, sigma_a, sigma_bg_rw, sigma_ba_rw, gravity
    p.R_CS[:] = [float(v) for v in np.asarray(R_CS, dtype=np.float64).ravel()]
    p.t_CS[:] = [float(v) for v in np.asarray(t_CS, dtype=np.float64)]
    return p


def imu_samples(stamps, gyro, acc):
    n = len(stamps)
    arr = (_abi.ImuSample * max(n, 1))()
    for k in range(n):
        arr[k].t = float(stamps[k])
        arr[k].gyro[:] = [float(v) for v in gyro[k]]
        arr[k].acc[:] = [float(v) for v in acc[k]]
    return arr, n


def _dptr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def check_images(depth, intensity, size=None, what="frame"):
    """Device images as the C ABI takes them: depth float32 (metres) and intensity uint8 (grey levels), both
    H x W, C-contiguous CUDA tensors whose row pitch is their width; size = (width, height) when the camera
    is known.  The library gets plain pointers and cannot check a buffer's type or extent, so a mismatch
    raises ValueError here, before anything is enqueued."""
    import torch
    for name, t, dt in (("depth", depth, torch.float32), ("intensity", intensity, torch.uint8)):
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{what} {name}: expected a torch tensor, got {type(t).__name__}")
        if t.dtype != dt:
            raise ValueError(f"{what} {name}: dtype {t.dtype}, expected {dt}")
        if t.dim() != 2:
            raise ValueError(f"{what} {name}: {t.dim()}-d tensor, expected H x W")
        if size is not None and tuple(t.shape) != (int(size[1]), int(size[0])):
            raise ValueError(f"{what} {name}: shape {tuple(t.shape)}, expected {(int(size[1]), int(size[0]))}")
        if not t.is_contiguous():
            raise ValueError(f"{what} {name}: not contiguous")
    if tuple(depth.shape) != tuple(intensity.shape):
        raise ValueError(f"{what}: depth {tuple(depth.shape)} and intensity {tuple(intensity.shape)} differ")
    for name, t in (("depth", depth), ("intensity", intensity)):
        if not t.is_cuda:
            raise ValueError(f"{what} {name}: not a CUDA (device) tensor")


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))


# --- host entry points ----------------------------------------------------------

def preintegrate_imu(stamps, gyro, acc, t0, t1, bg, ba, ip: _abi.ImuParams) -> dict:
    arr, n = imu_samples(stamps, gyro, acc)
    _, bgp = _dptr(bg)
    _, bap = _dptr(ba)
    out = _abi.Preint()
    _check(lib().dslam_preintegrate_imu(arr, n, float(t0), float(t1), bgp, bap, C.byref(ip), C.byref(out)),
           "dslam_preintegrate_imu")
    return {"dR": np.array(out.dR[:]).reshape(3, 3), "dv": np.array(out.dv[:]), "dp": np.array(out.dp[:]),
            "dt": out.dt, "bg": np.array(out.bg[:]), "ba": np.array(out.ba[:]),
            "J": np.array(out.J[:]).reshape(9, 6), "Sigma": np.array(out.Sigma[:]).reshape(9, 9), "_struct": out}


def preint_struct(pre: dict) -> _abi.Preint:
    if "_struct" in pre:
        return pre["_struct"]
    s = _abi.Preint()
    s.dR[:] = list(np.asarray(pre["dR"]).ravel())
    s.dv[:] = list(pre["dv"])
    s.dp[:] = list(pre["dp"])
    s.dt = float(pre["dt"])
    s.bg[:] = list(pre["bg"])
    s.ba[:] = list(pre["ba"])
    s.J[:] = list(np.asarray(pre["J"]).ravel())
    s.Sigma[:] = list(np.asarray(pre["Sigma"]).ravel())
    return s


def solve_step(raw, T_WM, pre, ip, tp, prior, x0, x1, q_IW, marginalise=False):
    """Host float64 Gauss-Newton step; returns (x0, x1, q_IW, dz, new_prior or None)."""
    _, rawp = _dptr(raw)
    _, Tp = _dptr(np.asarray(T_WM).ravel())
    a, b = state_struct(x0), state_struct(x1)
    q = np.ascontiguousarray(q_IW, dtype=np.float64).copy()
    dz = np.zeros(33)
    m = _abi.Prior() if marginalise else None
    pre_s = preint_struct(pre) if pre is not None else None
    prior_s = prior_struct(prior) if prior is not None else None
    code = lib().dslam_solve_step(rawp, Tp, C.byref(pre_s) if pre_s else None, C.byref(ip), C.byref(tp),
                                  C.byref(prior_s) if prior_s else None, C.byref(a), C.byref(b),
                                  q.ctypes.data_as(C.POINTER(C.c_double)), dz.ctypes.data_as(C.POINTER(C.c_double)),
                                  C.byref(m) if m is not None else None)
    _check(code, "dslam_solve_step")
    return state_dict(a), state_dict(b), q, dz, (prior_dict(m) if m is not None else None)


def result_dict(r: _abi.TrackResult) -> dict:
    return {"status": r.status, "frame_index": r.frame_index, "health": r.health,
            "tracking_lost": bool(r.tracking_lost), "x0": state_dict(r.x0), "x1": state_dict(r.x1),
            "q_IW": np.array(r.q_IW[:]), "cost_icp": r.cost_icp, "cost_rgb": r.cost_rgb, "cost_imu": r.cost_imu,
            "n_icp": list(r.n_icp), "n_rgb": list(r.n_rgb), "last_step_norm": r.last_step_norm,
            "prior": prior_dict(r.prior)}


# --- device objects ----------------------------------------------------------------

class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib().dslam_context_create(int(device), int(hbm_budget_bytes), C.byref(h)), "dslam_context_create")
        self.handle = h
        self.device = device

    def used_bytes(self) -> int:
        return int(lib().dslam_context_used_bytes(self.handle))

    def autotune(self, cams, levels=3, jac="fp32", stream=None) -> list:
        """Tile-shape autotuner (dslam_context_autotune); returns the chosen entries as dicts."""
        cs = [camera(c) if not isinstance(c, _abi.Camera) else c for c in cams]
        arr = (_abi.Camera * len(cs))(*cs)
        cap = len(cs) * _abi.MAX_LEVELS
        out = (_abi.TuneEntry * cap)()
        n = C.c_int32()
        jf = JAC[jac] if isinstance(jac, str) else int(jac)
        _check(lib().dslam_context_autotune(self.handle, arr, len(cs), int(levels), jf, _stream_ptr(stream), out, cap,
                                            C.byref(n)), "dslam_context_autotune")
        return [{"width": e.width, "height": e.height, "level": e.level, "jac_format": e.jac_format, "ppt": e.ppt,
                 "xcd_banded": e.xcd_banded, "us": e.us} for e in out[:n.value]]

    def set_tune(self, entries):
        """dslam_context_set_tune: record launch shapes (dicts as autotune returns them)."""
        arr = (_abi.TuneEntry * len(entries))()
        for i, e in enumerate(entries):
            jf = JAC[e["jac_format"]] if isinstance(e["jac_format"], str) else int(e["jac_format"])
            arr[i] = _abi.TuneEntry(int(e["width"]), int(e["height"]), int(e["level"]), jf, int(e["ppt"]),
                                    float(e.get("us", 0.0)), int(e.get("xcd_banded", 0)))
        _check(lib().dslam_context_set_tune(self.handle, arr, len(entries)), "dslam_context_set_tune")

    def close(self):
        if self.handle:
            _check(lib().dslam_context_destroy(self.handle), "dslam_context_destroy")
            self.handle = None


def session_bytes(cam, levels) -> int:
    c = camera(cam) if not isinstance(cam, _abi.Camera) else cam
    return int(lib().dslam_session_bytes(C.byref(c), int(levels)))


class Session:
    """One tracking session (device-resident pyramids and estimator state)."""

    def __init__(self, ctx: Context, cam, tp: _abi.TrackParams, ip: _abi.ImuParams, x0: dict, q_IW, prior=None):
        self.cam = camera(cam) if not isinstance(cam, _abi.Camera) else cam
        self.tp, self.ip = tp, ip
        h = C.c_void_p()
        xs = state_struct(x0)
        q, qp = _dptr(q_IW)
        ps = prior_struct(prior) if prior is not None else None
        _check(lib().dslam_session_open(ctx.handle, C.byref(self.cam), C.byref(tp), C.byref(ip), C.byref(xs), qp,
                                        C.byref(ps) if ps is not None else None, C.byref(h)), "dslam_session_open")
        self.handle = h
        self.ctx = ctx

    def close(self):
        if self.handle:
            _check(lib().dslam_session_close(self.handle), "dslam_session_close")
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def build_pyramid(self, which, depth, intensity, T_W_ref=None, stream=None):
        check_images(depth, intensity, (self.cam.width, self.cam.height), "pyramid")
        T = None
        if T_W_ref is not None:
            T, Tp = _dptr(np.asarray(T_W_ref).ravel())
        _check(lib().dslam_build_pyramid(self.handle, int(which), C.c_void_p(depth.data_ptr()),
                                         C.c_void_p(intensity.data_ptr()), int(depth.shape[1]),
                                         Tp if T is not None else None, _stream_ptr(stream)), "dslam_build_pyramid")

    def set_model(self, depth, intensity, T_WM, stream=None):
        self.build_pyramid(PYR_MODEL, depth, intensity, T_WM, stream)

    def track_frame(self, depth, intensity, imu=None, t0=0.0, t1=0.0, stream=None, out=None):
        """Enqueue one tracking step against the session's MODEL pyramid; imu = dict(t, gyro, acc) of the
        samples covering [t0, t1).  out: optional TrackResult (pinned host memory for a fully asynchronous
        copy) that receives the result once the stream passes the frame."""
        self.track_frame_input({"depth": depth, "intensity": intensity, "model_depth": None, "imu": imu,
                                "t0": t0, "t1": t1}, stream, out)

    def set_graphs(self, enable: bool):
        """Replay each level's Gauss-Newton launches from a captured HIP graph (True) or issue them one by
        one (False); the results are the same (dslam_session_set_graphs)."""
        _check(lib().dslam_session_set_graphs(self.handle, 1 if enable else 0), "dslam_session_set_graphs")
        self._graphs = bool(enable)

    @property
    def graphs(self) -> bool:
        """Whether the session replays captured graphs (the library's default until set_graphs)."""
        return getattr(self, "_graphs", SESSION_GRAPHS_DEFAULT)

    def track_frame_input(self, frame: dict, stream=None, out=None):
        """Enqueue one tracking step (dslam_track_frame): frame = dict(depth, intensity, model_depth,
        model_intensity, T_WM, imu, t0, t1) as for Batch.track; model_depth None tracks against the
        session's MODEL pyramid, otherwise both pyramids are built in the launch that initialises the
        frame."""
        fi, keep = frame_input(frame, (self.cam.width, self.cam.height))
        _check(lib().dslam_track_frame(self.handle, C.byref(fi), C.byref(out) if out is not None else None,
                                       _stream_ptr(stream)), "dslam_track_frame")
        self._keep_input = keep

    def track_frame_sync(self, frame: dict, stream=None) -> dict:
        """dslam_track_frame_sync: enqueue the frame, wait for it and return its result."""
        fi, keep = frame_input(frame, (self.cam.width, self.cam.height))
        r = _abi.TrackResult()
        _check(lib().dslam_track_frame_sync(self.handle, C.byref(fi), C.byref(r), _stream_ptr(stream)),
               "dslam_track_frame_sync")
        return result_dict(r)

    def checkpoint(self) -> bytes:
        """dslam_session_checkpoint: the session's opaque, versioned state blob."""
        n = C.c_uint64()
        _check(lib().dslam_session_checkpoint(self.handle, None, 0, C.byref(n)), "dslam_session_checkpoint")
        buf = C.create_string_buffer(n.value)
        _check(lib().dslam_session_checkpoint(self.handle, buf, n.value, C.byref(n)), "dslam_session_checkpoint")
        return buf.raw[:n.value]

    def restore(self, blob: bytes):
        """dslam_session_restore from a checkpoint blob."""
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(lib().dslam_session_restore(self.handle, buf, len(blob)), "dslam_session_restore")

    def result(self) -> dict:
        r = _abi.TrackResult()
        _check(lib().dslam_session_result(self.handle, C.byref(r)), "dslam_session_result")
        return result_dict(r)

    def linearize(self, level, Ra, ta, Rb, tb, x0, x1, mask=None, stream=None) -> dict:
        f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32).ravel())  # noqa: E731
        arrs = [f(Ra), f(ta), f(Rb), f(tb)]
        ptrs = [a.ctypes.data_as(C.POINTER(C.c_float)) for a in arrs]
        out = _abi.LinearSystem()
        a, b = state_struct(x0), state_struct(x1)
        mptr = C.c_void_p(mask.data_ptr()) if mask is not None else None
        _check(lib().dslam_linearize(self.handle, int(level), *ptrs, C.byref(a), C.byref(b), mptr, C.byref(out),
                                     _stream_ptr(stream)), "dslam_linearize")
        return {"H_icp": np.array(out.H_icp[:]).reshape(12, 12), "b_icp": np.array(out.b_icp[:]),
                "cost_icp": out.cost_icp, "n_icp": out.n_icp, "H_rgb": np.array(out.H_rgb[:]).reshape(12, 12),
                "b_rgb": np.array(out.b_rgb[:]), "cost_rgb": out.cost_rgb, "n_rgb": out.n_rgb,
                "raw": np.array(out.raw[:])}

    def profile_residual(self, level, reps, stream=None):
        _check(lib().dslam_profile_residual(self.handle, int(level), int(reps), _stream_ptr(stream)),
               "dslam_profile_residual")

    def copy_pyramid(self, which, level, channel) -> np.ndarray:
        W, H = self.cam.width >> level, self.cam.height >> level
        out = np.empty((H, W), dtype=np.float32)
        _check(lib().dslam_copy_pyramid(self.handle, int(which), int(level), int(channel),
                                        out.ctypes.data_as(C.POINTER(C.c_float))), "dslam_copy_pyramid")
        return out

    def get_state(self):
        x = _abi.FrameState()
        q = np.zeros(4)
        p = _abi.Prior()
        fi = C.c_int32()
        _check(lib().dslam_session_get_state(self.handle, C.byref(x), q.ctypes.data_as(C.POINTER(C.c_double)),
                                             C.byref(p), C.byref(fi)), "dslam_session_get_state")
        return state_dict(x), q, prior_dict(p), fi.value

    def set_state(self, x0, q_IW, prior, frame_index=0):
        xs = state_struct(x0)
        q, qp = _dptr(q_IW)
        ps = prior_struct(prior) if prior is not None else None
        _check(lib().dslam_session_set_state(self.handle, C.byref(xs), qp, C.byref(ps) if ps is not None else None,
                                             int(frame_index)), "dslam_session_set_state")


def frame_input(f: dict, size=None):
    """FrameInput for dict(depth, intensity, model_depth, model_intensity, T_WM, imu, t0, t1) (device images
    as check_images takes them, of the session's camera size (width, height) when given); returns (struct,
    keep-alive) -- the IMU array must outlive the struct's use."""
    d, im, md = f["depth"], f["intensity"], f.get("model_depth")
    check_images(d, im, size, "frame")
    fi = _abi.FrameInput()
    fi.depth, fi.intensity, fi.pitch = d.data_ptr(), im.data_ptr(), int(d.shape[1])
    if md is not None:  # else: track against the session's MODEL pyramid
        mi = f["model_intensity"]
        check_images(md, mi, size, "model view")
        fi.model_depth, fi.model_intensity, fi.model_pitch = md.data_ptr(), mi.data_ptr(), int(md.shape[1])
        fi.T_WM[:] = [float(v) for v in np.asarray(f["T_WM"], dtype=np.float64).ravel()]
    arr = None
    if f.get("imu") is not None:
        arr, cnt = imu_samples(f["imu"]["t"], f["imu"]["gyro"], f["imu"]["acc"])
        fi.imu, fi.n_imu = arr, cnt
    fi.t0, fi.t1 = float(f.get("t0", 0.0)), float(f.get("t1", 0.0))
    return fi, (arr, f)


MAP_FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "inten", "radius", "conf")
# the library's launch mode of a newly opened session (dslam_session_set_graphs)
SESSION_GRAPHS_DEFAULT = False


class Map:
    """Surfel map of one camera (dslam_map_*): fusion of tracked frames and model-view prediction."""

    def __init__(self, ctx: Context, cam, capacity: int, assoc_dist: float = 0.05, assoc_cos: float = 0.8,
                 render_band: float = 0.03):
        self.cam = camera(cam) if not isinstance(cam, _abi.Camera) else cam
        prm = _abi.MapParams(int(capacity), float(assoc_dist), float(assoc_cos), float(render_band))
        h = C.c_void_p()
        _check(lib().dslam_map_create(ctx.handle, C.byref(self.cam), C.byref(prm), C.byref(h)), "dslam_map_create")
        self.handle = h
        self.capacity = int(capacity)

    def close(self):
        if self.handle:
            _check(lib().dslam_map_destroy(self.handle), "dslam_map_destroy")
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        _check(lib().dslam_map_reset(self.handle, _stream_ptr(stream)), "dslam_map_reset")

    def fuse(self, session: "Session", T_WC, stream=None):
        T, Tp = _dptr(np.asarray(T_WC).ravel())
        _check(lib().dslam_map_fuse(self.handle, session.handle, Tp, _stream_ptr(stream)), "dslam_map_fuse")

    def predict(self, session: "Session", T_WM, stream=None):
        T, Tp = _dptr(np.asarray(T_WM).ravel())
        _check(lib().dslam_map_predict(self.handle, session.handle, Tp, _stream_ptr(stream)), "dslam_map_predict")

    def render(self, T_WM, depth, intensity, stream=None):
        check_images(depth, intensity, (self.cam.width, self.cam.height), "render target")
        T, Tp = _dptr(np.asarray(T_WM).ravel())
        _check(lib().dslam_map_render(self.handle, Tp, C.c_void_p(depth.data_ptr()), C.c_void_p(intensity.data_ptr()),
                                      _stream_ptr(stream)), "dslam_map_render")

    def deform(self, nodes, params, stream=None):
        """Apply a solved deformation graph (nodes N x 3, params N x 12) to every surfel."""
        nd, ndp = _dptr(np.asarray(nodes, dtype=np.float64).ravel())
        pr, prp = _dptr(np.asarray(params, dtype=np.float64).ravel())
        _check(lib().dslam_map_deform(self.handle, int(len(nd) // 3), ndp, prp, _stream_ptr(stream)),
               "dslam_map_deform")

    def count(self):
        n, d = C.c_int32(), C.c_int32()
        _check(lib().dslam_map_count(self.handle, C.byref(n), C.byref(d)), "dslam_map_count")
        return int(n.value), int(d.value)

    def arrays(self) -> dict:
        n, _ = self.count()
        out = {}
        for k, name in enumerate(MAP_FIELDS):
            a = np.empty(n, dtype=np.float32)
            _check(lib().dslam_map_copy(self.handle, k, a.ctypes.data_as(C.POINTER(C.c_float)), n), "dslam_map_copy")
            out[name] = a
        return out


class Deform:
    """Deformation-graph solver with the gravity term (dslam_deform_*)."""

    def __init__(self, ctx: Context, max_nodes: int, max_points: int):
        h = C.c_void_p()
        _check(lib().dslam_deform_create(ctx.handle, int(max_nodes), int(max_points), C.byref(h)),
               "dslam_deform_create")
        self.handle = h

    def close(self):
        if self.handle:
            _check(lib().dslam_deform_destroy(self.handle), "dslam_deform_destroy")
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def solve(self, nodes, con=(), pin=(), rel=(), g_W=(0.0, 0.0, -9.81), global_=False, iters=5, stream=None):
        """Node parameters (N x 12: A row-major, t) after `iters` Gauss-Newton steps, and the cost before
        each step.  con / rel: (source, destination) pairs; pin: points."""
        keep = []

        def arr(a, width):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, width))
            keep.append(a)
            return len(a), (a.ctypes.data_as(C.POINTER(C.c_double)) if len(a) else None)

        pr = _abi.DeformProblem()
        pr.n_nodes, pr.nodes = arr(nodes, 3)
        pr.n_con, pr.con = arr([np.r_[s, d] for s, d in con] if len(con) else np.zeros((0, 6)), 6)
        pr.n_pin, pr.pin = arr(pin if len(pin) else np.zeros((0, 3)), 3)
        pr.n_rel, pr.rel = arr([np.r_[s, d] for s, d in rel] if len(rel) else np.zeros((0, 6)), 6)
        pr.global_ = 1 if global_ else 0
        pr.g_W[:] = [float(v) for v in g_W]
        x = np.zeros(12 * pr.n_nodes)
        cost = np.zeros(iters)
        _check(lib().dslam_deform_solve(self.handle, C.byref(pr), int(iters), x.ctypes.data_as(C.POINTER(C.c_double)),
                                        cost.ctypes.data_as(C.POINTER(C.c_double)), _stream_ptr(stream)),
               "dslam_deform_solve")
        return x.reshape(-1, 12), cost


class Batch:
    """Staging for batched tracking steps over many sessions (dslam_batch_*)."""

    def __init__(self, ctx: Context, max_sessions: int):
        h = C.c_void_p()
        _check(lib().dslam_batch_create(ctx.handle, int(max_sessions), C.byref(h)), "dslam_batch_create")
        self.handle = h
        self.max_sessions = int(max_sessions)
        self._keep = None
        self._n = 0

    def close(self):
        if self.handle:
            _check(lib().dslam_batch_destroy(self.handle), "dslam_batch_destroy")
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def track(self, sessions, frames, stream=None):
        """Enqueue one step.  frames[i] = dict(depth, intensity, model_depth, model_intensity, T_WM,
        imu (dict t/gyro/acc or None), t0, t1) for sessions[i]; device images contiguous."""
        n = len(sessions)
        handles = (C.c_void_p * n)(*[s.handle for s in sessions])
        inputs = (_abi.FrameInput * n)()
        keep = []
        if len(frames) != n:
            raise ValueError(f"{n} sessions but {len(frames)} frames")
        for i, f in enumerate(frames):
            inputs[i], k = frame_input(f, (sessions[i].cam.width, sessions[i].cam.height))
            keep.append(k)
        _check(lib().dslam_batch_track(self.handle, n, handles, inputs, _stream_ptr(stream)), "dslam_batch_track")
        self._keep = (keep, frames)
        self._n = n

    def set_tile_order(self, order: int):
        """dslam_batch_set_tile_order: 1 XCD-banded (default), 0 round-robin, -1 the largest sessions' tuned order."""
        _check(lib().dslam_batch_set_tile_order(self.handle, int(order)), "dslam_batch_set_tile_order")

    def set_graphs(self, enable: bool):
        """dslam_batch_set_graphs: replay each batch composition's launches from a captured HIP graph."""
        _check(lib().dslam_batch_set_graphs(self.handle, int(bool(enable))), "dslam_batch_set_graphs")

    def profile_residual(self, level, reps, stream=None) -> int:
        """Relaunch the last step's batched residual pass; returns the pixels per launch."""
        px = C.c_uint64()
        _check(lib().dslam_batch_profile_residual(self.handle, int(level), int(reps), _stream_ptr(stream),
                                                  C.byref(px)), "dslam_batch_profile_residual")
        return px.value

    def results(self) -> list:
        out = (_abi.TrackResult * self._n)()
        _check(lib().dslam_batch_results(self.handle, out), "dslam_batch_results")
        return [result_dict(out[i]) for i in range(self._n)]


def batch_track_noalloc(sessions, frames, stream=None) -> list:
    """dslam_batch_track_noalloc: one batched step with the library's static scratch (no allocation); waits
    and returns the results in call order."""
    n = len(sessions)
    hs = (C.c_void_p * n)(*[s.handle for s in sessions])
    fis, keep = [], []
    if len(frames) != n:
        raise ValueError(f"{n} sessions but {len(frames)} frames")
    for s, f in zip(sessions, frames):
        fi, k = frame_input(f, (s.cam.width, s.cam.height))
        fis.append(fi)
        keep.append(k)
    arr = (_abi.FrameInput * n)(*fis)
    out = (_abi.TrackResult * n)()
    _check(lib().dslam_batch_track_noalloc(n, hs, arr, out, _stream_ptr(stream)), "dslam_batch_track_noalloc")
    return [result_dict(out[i]) for i in range(n)]


class Server:
    """Serving loop with continuous batching (dslam_server_*).  One thread drives it."""

    def __init__(self, ctx: Context, max_batch: int, pipeline_depth: int = 2, graphs: bool = False):
        p = _abi.ServerParams(int(max_batch), int(pipeline_depth), int(bool(graphs)))
        h = C.c_void_p()
        _check(lib().dslam_server_create(ctx.handle, C.byref(p), C.byref(h)), "dslam_server_create")
        self.handle = h
        self._buf = (_abi.RequestDone * 256)()

    def close(self):
        if self.handle:
            _check(lib().dslam_server_destroy(self.handle), "dslam_server_destroy")
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def clock() -> float:
        return float(lib().dslam_server_clock())

    def submit(self, session: Session, fi: _abi.FrameInput) -> int:
        rid = C.c_uint64()
        _check(lib().dslam_server_submit(self.handle, session.handle, C.byref(fi), C.byref(rid)),
               "dslam_server_submit")
        return rid.value

    def poll(self, wait: bool = False) -> list:
        """Finished requests as (request_id, session handle value, submit_s, launch_s, done_s, device_ms,
        batch_size, result struct copy)."""
        n = C.c_int32()
        code = lib().dslam_server_poll(self.handle, int(bool(wait)), self._buf, len(self._buf), C.byref(n))
        out = []
        for i in range(n.value):
            r = self._buf[i]
            res = _abi.TrackResult()
            C.pointer(res)[0] = r.result
            out.append((r.request_id, r.session, r.submit_s, r.launch_s, r.done_s, r.device_ms, r.batch_size, res))
        _check(code, "dslam_server_poll")
        return out

    def counts(self):
        p, f = C.c_int32(), C.c_int32()
        _check(lib().dslam_server_counts(self.handle, C.byref(p), C.byref(f)), "dslam_server_counts")
        return p.value, f.value
