"""Benchmark: dense RGB-D-inertial tracking of a 640x480 sequence on one MI355X.

One step = one tracked frame through the whole hot path: the model-view and
current-frame pyramids, IMU preintegration and prediction, 3 pyramid levels
of Gauss-Newton (10/5/4 iterations of the residual pass + float64 solve) and
the marginalisation.  Inputs (300 synthetic frames rendered from the
procedural scene along a seeded spline trajectory, IMU at 200 Hz) are
resident in HBM before timing starts.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects for the
dominant kernel's achieved bandwidth and the CPU oracle's rate).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tracked frames/s + residual-pass GB/s at 640x480; p50/p99 track latency"
HBM_PEAK_GBS = 8000.0
# vector-ALU issue peak without packed FP32 (the library is built with it off): 256 CUs x 4 SIMDs x 2.4 GHz,
# one wave64 instruction per SIMD every 4 cycles
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4
COPY_BYTES = 256 << 20  # calibration copy for the HBM byte counters
# bytes per pixel-iteration of the residual pass under three accountings: the algorithmic floor (depth 4 +
# intensity 1 of the current frame and of the model view; everything else can be recomputed), the reference
# layout (all-float32 maps: V1 12 + N1 12 + I1 4 + V0 12 + N0 12 + I0 4 + G0 8) and this library's layout
# (current vertex 12 + intensity 2, model vertex 12 + normal 12 + intensity 2 + gradient 4, 16-bit
# fixed-point intensity and gradient; the current normal is unread without the normal gate)
FLOOR_BYTES_PER_PIXEL = 10
REF_LAYOUT_BYTES_PER_PIXEL = 64
LAYOUT_BYTES_PER_PIXEL = 44
# hardware counters of one level-0 residual launch at 640x480 (float32 rows) per launch shape ("ppt,banded")
# and of a 256 MiB calibration copy, from rocprofv3 --pmc runs of `bench.py --counters --counters-batch`
# (profiles/residual_kernel_640x480_counters.md); valid for the residual-pass sources with this hash
COUNTERS = {
    "source_sha256": "49860b2aed08462e",
    "copy_fetch_kib": 131086.7, "copy_write_kib": 262144.0,
    "shapes": {  # "ppt,banded": per-dispatch means over 50 back-to-back launches
        "1,0": {"fetch_kib": 7939.7, "write_kib": 300.0, "valu_insts": 1993316, "waves": 4800},
        "1,1": {"fetch_kib": 5151.2, "write_kib": 300.0, "valu_insts": 1993316, "waves": 4800},
        "2,0": {"fetch_kib": 7861.9, "write_kib": 150.0, "valu_insts": 1747316, "waves": 2400},
        "2,1": {"fetch_kib": 5189.7, "write_kib": 150.0, "valu_insts": 1747316, "waves": 2400},
        "4,0": {"fetch_kib": 6821.0, "write_kib": 75.0, "valu_insts": 1624316, "waves": 1200},
        "4,1": {"fetch_kib": 5252.8, "write_kib": 75.0, "valu_insts": 1624316, "waves": 1200},
    },
    # the batched level-0 pass over a 16-session mix (2 at 1280x720, 8 at 640x480, 6 at 320x240), banded tiles
    "batch_banded": {"pixels": 4761600, "fetch_kib": 96006.7, "write_kib": 2100.0, "valu_insts": 26489876},
}
RESIDUAL_SOURCES = ("kernels.hip", "residual.h", "device.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "bench_oracle.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_sequence(n_frames, W, H, device):
    import synth
    t = time.time()
    seq = synth.configs.sequence(seed=2001, n_frames=n_frames, width=W, height=H, device=device)
    log(f"[bench] generated {n_frames} frames {W}x{H} in {time.time() - t:.1f}s")
    return seq


def frame_inputs(seq, j):
    """(model depth, model intensity, T_WM, depth, intensity, imu window, t0, t1) for tracking frame j."""
    import synth
    md, mi, T = synth.configs.model_view(seq, j)
    t0, t1 = seq["times"][j - 1], seq["times"][j]
    a, b = synth.configs.imu_window(seq["imu"]["t"], t0, t1)
    imu = {k: v[a:b] for k, v in seq["imu"].items()}
    return md, mi, T, seq["depth"][j], seq["intensity"][j], imu, t0, t1


def residual_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in RESIDUAL_SOURCES:
        with open(os.path.join(ROOT, "paper_2207_10940_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_figures(ppt, banded):
    """HBM bytes (FETCH_SIZE and WRITE_SIZE, each scaled by its reading for a copy of known size) and VALU
    wave-instructions of one level-0 residual launch of the given shape, or None when the kernel sources
    changed since the counters were taken."""
    c = COUNTERS
    f = c["shapes"].get(f"{ppt},{banded}")
    if c["source_sha256"] is None or f is None or not residual_source_hash().startswith(c["source_sha256"]):
        return None
    fetch = f["fetch_kib"] * (COPY_BYTES / 1024) / c["copy_fetch_kib"] * 1024
    write = f["write_kib"] * (COPY_BYTES / 1024) / c["copy_write_kib"] * 1024
    return {"traffic_bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
            "valu_insts": f["valu_insts"], "waves": f["waves"]}


def batch_counter_figures():
    """HBM bytes and VALU wave-instructions per pixel of the banded batched level-0 pass (16-session mix
    counters, scaled like counter_figures), or None when the kernel sources changed since."""
    c = COUNTERS
    if c["source_sha256"] is None or not residual_source_hash().startswith(c["source_sha256"]):
        return None
    b = c["batch_banded"]
    fetch = b["fetch_kib"] * (COPY_BYTES / 1024) / c["copy_fetch_kib"] * 1024
    write = b["write_kib"] * (COPY_BYTES / 1024) / c["copy_write_kib"] * 1024
    return {"bytes_per_pixel": (fetch + write) / b["pixels"], "valu_insts_per_pixel": b["valu_insts"] / b["pixels"]}


def measure_copy_gbs(nbytes, reps):
    """Read + write bandwidth of a plain device copy of nbytes (HIP events around reps back-to-back copies)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2 * nbytes / t / 1e9


def roofline(k_ms, px, kernel, launch):
    """Roofline object of the level-0 residual pass: `achieved` counts the algorithmic floor bytes; the
    reference-layout, own-layout and counter accountings, the measured copy bandwidths and the vector-ALU
    issue roof sit beside it, and `binding` names the roof the kernel is closest to."""
    t = k_ms * 1e-3
    floor_b = FLOOR_BYTES_PER_PIXEL * px
    hbm_copy = measure_copy_gbs(1 << 30, 20)
    mall_copy = measure_copy_gbs(16 << 20, 200)
    acc = {}
    for name, bpp in (("floor_10B", FLOOR_BYTES_PER_PIXEL), ("ref_layout_64B", REF_LAYOUT_BYTES_PER_PIXEL),
                      ("own_layout_44B", LAYOUT_BYTES_PER_PIXEL)):
        gbs = bpp * px / t / 1e9
        acc[name] = {"bytes_per_launch": bpp * px, "GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}
    cf = counter_figures(launch["pixels_per_thread"], launch["xcd_banded"])
    valu = None
    if cf is not None:
        gbs = cf["traffic_bytes"] / t / 1e9
        acc["counter_traffic"] = {"bytes_per_launch": cf["traffic_bytes"], "GBs": gbs,
                                  "frac_of_peak": gbs / HBM_PEAK_GBS, "frac_of_measured_copy": gbs / hbm_copy}
        rate = cf["valu_insts"] / t / 1e9
        valu = {"insts_per_launch": cf["valu_insts"], "wave_insts_per_pixel": cf["valu_insts"] / px,
                "lane_insts_per_pixel": 64.0 * cf["valu_insts"] / px,
                "achieved_ginst_s": rate, "peak_ginst_s": VALU_PEAK_GINST, "frac": rate / VALU_PEAK_GINST,
                "waves": cf["waves"]}
    binding = None
    if valu is not None:
        fr = {"valu": valu["frac"], "hbm": acc["counter_traffic"]["frac_of_measured_copy"]}
        name = max(fr, key=fr.get)
        # a roof binds when the launch reaches 0.6 of it; below that on both, latency does
        binding = name if fr[name] >= 0.6 else f"latency ({name} closest, at {fr[name]:.2f} of its roof)"
    achieved = floor_b / t / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": cf["traffic_bytes"] if cf else None,
            "kernel": kernel, "kernel_us": k_ms * 1e3, "launch": launch, "pixels": px,
            "bytes_per_launch": floor_b, "bytes_per_pixel": FLOOR_BYTES_PER_PIXEL,
            "accountings": acc, "measured_copy_GBs": {"hbm_1GiB": hbm_copy, "mall_16MiB": mall_copy},
            "frac_of_measured_hbm": achieved / hbm_copy, "valu": valu, "binding": binding}


def run_gpu(args):
    import torch

    import paper_2207_10940_amd as P
    W, H = 640, 480
    n_frames = args.warmup + args.steps + 1
    seq = make_sequence(n_frames, W, H, "cuda")
    frames = [frame_inputs(seq, j) for j in range(1, n_frames)]
    frames = [(md.contiguous(), mi.contiguous(), T, d.contiguous(), i.contiguous(), imu, t0, t1)
              for (md, mi, T, d, i, imu, t0, t1) in frames]
    torch.cuda.synchronize()
    ctx = P.Context(0)
    # the residual pass's launch shape per level from the autotuner (kept by the context for its sessions), or
    # pinned from a file (profiler runs, whose timing the tuner must not see)
    if args.shapes:
        with open(args.shapes) as f:
            tuned = [e for e in json.load(f) if e["width"] == W and e["height"] == H]
        ctx.set_tune(tuned)
    else:
        tuned = ctx.autotune([seq["camera"]], levels=3, jac="fp32")
    log("[bench] autotuned: " + ", ".join(f"L{e['level']} ppt {e['ppt']} {'banded' if e['xcd_banded'] else 'round-robin'} "
                                          f"({e['us']:.1f} us)" for e in tuned))
    tp = P.track_params(levels=3, iters=(10, 5, 4), mode="rgbdi", jac="fp32")
    sess = P.Session(ctx, seq["camera"], tp, P.imu_params(), seq["x0"], seq["q_IW"], seq["prior"])
    x_init = sess.get_state()
    stream = torch.cuda.current_stream()

    def track(k):  # both pyramids, preintegration and prediction share the frame's first launch
        md, mi, T, d, i, imu, t0, t1 = frames[k]
        sess.track_frame_input({"depth": d, "intensity": i, "model_depth": md, "model_intensity": mi, "T_WM": T,
                                "imu": imu, "t0": t0, "t1": t1}, stream)

    for k in range(args.warmup):
        track(k)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} frames done")
    t_start = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        track(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    res = sess.result()
    log(f"[bench] timed {args.steps} frames in {elapsed * 1e3:.1f} ms; last status {res['status']}")
    gt = seq["gt"][args.warmup + args.steps]
    pos_err = float(np.linalg.norm(res["x1"]["r"] - gt["r"]))

    # latency: each frame submitted and waited for on its own
    sess.set_state(*x_init)
    lat = []
    n_lat = min(args.latency_frames, n_frames - 1)
    for k in range(n_lat):
        md, mi, T, d, i, imu, t0, t1 = frames[k]
        t = time.perf_counter()
        sess.track_frame_sync({"depth": d, "intensity": i, "model_depth": md, "model_intensity": mi, "T_WM": T,
                               "imu": imu, "t0": t0, "t1": t1}, stream)
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat[5:] if len(lat) > 10 else lat)
    log(f"[bench] latency over {len(lat)} frames: p50 {np.percentile(lat, 50):.3f} ms p99 {np.percentile(lat, 99):.3f} ms")

    # accuracy over the whole sequence, frame by frame from the initial state (outside the timed region):
    # the analogue of the paper's velocity / bias convergence plots and its ATE RMSE.  Closed loop: each
    # frame's model view is rendered (noise-free) at the previous frame's estimate, so the tracker never sees
    # the ground truth.  The open-loop figure (model views at the previous ground-truth pose, as timed above)
    # is reported beside it.
    import synth
    accuracy = {}
    for loop in ("closed", "open"):
        sess.set_state(*x_init)
        est = []
        prev = seq["x0"]
        for k in range(n_frames - 1):
            if loop == "closed":
                md, mi, T = synth.configs.model_view_at(seq, prev)
                f = frames[k]
                sess.track_frame_input({"depth": f[3], "intensity": f[4], "model_depth": md.contiguous(),
                                        "model_intensity": mi.contiguous(), "T_WM": T, "imu": f[5], "t0": f[6],
                                        "t1": f[7]}, stream)
            else:
                track(k)
            prev = sess.result()["x1"]
            est.append(prev)
        accuracy[loop] = sequence_accuracy(est, seq["gt"][1:n_frames])
        a = accuracy[loop]
        log(f"[bench] {loop}-loop accuracy over {len(est)} frames: ATE {a['ate_rmse_m'] * 100:.3f} cm, velocity "
            f"error {a['windows'][-1]['vel_err_mps']:.2e} m/s, gyro bias {a['windows'][-1]['bg_err_radps']:.2e} "
            f"rad/s, accel bias {a['windows'][-1]['ba_err_mps2']:.2e} m/s^2 (last window)")
    accuracy = dict(accuracy["closed"], model_view="rendered at the previous frame's estimate (closed loop)",
                    open_loop=dict(accuracy["open"], model_view="rendered at the previous ground-truth pose"))

    # launch modes (outside the timed region): the frame's Gauss-Newton launches replayed from per-level HIP
    # graphs, or issued one by one; the same frames, throughput and latency as above
    launch_modes = {}
    default_graphs = sess.graphs
    for name, on in (("graphs", True), ("eager", False)):
        sess.set_graphs(on)
        sess.set_state(*x_init)
        for k in range(args.warmup):
            track(k)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            track(k)
        torch.cuda.synchronize()
        fps = args.steps / (time.perf_counter() - t)
        sess.set_state(*x_init)
        ml = []
        for k in range(n_lat):
            t = time.perf_counter()
            track(k)
            sess.result()
            ml.append((time.perf_counter() - t) * 1e3)
        ml = np.array(ml[5:] if len(ml) > 10 else ml)
        launch_modes[name] = {"frames_per_s": fps, "latency_p50_ms": float(np.percentile(ml, 50)),
                              "latency_p99_ms": float(np.percentile(ml, 99))}
        log(f"[bench] {name}: {fps:.0f} frames/s, latency p50 {launch_modes[name]['latency_p50_ms']:.3f} ms "
            f"p99 {launch_modes[name]['latency_p99_ms']:.3f} ms")
    sess.set_graphs(default_graphs)
    launch_modes["default"] = "graphs" if default_graphs else "eager"

    # dominant kernel: the level-0 residual pass, timed back to back with events on the same stream
    reps = args.kernel_reps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sess.profile_residual(0, 20, stream)
    e0.record(stream)
    sess.profile_residual(0, reps, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / reps
    px = W * H
    ppt0 = next((e["ppt"] for e in tuned if e["level"] == 0), None)
    band0 = next((e["xcd_banded"] for e in tuned if e["level"] == 0), None)
    roof = roofline(k_ms, px, f"residual_kernel<{ppt0}> (level 0, 640x480, float32 rows)",
                    {"pixels_per_thread": ppt0, "xcd_banded": band0, "block": 256})
    log(f"[bench] level-0 residual pass: {k_ms * 1e3:.2f} us/launch, {roof['achieved']:.1f} GB/s at the "
        f"{FLOOR_BYTES_PER_PIXEL} B/px floor; measured copy {roof['measured_copy_GBs']['hbm_1GiB']:.0f} GB/s; "
        f"binding: {roof['binding']}")
    sess.close()
    ctx.close()
    return {
        "value": args.steps / elapsed, "ms_per_step": elapsed * 1e3 / args.steps,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "frames": int(len(lat)), "kind": "host submit to result, one frame at a time (dslam_track_frame_sync)"},
        "pose_err_final_m": pos_err,
        "accuracy": accuracy,
        "launch_modes": launch_modes,
        "autotune": tuned,
        "roofline": roof,
        "seq": seq,
    }


def run_counters(args):
    """Hardware-counter run: the level-0 residual pass on a tracked sequence frame, then a plain
    device copy of known size whose FETCH_SIZE / WRITE_SIZE readings scale the counters to bytes.
    Meant to be run under rocprofv3 --pmc.  The inputs are generated on the host and copied over, so the
    only kernels are the library's and the calibration copy; prints one JSON line describing what ran."""
    import torch

    import paper_2207_10940_amd as P
    W, H = 640, 480
    seq = make_sequence(4, W, H, "cpu")
    ctx = P.Context(0)
    tp = P.track_params(levels=3, iters=(10, 5, 4), mode="rgbdi", jac=args.counters_jac)
    stream = torch.cuda.current_stream()
    frames = []
    for j in range(1, 4):
        md, mi, T, d, i, imu, t0, t1 = frame_inputs(seq, j)
        frames.append({"depth": d.to("cuda"), "intensity": i.to("cuda"), "model_depth": md.to("cuda"),
                       "model_intensity": mi.to("cuda"), "T_WM": T, "imu": imu, "t0": t0, "t1": t1})
    # every level-0 launch shape the autotuner can pick, pinned in turn (levels 1-2 keep the library's
    # defaults): three tracked frames (30 level-0 passes), then kernel_reps passes back to back
    shapes = [(ppt, banded) for ppt in (1, 2, 4) for banded in (0, 1)]
    for ppt, banded in shapes:
        ctx.set_tune([{"width": W, "height": H, "level": 0, "jac_format": args.counters_jac, "ppt": ppt,
                       "xcd_banded": banded}])
        sess = P.Session(ctx, seq["camera"], tp, P.imu_params(), seq["x0"], seq["q_IW"], seq["prior"])
        for f in frames:
            sess.track_frame_input(f, stream)
        torch.cuda.synchronize()
        sess.profile_residual(0, args.kernel_reps, stream)
        torch.cuda.synchronize()
        sess.close()
    batch_px = None
    if args.counters_batch:
        # the batched pass over a 16-session mix (2 at 1280x720, 8 at 640x480, 6 at 320x240; inputs made on the
        # host), with level 0 pinned to 4 / 2 / 1 pixels per thread, the batch's round-robin then XCD-banded
        # tile order:
        # one tracked step (10 level-0 passes), then kernel_reps passes back to back, for each order
        import synth
        mix = ((1280, 720, 2, 4), (640, 480, 8, 2), (320, 240, 6, 1))
        seqs = [synth.configs.session_sequence(4000 + 1000 * ci + k, 2, w, h)
                for ci, (w, h, count, _) in enumerate(mix) for k in range(count)]
        bf = []
        for sq in seqs:
            f = serving_frame(sq, 1)
            for key in ("depth", "intensity", "model_depth", "model_intensity"):
                f[key] = f[key].to("cuda")
            bf.append(f)
        for banded in (0, 1):
            ctx.set_tune([{"width": w, "height": h, "level": 0, "jac_format": args.counters_jac, "ppt": ppt,
                           "xcd_banded": banded} for w, h, _, ppt in mix])
            bs = [P.Session(ctx, sq["camera"], tp, P.imu_params(), sq["x0"], sq["q_IW"], sq["prior"]) for sq in seqs]
            batch = P.Batch(ctx, len(bs))
            batch.set_tile_order(banded)
            batch.track(bs, bf, stream)
            batch.results()
            batch_px = batch.profile_residual(0, args.kernel_reps, stream)
            torch.cuda.synchronize()
            batch.close()
            for s in bs:
                s.close()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32).to("cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"counters_run": True, "jac": args.counters_jac, "residual_reps": args.kernel_reps,
                      "residual_pixels": W * H, "level0_shapes_in_order": shapes,
                      "level0_dispatches_per_shape": 30 + args.kernel_reps,
                      "batch_pixels": batch_px, "copy_bytes_each_way": COPY_BYTES, "copy_reps": 3}), flush=True)


SERVING_MIX = ((1280, 720, 8), (640, 480, 32), (320, 240, 24))  # (width, height, sessions)


def serving_frame(seq, j):
    md, mi, T = synth_mod().configs.model_view(seq, j)
    t0, t1 = seq["times"][j - 1], seq["times"][j]
    a, b = synth_mod().configs.imu_window(seq["imu"]["t"], t0, t1)
    return {"depth": seq["depth"][j].contiguous(), "intensity": seq["intensity"][j].contiguous(),
            "model_depth": md.contiguous(), "model_intensity": mi.contiguous(), "T_WM": T,
            "imu": {k: v[a:b] for k, v in seq["imu"].items()}, "t0": t0, "t1": t1}


def synth_mod():
    import synth
    return synth


def run_serving(args):
    """Serving form: 64 concurrent sessions (8 at 1280x720, 32 at 640x480, 24 at 320x240) through the
    continuous-batching server.  Saturation throughput (every frame queued at once), latency under Poisson
    arrivals at 30 Hz per session, the plain path (one session, one frame at a time, synchronous) on the
    same mix, and the batched level-0 residual pass against the HBM roofline."""
    import torch

    import paper_2207_10940_amd as P
    synth = synth_mod()
    nf = args.serving_frames
    t = time.time()
    seqs, specs = {}, []
    for ci, (w, h, count) in enumerate(SERVING_MIX):  # every session its own scene, trajectory and IMU stream
        seqs[(w, h)] = [synth.configs.session_sequence(4000 + 1000 * ci + k, nf + 1, w, h, device="cuda")
                        for k in range(count)]
        specs += [(w, h, k) for k in range(count)]
    frames = {key: [[serving_frame(sq, j) for j in range(1, nf + 1)] for sq in lst] for key, lst in seqs.items()}
    fins = {key: [[P.frame_input(f)[0] for f in fl] for fl in lst] for key, lst in frames.items()}
    torch.cuda.synchronize()
    log(f"[serving] generated {sum(len(v) for v in seqs.values())} sequences x {nf} frames in {time.time() - t:.1f}s")
    ctx = P.Context(0)
    tp = P.track_params(levels=3, iters=(10, 5, 4), mode="rgbdi", jac="fp32")
    sess = []
    for w, h, k in specs:
        sq = seqs[(w, h)][k]
        sess.append(P.Session(ctx, sq["camera"], tp, P.imu_params(), sq["x0"], sq["q_IW"], sq["prior"]))

    def reset():
        for (w, h, k), s in zip(specs, sess):
            sq = seqs[(w, h)][k]
            s.set_state(sq["x0"], sq["q_IW"], sq["prior"])

    total = len(sess) * nf

    def serve(graphs):
        """Saturation and nominal-load runs of the server, its steps' launches issued one by one or
        replayed from graphs."""
        server = P.Server(ctx, max_batch=min(args.serving_batch, len(sess)), pipeline_depth=args.serving_depth,
                          graphs=graphs)
        tag = "graphs" if graphs else "eager"
        # ---- saturation: every frame queued at once (each session's frames in order)
        reset()
        torch.cuda.synchronize()
        t0 = P.Server.clock()
        for j in range(nf):
            for (w, h, k), s in zip(specs, sess):
                server.submit(s, fins[(w, h)][k][j])
        done, bad, dev_ms, sizes = 0, 0, [], []
        while done < total:
            for rec in server.poll(wait=True):
                done += 1
                bad += rec[7].status != 0
                dev_ms.append(rec[5])
                sizes.append(rec[6])
        t_sat = P.Server.clock() - t0
        sat_fps = total / t_sat
        log(f"[serving] {tag} saturation: {total} frames in {t_sat * 1e3:.1f} ms = {sat_fps:.0f} frames/s, "
            f"mean batch {np.mean(sizes):.1f}, failed {bad}")
        # ---- nominal load: Poisson arrivals at 30 Hz per session
        reset()
        torch.cuda.synchronize()
        rng = np.random.default_rng(7)
        arrivals = []
        for i in range(len(sess)):
            ts = np.cumsum(rng.exponential(1.0 / 30.0, size=nf))
            arrivals += [(float(ta), i, j) for j, ta in enumerate(ts)]
        arrivals.sort()
        start = P.Server.clock() + 0.01
        owner, lat, dev_nom, sizes_nom = {}, [], [], []
        nxt, done = 0, 0
        while done < total:
            now = P.Server.clock() - start
            while nxt < total and arrivals[nxt][0] <= now:
                ta, i, j = arrivals[nxt]
                w, h, k = specs[i]
                owner[server.submit(sess[i], fins[(w, h)][k][j])] = ta
                nxt += 1
            for rec in server.poll(wait=False):
                done += 1
                ta = owner[rec[0]]
                if ta >= args.serving_warmup:
                    lat.append((rec[4] - start - ta) * 1e3)
                    dev_nom.append(rec[5])
                sizes_nom.append(rec[6])
        span = P.Server.clock() - start
        log(f"[serving] {tag} nominal 30 Hz x {len(sess)}: p50 {np.percentile(lat, 50):.2f} ms p99 "
            f"{np.percentile(lat, 99):.2f} ms over {len(lat)} frames, mean batch {np.mean(sizes_nom):.1f}")
        server.close()
        return {"saturation_fps": sat_fps, "saturation_mean_batch": float(np.mean(sizes)),
                "saturation_device_ms_per_step_p50": float(np.percentile(dev_ms, 50)), "failed": int(bad),
                "nominal": {"offered_fps": 30.0 * len(sess), "achieved_fps": total / span,
                            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                            "device_p50_ms": float(np.percentile(dev_nom, 50)), "frames": len(lat),
                            "mean_batch": float(np.mean(sizes_nom)),
                            "kind": "arrival (Poisson, 30 Hz per session) to result on the host"}}

    runs = {"eager": serve(False), "graphs": serve(True)}
    main_run = runs[args.serving_launch]
    sat_fps = main_run["saturation_fps"]
    # ---- plain path on the same mix: one session, one frame at a time, synchronous
    stream = torch.cuda.current_stream()
    per_class = {}
    for w, h, count in SERVING_MIX:
        i = next(n for n, sp in enumerate(specs) if sp[:2] == (w, h))
        sq = seqs[(w, h)][specs[i][2]]
        s = sess[i]
        s.set_state(sq["x0"], sq["q_IW"], sq["prior"])
        tl = []
        for j in range(min(nf, 12)):
            f = frames[(w, h)][specs[i][2]][j]
            ts = time.perf_counter()
            s.track_frame_input(f, stream)
            s.result()
            tl.append(time.perf_counter() - ts)
        per_class[f"{w}x{h}"] = float(np.median(tl[2:]))
    plain_s = sum(per_class[f"{w}x{h}"] * c for w, h, c in SERVING_MIX)  # one frame of every session
    plain_fps = len(sess) / plain_s
    log(f"[serving] plain path on the mix: {plain_fps:.0f} frames/s ({per_class})")
    # ---- batched level-0 residual pass over all 64 sessions
    reset()
    batch = P.Batch(ctx, len(sess))
    batch.track(sess, [frames[(w, h)][k][0] for w, h, k in specs], stream)
    batch.results()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    order_us = {}
    for name, order in (("round_robin", 0), ("xcd_banded", 1)):  # the batch default last
        batch.set_tile_order(order)
        batch.profile_residual(0, 5, stream)
        e0.record(stream)
        px = batch.profile_residual(0, reps, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        order_us[name] = e0.elapsed_time(e1) * 1e3 / reps
    k_ms = order_us["xcd_banded"] * 1e-3
    gbs = FLOOR_BYTES_PER_PIXEL * px / (k_ms * 1e-3) / 1e9
    hbm_copy = measure_copy_gbs(1 << 30, 20)
    accountings = {}
    for name, bpp in (("floor_10B", FLOOR_BYTES_PER_PIXEL), ("ref_layout_64B", REF_LAYOUT_BYTES_PER_PIXEL),
                      ("own_layout_44B", LAYOUT_BYTES_PER_PIXEL)):
        g = bpp * px / (k_ms * 1e-3) / 1e9
        accountings[name] = {"GBs": g, "frac_of_peak": g / HBM_PEAK_GBS, "frac_of_measured_copy": g / hbm_copy}
    bc = batch_counter_figures()
    if bc is not None:  # bytes and instructions per pixel from the 16-session mix's counters
        g = bc["bytes_per_pixel"] * px / (k_ms * 1e-3) / 1e9
        rate = bc["valu_insts_per_pixel"] * px / (k_ms * 1e-3) / 1e9
        accountings["counter_traffic_16_session_mix"] = {
            "bytes_per_pixel": bc["bytes_per_pixel"], "GBs": g, "frac_of_peak": g / HBM_PEAK_GBS,
            "frac_of_measured_copy": g / hbm_copy, "valu_lane_insts_per_pixel": 64.0 * bc["valu_insts_per_pixel"],
            "valu_frac": rate / VALU_PEAK_GINST}
    log(f"[serving] batched level-0 residual pass: {px} px in {k_ms * 1e3:.1f} us = {gbs:.0f} GB/s at the "
        f"{FLOOR_BYTES_PER_PIXEL} B/px floor (round-robin tile order: {order_us['round_robin']:.1f} us)")
    batch.close()
    for s in sess:
        s.close()
    ctx.close()
    return {
        "workload": "64 sessions: 8 at 1280x720, 32 at 640x480, 24 at 320x240; 3 levels 10/5/4 iterations, "
                    f"RGB-D-inertial, float32 Jacobians; continuous batching, steps of up to "
                    f"{min(args.serving_batch, len(sess))} sessions, {args.serving_depth} in flight",
        "frames": total, "sequences": "one seeded scene, trajectory and IMU stream per session",
        "saturation_fps": sat_fps, "saturation_mean_batch": main_run["saturation_mean_batch"],
        "saturation_device_ms_per_step_p50": main_run["saturation_device_ms_per_step_p50"],
        "nominal": main_run["nominal"],
        "plain_fps_same_mix": plain_fps, "plain_ms_per_frame": {k: v * 1e3 for k, v in per_class.items()},
        "speedup_vs_plain": sat_fps / plain_fps,
        "failed": runs["eager"]["failed"] + runs["graphs"]["failed"],
        "launches": f"{args.serving_launch} (the figures above); eager: steps' kernels issued one by one, "
                    "graphs: each step replayed from a graph; both runs below",
        "eager": runs["eager"], "graphs": runs["graphs"],
        "batched_residual_roofline": {
            "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "kernel_us": k_ms * 1e3, "pixels": px, "bytes_per_launch": FLOOR_BYTES_PER_PIXEL * px,
            "bytes_per_pixel": FLOOR_BYTES_PER_PIXEL, "tile_order": "xcd_banded",
            "kernel_us_by_tile_order": order_us, "measured_copy_GBs": hbm_copy, "accountings": accountings},
    }


STRESS_MIX = ((1920, 1080, 64), (1280, 720, 64), (640, 480, 64), (320, 240, 64))  # (width, height, sessions)


def mmpp_arrivals(rng, n, base=30.0, on=3.0, off=1.0 / 3.0, switch=4.0):
    """First n arrival times of a two-state Markov-modulated Poisson process: rate base*on or base*off,
    the state flipping at `switch` per second (exponential sojourns)."""
    t, state, out = 0.0, bool(rng.random() < 0.5), []
    nxt = rng.exponential(1.0 / switch)
    while len(out) < n:
        dt = rng.exponential(1.0 / (base * (on if state else off)))
        if t + dt >= nxt:
            t, state, nxt = nxt, not state, nxt + rng.exponential(1.0 / switch)
            continue
        t += dt
        out.append(t)
    return out


def run_precision():
    """Precision form on the 160x120 frame pair (2 levels): per level and term, the relative Frobenius error
    of J^T J with FP16 / BF16 rows contracted on MFMA, against the oracle's float64 normal equations (stored by
    tests/golden/make_bench_golden.py) and against the plain float32 form at the same linearisation point;
    then the pose Gauss-Newton reaches (4/4 iterations) against the oracle's and the float32 form's."""
    import torch

    import paper_2207_10940_amd as P
    import synth
    g = load_golden()["precision"]
    W, H, L = g["width"], g["height"], g["levels"]
    d = synth.configs.frame_pair(seed=g["seed"], width=W, height=H)  # generated as the stored values were
    for k in ("depth", "intensity", "model_depth", "model_intensity"):
        d[k] = d[k].to("cuda")
    lz = g["linearize"]
    st = lambda x: {k: np.array(v) for k, v in x.items()}  # noqa: E731
    x0, x1 = st(lz["x0"]), st(lz["x1"])
    T_WM = np.array(lz["T_WM"]).reshape(4, 4)
    tr = [np.array(lz[k], dtype=np.float32) for k in ("Ra", "ta", "Rb", "tb")]
    stream = torch.cuda.current_stream()
    ctx = P.Context(0)

    def open_session(jac, iters):
        tp = P.track_params(levels=L, iters=iters, mode=g["mode"], jac=jac)
        return P.Session(ctx, d["camera"], tp, P.imu_params(), d["x0"], d["q_IW"], d["prior"])

    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))  # noqa: E731
    systems = {}
    for jac in ("fp32", "fp16", "bf16"):
        s = open_session(jac, [1] * L)
        s.set_model(d["model_depth"].contiguous(), d["model_intensity"].contiguous(), T_WM, stream)
        s.build_pyramid(P.PYR_CURRENT, d["depth"].contiguous(), d["intensity"].contiguous(), stream=stream)
        systems[jac] = [s.linearize(l, *tr, x0, x1, stream=stream) for l in range(L)]
        s.close()
    poses = {}
    for jac in ("fp32", "fp16", "bf16"):
        s = open_session(jac, list(g["iters"]))
        s.track_frame_input({"depth": d["depth"].contiguous(), "intensity": d["intensity"].contiguous(),
                             "model_depth": d["model_depth"].contiguous(),
                             "model_intensity": d["model_intensity"].contiguous(), "T_WM": d["T_WM"],
                             "imu": d["imu"], "t0": d["t0"], "t1": d["t1"]}, stream)
        poses[jac] = s.result()["x1"]
        s.close()
    ctx.close()
    ox = st(g["track_x1"])
    out = {"workload": f"{W}x{H} frame pair (seed {g['seed']}), {L} levels; J^T J at a fixed linearisation point, "
                       f"then Gauss-Newton {'/'.join(map(str, g['iters']))} iterations, RGB-D-inertial",
           "oracle": "float64 values stored by tests/golden/make_bench_golden.py"}
    for jac in ("fp16", "bf16", "fp32"):
        lv = []
        for l in range(L):
            o = g["linearize"]["levels"][l]
            e = {}
            for term in ("icp", "rgb"):
                Ho = np.array(o["H_" + term]).reshape(12, 12)
                e[term] = {"jtj_vs_oracle": rel(systems[jac][l]["H_" + term], Ho),
                           "jtj_vs_fp32": rel(systems[jac][l]["H_" + term], systems["fp32"][l]["H_" + term]),
                           "n_equal_oracle": int(systems[jac][l]["n_" + term]) == o["n_" + term]}
            lv.append(e)
        p = poses[jac]
        out[jac] = {"levels": lv,
                    "pose_vs_oracle": {"m": float(np.linalg.norm(p["r"] - ox["r"])), "rad": quat_angle(p["q"], ox["q"])},
                    "pose_vs_fp32": {"m": float(np.linalg.norm(p["r"] - poses["fp32"]["r"])),
                                     "rad": quat_angle(p["q"], poses["fp32"]["q"])}}
    log("[precision] " + "; ".join(
        f"{jac}: L0 J^T J icp {out[jac]['levels'][0]['icp']['jtj_vs_oracle']:.1e} rgb "
        f"{out[jac]['levels'][0]['rgb']['jtj_vs_oracle']:.1e}, pose {out[jac]['pose_vs_oracle']['m']:.1e} m"
        for jac in ("fp16", "bf16", "fp32")))
    return out


def load_golden():
    with open(GOLDEN) as f:
        return json.load(f)


def quat_angle(qa, qb):
    """Angle of the relative rotation of two unit quaternions (w, x, y, z), from the sine and the cosine."""
    qa, qb = np.asarray(qa, dtype=np.float64), np.asarray(qb, dtype=np.float64)
    w = qa[0] * qb[0] + qa[1:] @ qb[1:]  # conj(qa) * qb
    v = qa[0] * qb[1:] - qb[0] * qa[1:] - np.cross(qa[1:], qb[1:])
    return float(2.0 * np.arctan2(np.linalg.norm(v), abs(w)))


def stored_pose_errors(specs, first, nf):
    """Pose error of the first tracked frame of session 0 per resolution against the stored oracle pose
    (None where the stored case does not match the workload's frame count)."""
    out = {}
    for g in load_golden()["stress_first_frame"]:
        key = f"{g['width']}x{g['height']}"
        i = next((n for n, sp in enumerate(specs) if sp == (g["width"], g["height"], g["session"])), None)
        if i is None or i not in first or g["n_frames"] != nf + 1:
            out[key] = None
            continue
        x = first[i]["x1"]
        out[key] = {"m": float(np.linalg.norm(x["r"] - np.array(g["x1"]["r"]))),
                    "rad": quat_angle(x["q"], g["x1"]["q"])}
    return out


def run_stress(args):
    """Serving + precision stress: 256 sessions (64 each at 1920x1080, 1280x720, 640x480, 320x240), FP16
    Jacobian rows on MFMA with float64 solves, tile shapes from the autotuner, 5% of frames with 80% zero-depth
    holes and 10% low-texture frames; saturation throughput, latency under bursty (Markov-modulated Poisson)
    arrivals, and the pose error of sampled sessions against the oracle."""
    import torch

    import paper_2207_10940_amd as P
    synth = synth_mod()
    nf = args.stress_frames
    rng = np.random.default_rng(5)  # arrival times
    t = time.time()
    seqs, specs, flags = {}, [], {"holes": 0, "low_texture": 0, "frames": 0}
    for ci, (w, h, count) in enumerate(STRESS_MIX):  # every session its own scene, trajectory and IMU stream
        lst = [synth.configs.session_sequence(5000 + 1000 * ci + k, nf + 1, w, h, device="cuda", hole_rate=0.05,
                                              low_texture_rate=0.10) for k in range(count)]
        for sq in lst:
            flags["holes"] += len(sq["hole_frames"])
            flags["low_texture"] += len(sq["low_texture_frames"])
            flags["frames"] += nf
        seqs[(w, h)] = lst
        specs += [(w, h, k) for k in range(count)]
    frames = {key: [[serving_frame(sq, j) for j in range(1, nf + 1)] for sq in lst] for key, lst in seqs.items()}
    fins = {key: [[P.frame_input(f)[0] for f in fl] for fl in lst] for key, lst in frames.items()}
    torch.cuda.synchronize()
    log(f"[stress] generated {sum(len(v) for v in seqs.values())} sequences x {nf} frames in {time.time() - t:.1f}s "
        f"({flags['holes']} hole frames, {flags['low_texture']} low-texture of {flags['frames']})")
    ctx = P.Context(0)
    tuned = ctx.autotune([seqs[(w, h)][0]["camera"] for w, h, _ in STRESS_MIX], levels=3, jac="fp16")
    log("[stress] autotuned pixels per thread / tile order: " +
        ", ".join(f"{e['width']}x{e['height']} L{e['level']}: {e['ppt']}{'b' if e['xcd_banded'] else ''} "
                  f"({e['us']:.1f} us)" for e in tuned))
    tp = P.track_params(levels=3, iters=(10, 5, 4), mode="rgbdi", jac="fp16")
    sess = []
    for w, h, k in specs:
        sq = seqs[(w, h)][k]
        sess.append(P.Session(ctx, sq["camera"], tp, P.imu_params(), sq["x0"], sq["q_IW"], sq["prior"]))
    hbm = ctx.used_bytes()

    def reset():
        for (w, h, k), s in zip(specs, sess):
            sq = seqs[(w, h)][k]
            s.set_state(sq["x0"], sq["q_IW"], sq["prior"])

    server = P.Server(ctx, max_batch=min(args.stress_batch, len(sess)), pipeline_depth=args.stress_depth,
                      graphs=args.stress_launch == "graphs")
    total = len(sess) * nf
    # ---- saturation
    reset()
    torch.cuda.synchronize()
    owner = {}
    t0 = P.Server.clock()
    for j in range(nf):
        for i, ((w, h, k), s) in enumerate(zip(specs, sess)):
            owner[server.submit(s, fins[(w, h)][k][j])] = (i, j)
    done, bad, first = 0, 0, {}
    while done < total:
        for rec in server.poll(wait=True):
            done += 1
            bad += rec[7].status != 0
            i, j = owner[rec[0]]
            if j == 0:
                first[i] = P.result_dict(rec[7])
    t_sat = P.Server.clock() - t0
    log(f"[stress] saturation: {total} frames in {t_sat * 1e3:.1f} ms = {total / t_sat:.0f} frames/s, failed {bad}")
    # ---- bursty arrivals
    reset()
    torch.cuda.synchronize()
    arr = []
    for i in range(len(sess)):
        arr += [(ta, i, j) for j, ta in enumerate(mmpp_arrivals(rng, nf))]
    arr.sort()
    start = P.Server.clock() + 0.01
    own, lat, nxt, done = {}, [], 0, 0
    while done < total:
        now = P.Server.clock() - start
        while nxt < total and arr[nxt][0] <= now:
            ta, i, j = arr[nxt]
            w, h, k = specs[i]
            own[server.submit(sess[i], fins[(w, h)][k][j])] = ta
            nxt += 1
        for rec in server.poll(wait=False):
            done += 1
            ta = own[rec[0]]
            if ta >= args.serving_warmup:
                lat.append((rec[4] - start - ta) * 1e3)
    span = P.Server.clock() - start
    log(f"[stress] bursty arrivals: p50 {np.percentile(lat, 50):.2f} ms p99 {np.percentile(lat, 99):.2f} ms "
        f"over {len(lat)} frames in {span:.2f} s")
    server.close()
    for s in sess:
        s.close()
    ctx.close()
    # ---- pose error of session 0 of every resolution (first frame, from the initial state) against the
    # oracle's values stored by tests/golden/make_bench_golden.py for the same seeded inputs
    pose = stored_pose_errors(specs, first, nf)
    log(f"[stress] pose vs oracle (fp16): {pose}")
    return {
        "workload": "256 sessions: 64 each at 1920x1080, 1280x720, 640x480, 320x240; RGB-D-inertial, 3 levels "
                    "10/5/4, FP16 Jacobian rows on MFMA, float64 solve; 5% of frames with 80% zero-depth holes, "
                    "10% low-texture; Markov-modulated Poisson arrivals (30 Hz mean, x3 / x0.33 states)",
        "frames": total, "hole_frames": flags["holes"], "low_texture_frames": flags["low_texture"],
        "sequences": "one seeded scene, trajectory and IMU stream per session", "hbm_bytes_admitted": hbm,
        "saturation_fps": total / t_sat, "failed": int(bad),
        "bursty": {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "frames": len(lat), "achieved_fps": total / span,
                   "kind": "arrival to result on the host"},
        "autotune": tuned, "pose_err_vs_oracle": pose,
    }


def ate_rmse(est, gt, align=True):
    """Absolute trajectory error (RMSE of the position differences, the metric of the paper's evaluation
    after Sturm et al.): est and gt are N x 3 positions; with align, est is first moved by the rigid
    transform (rotation and translation, no scale) that minimises the squared error (closed form from the
    SVD of the cross-covariance, with the reflection excluded)."""
    est = np.asarray(est, dtype=np.float64)
    gt = np.asarray(gt, dtype=np.float64)
    if align and len(est) >= 3:
        me, mg = est.mean(axis=0), gt.mean(axis=0)
        U, _, Vt = np.linalg.svd((gt - mg).T @ (est - me))
        D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
        R = U @ D @ Vt
        est = (est - me) @ R.T + mg
    return float(np.sqrt(np.mean(np.sum((est - gt) ** 2, axis=1))))


def rot_angle_deg(Ra, Rb):
    """Angle of Ra^T Rb in degrees (from the sine and the cosine: accurate for small angles too)."""
    R = Ra.T @ Rb
    s = 0.5 * np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    c = (np.trace(R) - 1.0) / 2.0
    return float(np.degrees(np.arctan2(s, c)))


def run_mapping(args, seq):
    """Tracking against the fused surfel map on the 640x480 sequence: per frame the model view is predicted
    from the map at the previous estimate (splat rendering, model pyramid), the frame is tracked, and it
    is fused into the map at its new estimate.  The loop waits for each frame's pose (the next prediction
    needs it on the host).  Reports frames/s of the whole loop, the device time of each part (HIP events on
    the stream), the surfel count and the ATE against the ground truth."""
    import torch

    import paper_2207_10940_amd as P
    S = synth_mod()
    n = min(args.map_frames, seq["n_frames"] - 1)
    W, H = seq["camera"].width, seq["camera"].height
    ctx = P.Context(0)
    tp = P.track_params(levels=3, iters=(10, 5, 4), mode="rgbdi", jac="fp32")
    sess = P.Session(ctx, seq["camera"], tp, P.imu_params(), seq["x0"], seq["q_IW"], seq["prior"])
    mp = P.Map(ctx, seq["camera"], args.map_capacity)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    R = S.configs._rot_from_quat

    def pose(x):
        T = np.eye(4)
        T[:3, :3], T[:3, 3] = R(x["q"]), x["r"]
        return T

    sess.build_pyramid(P.PYR_CURRENT, seq["depth"][0].contiguous(), seq["intensity"][0].contiguous(), None, st)
    prev = pose(seq["x0"])
    mp.fuse(sess, prev, st)
    parts = np.zeros(3)
    est = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for j in range(1, n + 1):
        t0, t1 = seq["times"][j - 1], seq["times"][j]
        a, b = S.configs.imu_window(seq["imu"]["t"], t0, t1)
        imu = {k: v[a:b] for k, v in seq["imu"].items()}
        ev[0].record(st)
        mp.predict(sess, prev, st)
        ev[1].record(st)
        sess.track_frame(seq["depth"][j].contiguous(), seq["intensity"][j].contiguous(), imu, t0, t1, st)
        ev[2].record(st)
        r = sess.result()
        prev = pose(r["x1"])
        mp.fuse(sess, prev, st)
        ev[3].record(st)
        ev[3].synchronize()
        parts += [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
        est.append(r["x1"])
    elapsed = time.perf_counter() - t_start
    count, dropped = mp.count()
    acc = sequence_accuracy(est, seq["gt"][1:n + 1])
    deform = run_deformation(args, ctx, mp, st)
    mp.close()
    sess.close()
    ctx.close()
    out = {"workload": f"{W}x{H} sequence, {n} frames: predict the model view from the map at the previous "
                       f"estimate, track (3 levels 10/5/4), fuse at the new estimate",
           "frames_per_s": n / elapsed, "ms_per_frame": elapsed * 1e3 / n,
           "device_ms_per_frame": {"predict": parts[0] / n, "track": parts[1] / n, "fuse": parts[2] / n},
           "surfels": count, "dropped": dropped, "capacity": args.map_capacity,
           "ate_rmse_m": acc["ate_rmse_m"], "ate_rmse_aligned_m": acc["ate_rmse_aligned_m"],
           "max_rot_err_deg": acc["max_rot_err_deg"], "deformation": deform}
    log(f"[mapping] {n} frames in {elapsed * 1e3:.1f} ms ({out['frames_per_s']:.0f} frames/s); device ms/frame "
        f"predict {parts[0] / n:.3f} track {parts[1] / n:.3f} fuse {parts[2] / n:.3f}; {count} surfels; "
        f"ATE {acc['ate_rmse_m'] * 100:.2f} cm, max rotation error {acc['max_rot_err_deg']:.3f} deg")
    return out


def run_deformation(args, ctx, mp, st):
    """A loop-closure deformation of the fused map (the paper's map correction with the gravity term,
    Section V): 64 nodes sampled from the surfels, 256 constraints that pull one part of the map by a
    2 cm / 1 degree drift correction, 128 pinned points elsewhere and 64 earlier registrations (a global
    closure); solved by 5 Gauss-Newton steps on the device and applied to every surfel."""
    import torch

    import paper_2207_10940_amd as P
    rng = np.random.default_rng(77)
    a = mp.arrays()
    pos = np.stack([a["px"], a["py"], a["pz"]], 1).astype(np.float64)
    pos = pos[np.all(np.isfinite(pos), axis=1)]
    nodes = pos[rng.choice(len(pos), args.deform_nodes, replace=False)]
    c = pos.mean(axis=0)
    side = pos[:, 0] > c[0]  # the part of the map the closure moves
    th = np.radians(1.0)
    R = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    t = np.array([0.02, -0.01, 0.0])
    src = pos[side][rng.choice(side.sum(), 256, replace=False)]
    con = [(s, R @ (s - c) + c + t) for s in src]
    pin = list(pos[~side][rng.choice((~side).sum(), 128, replace=False)])
    rs = pos[rng.choice(len(pos), 64, replace=False)]
    rel = [(s, s) for s in rs]
    df = P.Deform(ctx, args.deform_nodes, 512)
    df.solve(nodes, con=con, pin=pin, rel=rel, global_=True, iters=1)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, cost = df.solve(nodes, con=con, pin=pin, rel=rel, global_=True, iters=5)
    t_solve = time.perf_counter() - t0
    df.close()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    mp.deform(nodes, x, st)
    e1.record(st)
    e1.synchronize()
    out = {"nodes": int(args.deform_nodes), "constraints": 256, "pinned": 128, "registrations": 64,
           "gauss_newton_steps": 5, "solve_ms": t_solve * 1e3, "cost_first_step": float(cost[0]),
           "cost_last_step": float(cost[-1]), "apply_ms": e0.elapsed_time(e1), "surfels": int(len(pos))}
    log(f"[deform] {args.deform_nodes} nodes, 256+128+64 points: 5 steps in {t_solve * 1e3:.2f} ms (cost "
        f"{cost[0]:.3e} -> {cost[-1]:.3e}); applied to {len(pos)} surfels in {out['apply_ms']:.3f} ms")
    return out


def sequence_accuracy(est, gt, windows=((0, 30), (30, 100), (100, None))):
    """Tracking accuracy of a sequence against ground truth: the ATE RMSE of the positions (raw and aligned),
    the largest orientation error, and per window of frames the mean error of the velocity and of the two
    bias estimates (the analogue of the paper's convergence plots of the IMU states)."""
    n = len(est)
    err = {k: np.array([np.linalg.norm(np.asarray(e[k]) - np.asarray(g[k])) for e, g in zip(est, gt)])
           for k in ("v", "bg", "ba")}
    R = synth_mod().configs._rot_from_quat
    rot = [rot_angle_deg(R(g["q"]), R(e["q"])) for e, g in zip(est, gt)]
    out = {"frames": n, "ate_rmse_m": ate_rmse([e["r"] for e in est], [g["r"] for g in gt], align=False),
           "ate_rmse_aligned_m": ate_rmse([e["r"] for e in est], [g["r"] for g in gt]),
           "max_rot_err_deg": float(max(rot)), "windows": []}
    for a, b in windows:
        b = n if b is None else min(b, n)
        if a >= b:
            continue
        out["windows"].append({"frames": [a + 1, b], "vel_err_mps": float(err["v"][a:b].mean()),
                               "bg_err_radps": float(err["bg"][a:b].mean()),
                               "ba_err_mps2": float(err["ba"][a:b].mean())})
    return out


ROBUST_LOST_M, ROBUST_LOST_DEG = 0.10, 5.0


def run_robustness(args):
    """The paper's robustness comparison (RGB-D-inertial against RGB-D-only, plus the gyro-aided variant)
    on synthetic stand-ins: one seeded sequence tracked at 30 Hz, with frames skipped (fast motion: the
    same trajectory at 15 and 7.5 Hz), with low-texture albedo, and low texture with the back wall alone
    in view (little photometric and geometric variation).  Every frame is tracked against the
    noise-free model view rendered at the previous frame's estimate (as a dense map would supply it), so
    a frame that fails to converge hands its error on.  Reports per case and estimator the ATE RMSE of
    the current-frame positions (raw and rigidly aligned), the largest orientation error and the frames
    lost (position error above ROBUST_LOST_M or orientation error above ROBUST_LOST_DEG)."""
    import torch

    import paper_2207_10940_amd as P
    S = synth_mod()
    W, H, n = args.robust_width, args.robust_height, args.robust_frames
    t = time.time()
    variants = [("room", False), ("room", True), ("wall", True)]
    seqs = {v: S.configs.sequence(seed=5001, n_frames=n, width=W, height=H, device="cuda",
                                  low_texture_every=1 if v[1] else 0, layout=v[0]) for v in variants}
    log(f"[robust] generated {len(seqs)} sequences x {n} frames {W}x{H} in {time.time() - t:.1f}s")
    cases = [("30 Hz", ("room", False), 1), ("15 Hz", ("room", False), 2), ("7.5 Hz", ("room", False), 4),
             ("low texture, 30 Hz", ("room", True), 1), ("low texture, 7.5 Hz", ("room", True), 4),
             ("flat wall, low texture, 30 Hz", ("wall", True), 1)]
    stream = torch.cuda.current_stream()
    out = {"workload": f"{W}x{H} spline sequence (seed 5001, peak 1.5 m/s and 180 deg/s), {n} frames at 30 Hz, "
                       f"every k-th frame tracked; 3 levels 10/5/4 iterations; model view rendered at the "
                       f"previous estimate; scene: room corner with spheres, or the back wall alone",
           "lost_threshold": {"m": ROBUST_LOST_M, "deg": ROBUST_LOST_DEG}, "cases": {}}
    for name, var, skip in cases:
        seq = seqs[var]
        tex = var[1]
        cam = seq["camera"]
        R_IW = S.configs._rot_from_quat(seq["q_IW_gt"])
        res = {}
        for mode in ("rgbdi", "rgbd", "gyro"):
            ctx = P.Context(0)
            tp = P.track_params(levels=3, iters=(10, 5, 4), mode=mode, jac="fp32")
            sess = P.Session(ctx, cam, tp, P.imu_params(), seq["x0"], seq["q_IW"],
                             seq["prior"] if mode != "rgbd" else None)
            prev = seq["x0"]
            est, gtp, rot_err, lost, failed = [], [], [], 0, 0
            for j in range(skip, n, skip):
                R_WC = S.configs._rot_from_quat(prev["q"])
                z, inten = S.scene.render(seq["scene"], R_IW @ R_WC, R_IW @ prev["r"], W, H, cam.fx, cam.fy,
                                          cam.cx, cam.cy, depth_noise_k=0.0, low_texture=tex, device="cuda")
                T = np.eye(4)
                T[:3, :3], T[:3, 3] = R_WC, prev["r"]
                t0, t1 = seq["times"][j - skip], seq["times"][j]
                a, b = S.configs.imu_window(seq["imu"]["t"], t0, t1)
                imu = {k: v[a:b] for k, v in seq["imu"].items()} if mode != "rgbd" else None
                sess.track_frame_input({"depth": seq["depth"][j].contiguous(),
                                        "intensity": seq["intensity"][j].contiguous(),
                                        "model_depth": z.contiguous(), "model_intensity": inten.contiguous(),
                                        "T_WM": T, "imu": imu, "t0": t0, "t1": t1}, stream)
                r = sess.result()
                failed += r["status"] != 0
                prev = r["x1"]
                g = seq["gt"][j]
                est.append(prev["r"])
                gtp.append(g["r"])
                dr = float(np.linalg.norm(prev["r"] - g["r"]))
                da = rot_angle_deg(S.configs._rot_from_quat(g["q"]), S.configs._rot_from_quat(prev["q"]))
                rot_err.append(da)
                lost += (dr > ROBUST_LOST_M) or (da > ROBUST_LOST_DEG)
            sess.close()
            ctx.close()
            res[mode] = {"ate_rmse_m": ate_rmse(est, gtp, align=False), "ate_rmse_aligned_m": ate_rmse(est, gtp),
                         "max_rot_err_deg": max(rot_err), "lost_frames": int(lost), "failed_frames": int(failed),
                         "frames": len(est)}
        out["cases"][name] = res
        log(f"[robust] {name}: " + "  ".join(f"{m} ATE {v['ate_rmse_m'] * 100:.2f} cm lost {v['lost_frames']}/"
                                            f"{v['frames']}" for m, v in res.items()))
    return out


def _oracle_frames(job):
    """Pool worker of the all-core CPU baseline: track the given frames with the oracle on one thread,
    each from the ground-truth state of the previous frame; returns the seconds spent tracking."""
    from threadpoolctl import threadpool_limits

    from oracle import track
    params = track.default_params(levels=3, iters=(10, 5, 4), mode="rgbdi")
    t = 0.0
    with threadpool_limits(limits=1):
        for f in job:
            t0 = time.perf_counter()
            track.track_frame(*f)
            t += time.perf_counter() - t0
    return t


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(seq, n_single, per_worker):
    """The oracle as it stands, timed on the host: (1) one thread, on the first n_single frames of the
    sequence, chained; (2) every core the process may use (at most 16), one oracle per core, each tracking
    per_worker frames from the previous frame's ground-truth state (the frames of one sequence are
    dependent, so more cores serve more frames, not one frame faster); (3) one thread on the 160x120 frame
    pair (2 levels, 4/4 iterations)."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    import synth
    from oracle import track
    params = track.default_params(levels=3, iters=(10, 5, 4), mode="rgbdi")

    def args_of(j, x0, q, prior):
        md, mi, T, d, i, imu, t0, t1 = frame_inputs(seq, j)
        return (d.cpu().numpy(), i.cpu().numpy(), md.cpu().numpy(), mi.cpu().numpy(), T, seq["camera"], imu, t0, t1,
                x0, q, prior, params)

    x0, q, prior = seq["x0"], seq["q_IW"], seq["prior"]
    t_single = 0.0
    with threadpool_limits(limits=1):
        for j in range(1, n_single + 1):
            a = args_of(j, x0, q, prior)
            t = time.perf_counter()
            o = track.track_frame(*a)
            t_single += time.perf_counter() - t
            x0, q, prior = o["x1"], o["q_IW"], o["prior"]
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    n_all = workers * per_worker
    jobs = [[] for _ in range(workers)]
    for j in range(1, n_all + 1):
        g = seq["gt"][j - 1]
        jobs[(j - 1) % workers].append(args_of(j, g, seq["q_IW"], synth.configs.initial_prior(g, seq["q_IW"])))
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_oracle_frames, [[] for _ in range(workers)])  # start-up and imports outside the timing
        t = time.perf_counter()
        busy = pool.map(_oracle_frames, jobs)
        t_all = time.perf_counter() - t
    d = synth.configs.frame_pair(seed=1001, width=160, height=120)
    pp = track.default_params(levels=2, iters=(4, 4), mode="rgbdi")
    reps = 5
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        for _ in range(reps):
            track.track_frame(d["depth"].numpy(), d["intensity"].numpy(), d["model_depth"].numpy(),
                              d["model_intensity"].numpy(), d["T_WM"], d["camera"], d["imu"], d["t0"], d["t1"],
                              d["x0"], d["q_IW"], d["prior"], pp)
        t_pair = time.perf_counter() - t
    return {"value": n_all / t_all, "unit": "frames/s", "cores": workers, "kind": "oracle",
            "sample": f"{n_all} frames of the 640x480 sequence ({per_worker} per worker, one single-threaded oracle "
                      f"per core, each frame from the previous ground-truth state), 3 levels 10/5/4 iterations, "
                      f"numpy float64 value layer + float32 mask layer",
            "busy_s_per_worker": [float(b) for b in busy], "wall_s": t_all,
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "single_core": {"value": n_single / t_single, "unit": "frames/s", "cores": 1,
                            "sample": f"first {n_single} frames of the 640x480 sequence, chained"},
            "pair_160x120": {"value": reps / t_pair, "unit": "frames/s", "cores": 1,
                             "sample": f"the 160x120 frame pair (seed 1001), 2 levels 4/4 iterations, {reps} times"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=279)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-frames", type=int, default=100)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-frames", type=int, default=10, help="frames of the single-core oracle sample")
    ap.add_argument("--cpu-frames-per-core", type=int, default=2, help="frames per core of the all-core sample")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-frames", type=int, default=24, help="frames per session of the serving workload")
    # steps of 32 sessions, 3 in flight, replayed from graphs: two half-steps overlap each other's latency-bound
    # Gauss-Newton steps, and the graphs keep the host ahead of the twice as many launches
    ap.add_argument("--serving-batch", type=int, default=32, help="server max_batch of the serving workload")
    ap.add_argument("--serving-depth", type=int, default=3, help="server pipeline_depth of the serving workload")
    ap.add_argument("--serving-launch", choices=("eager", "graphs"), default="graphs",
                    help="launch mode whose serving run gives the top-level serving figures")
    ap.add_argument("--serving-warmup", type=float, default=0.25, help="seconds of arrivals left out of latency")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--stress-frames", type=int, default=8, help="frames per session of the stress workload")
    ap.add_argument("--stress-batch", type=int, default=256, help="server max_batch of the stress workload")
    ap.add_argument("--stress-depth", type=int, default=2, help="server pipeline_depth of the stress workload")
    ap.add_argument("--stress-launch", choices=("eager", "graphs"), default="eager",
                    help="launch mode of the stress workload's steps")
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--robust-frames", type=int, default=91, help="frames of the robustness sequences")
    ap.add_argument("--robust-width", type=int, default=320)
    ap.add_argument("--robust-height", type=int, default=240)
    ap.add_argument("--no-robustness", action="store_true")
    ap.add_argument("--map-frames", type=int, default=299, help="frames of the surfel-map tracking loop")
    ap.add_argument("--map-capacity", type=int, default=8_000_000)
    ap.add_argument("--no-mapping", action="store_true")
    ap.add_argument("--deform-nodes", type=int, default=64, help="nodes of the map-deformation problem")
    ap.add_argument("--robustness-only", action="store_true", help="only run the robustness comparison")
    ap.add_argument("--counters", action="store_true",
                    help="only run the level-0 residual pass and a calibration copy (for rocprofv3 --pmc)")
    ap.add_argument("--shapes", default=None,
                    help="JSON list of launch shapes (the \"autotune\" entries of an earlier run) to pin instead "
                         "of running the autotuner")
    ap.add_argument("--counters-batch", action="store_true",
                    help="with --counters: also the batched level-0 pass over a 16-session mix")
    ap.add_argument("--counters-jac", default="fp32", choices=("fp32", "fp32_mfma", "fp16", "bf16"),
                    help="row format of the --counters run (the matrix-core forms for MFMA counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the tracking step shards by session (one process per GPU), and only "
              "the single-GPU figure is measured and reported", file=sys.stderr)
        sys.exit(2)
    if args.counters:
        run_counters(args)
        return
    if args.robustness_only:
        print(json.dumps(run_robustness(args)), flush=True)
        return
    g = run_gpu(args)
    serving = None
    if not args.no_serving:
        serving = run_serving(args)
    stress = None
    if not args.no_stress:
        stress = run_stress(args)
    robust = None
    if not args.no_robustness:
        robust = run_robustness(args)
    mapping = None
    if not args.no_mapping:
        mapping = run_mapping(args, g["seq"])
    precision = None
    if not args.no_precision:
        precision = run_precision()
    cpu = None
    if not args.no_cpu_baseline and args.cpu_frames > 0:
        t = time.time()
        cpu = cpu_baseline(g["seq"], args.cpu_frames, args.cpu_frames_per_core)
        log(f"[bench] cpu baseline {cpu['value']:.3f} frames/s on {cpu['cores']} cores, single core "
            f"{cpu['single_core']['value']:.3f} frames/s, in {time.time() - t:.1f}s")
    out = {
        "metric": METRIC, "value": g["value"], "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": g["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "single-session 640x480 RGB-D-inertial sequence, 3 levels 10/5/4 GN iterations, "
                               "IMU 200 Hz, procedural 3-plane/4-sphere scene", "width": 640, "height": 480,
                   "levels": 3, "iters": [10, 5, 4], "jac_format": "fp32", "frames": args.steps},
        "latency_ms": g["latency_ms"], "pose_err_final_m": g["pose_err_final_m"], "accuracy": g["accuracy"],
        "launch_modes": g["launch_modes"], "autotune": g["autotune"], "roofline": g["roofline"],
        "cpu_baseline": cpu, "precision": precision, "serving": serving, "stress": stress,
        "robustness": robust, "mapping": mapping,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
