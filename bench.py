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
COPY_BYTES = 256 << 20  # calibration copy for the HBM byte counters
# HBM bytes per level-0 residual launch from rocprofv3 FETCH_SIZE / WRITE_SIZE, each scaled by the
# reading of a 256 MiB copy (fetch x1.99985, write x1.0); valid for the kernel source with this hash.
TRAFFIC_BYTES_LEVEL0 = (7810.9 * 262144 / 131085.1 + 150.0) * 1024
TRAFFIC_SOURCE_SHA256 = "fd49821d72aecd30"
# bytes the residual pass reads per pixel-iteration: current vertex 12 + intensity 2, model-view vertex 12 +
# normal 12 + intensity 2 + gradient 4 (16-bit fixed-point intensity and gradient; N1 unread without the
# normal gate)
REF_BYTES_PER_PIXEL = 44


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


def measured_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2207_10940_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()
    return TRAFFIC_BYTES_LEVEL0 if h.startswith(TRAFFIC_SOURCE_SHA256) else None


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
        t = time.perf_counter()
        track(k)
        sess.result()
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat[5:] if len(lat) > 10 else lat)
    log(f"[bench] latency over {len(lat)} frames: p50 {np.percentile(lat, 50):.3f} ms p99 {np.percentile(lat, 99):.3f} ms")

    # accuracy over the whole sequence, frame by frame from the initial state (outside the timed region):
    # the analogue of the paper's velocity / bias convergence plots and its ATE RMSE
    sess.set_state(*x_init)
    est = []
    for k in range(n_frames - 1):
        track(k)
        est.append(sess.result()["x1"])
    accuracy = sequence_accuracy(est, seq["gt"][1:n_frames])
    log(f"[bench] accuracy over {len(est)} frames: ATE {accuracy['ate_rmse_m'] * 100:.3f} cm, velocity error "
        f"{accuracy['windows'][-1]['vel_err_mps']:.2e} m/s, gyro bias {accuracy['windows'][-1]['bg_err_radps']:.2e} "
        f"rad/s, accel bias {accuracy['windows'][-1]['ba_err_mps2']:.2e} m/s^2 (last window)")

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
    achieved = REF_BYTES_PER_PIXEL * px / (k_ms * 1e-3) / 1e9
    log(f"[bench] level-0 residual pass: {k_ms * 1e3:.2f} us/launch, {achieved:.1f} GB/s ({REF_BYTES_PER_PIXEL} B/px algorithmic)")
    sess.close()
    ctx.close()
    return {
        "value": args.steps / elapsed, "ms_per_step": elapsed * 1e3 / args.steps,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "frames": int(len(lat)), "kind": "host submit to result, one frame at a time"},
        "pose_err_final_m": pos_err,
        "accuracy": accuracy,
        "launch_modes": launch_modes,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "residual_kernel<2> (level 0, 640x480)", "kernel_us": k_ms * 1e3,
                     "bytes_per_launch": REF_BYTES_PER_PIXEL * px},
        "seq": seq,
    }


def run_counters(args):
    """Hardware-counter run: the level-0 residual pass on a tracked sequence frame, then a plain
    device copy of known size whose FETCH_SIZE / WRITE_SIZE readings scale the counters to bytes.
    Meant to be run under rocprofv3 --pmc; prints one JSON line describing what ran."""
    import torch

    import paper_2207_10940_amd as P
    W, H = 640, 480
    seq = make_sequence(4, W, H, "cuda")
    ctx = P.Context(0)
    tp = P.track_params(levels=3, iters=(10, 5, 4), mode="rgbdi", jac=args.counters_jac)
    sess = P.Session(ctx, seq["camera"], tp, P.imu_params(), seq["x0"], seq["q_IW"], seq["prior"])
    stream = torch.cuda.current_stream()
    for j in range(1, 4):
        md, mi, T, d, i, imu, t0, t1 = frame_inputs(seq, j)
        sess.set_model(md.contiguous(), mi.contiguous(), T, stream)
        sess.track_frame(d.contiguous(), i.contiguous(), imu, t0, t1, stream)
    torch.cuda.synchronize()
    sess.profile_residual(0, args.kernel_reps, stream)
    torch.cuda.synchronize()
    n = COPY_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    sess.close()
    ctx.close()
    print(json.dumps({"counters_run": True, "jac": args.counters_jac, "residual_reps": args.kernel_reps,
                      "residual_pixels": W * H,
                      "copy_bytes_each_way": COPY_BYTES, "copy_reps": 3}), flush=True)


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
    for ci, (w, h, count) in enumerate(SERVING_MIX):
        nseq = min(count, args.serving_sequences)
        seqs[(w, h)] = [synth.configs.sequence(seed=4000 + 100 * ci + k, n_frames=nf + 1, width=w, height=h,
                                               device="cuda", duration=(nf + 3) / 30.0) for k in range(nseq)]
        specs += [(w, h, k % nseq) for k in range(count)]
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

    server = P.Server(ctx, max_batch=len(sess), pipeline_depth=2)
    total = len(sess) * nf
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
    log(f"[serving] saturation: {total} frames in {t_sat * 1e3:.1f} ms = {sat_fps:.0f} frames/s, "
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
    log(f"[serving] nominal 30 Hz x {len(sess)}: p50 {np.percentile(lat, 50):.2f} ms p99 "
        f"{np.percentile(lat, 99):.2f} ms over {len(lat)} frames, mean batch {np.mean(sizes_nom):.1f}")
    server.close()
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
    batch.profile_residual(0, 5, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(stream)
    px = batch.profile_residual(0, reps, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / reps
    gbs = REF_BYTES_PER_PIXEL * px / (k_ms * 1e-3) / 1e9
    log(f"[serving] batched level-0 residual pass: {px} px in {k_ms * 1e3:.1f} us = {gbs:.0f} GB/s")
    batch.close()
    for s in sess:
        s.close()
    ctx.close()
    return {
        "workload": "64 sessions: 8 at 1280x720, 32 at 640x480, 24 at 320x240; 3 levels 10/5/4 iterations, "
                    "RGB-D-inertial, float32 Jacobians; continuous batching, 2 steps in flight",
        "frames": total, "distinct_sequences_per_resolution": args.serving_sequences,
        "saturation_fps": sat_fps, "saturation_mean_batch": float(np.mean(sizes)),
        "saturation_device_ms_per_step_p50": float(np.percentile(dev_ms, 50)),
        "nominal": {"offered_fps": 30.0 * len(sess), "achieved_fps": total / span,
                    "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                    "device_p50_ms": float(np.percentile(dev_nom, 50)), "frames": len(lat),
                    "mean_batch": float(np.mean(sizes_nom)),
                    "kind": "arrival (Poisson, 30 Hz per session) to result on the host"},
        "plain_fps_same_mix": plain_fps, "plain_ms_per_frame": {k: v * 1e3 for k, v in per_class.items()},
        "speedup_vs_plain": sat_fps / plain_fps,
        "failed": int(bad),
        "batched_residual_roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": gbs / HBM_PEAK_GBS, "kernel_us": k_ms * 1e3, "pixels": px,
                                      "bytes_per_launch": REF_BYTES_PER_PIXEL * px},
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


def run_stress(args):
    """Serving + precision stress: 256 sessions (64 each at 1920x1080, 1280x720, 640x480, 320x240), FP16
    Jacobian rows on MFMA with float64 solves, tile shapes from the autotuner, 5% of frames with 80% zero-depth
    holes and 10% low-texture frames; saturation throughput, latency under bursty (Markov-modulated Poisson)
    arrivals, and the pose error of sampled sessions against the oracle."""
    import torch

    import paper_2207_10940_amd as P
    synth = synth_mod()
    nf, nseq = args.stress_frames, args.stress_sequences
    rng = np.random.default_rng(5)
    t = time.time()
    seqs, specs, flags = {}, [], {"holes": 0, "low_texture": 0, "frames": 0}
    for ci, (w, h, count) in enumerate(STRESS_MIX):
        lst = []
        for k in range(nseq):
            holes = [j for j in range(1, nf + 1) if rng.random() < 0.05]
            lowt = [j for j in range(1, nf + 1) if rng.random() < 0.10]
            flags["holes"] += len(holes)
            flags["low_texture"] += len(lowt)
            flags["frames"] += nf
            lst.append(synth.configs.sequence(seed=5000 + 100 * ci + k, n_frames=nf + 1, width=w, height=h,
                                              device="cuda", duration=(nf + 3) / 30.0, hole_frames=holes,
                                              low_texture_frames=lowt))
        seqs[(w, h)] = lst
        specs += [(w, h, k % nseq) for k in range(count)]
    frames = {key: [[serving_frame(sq, j) for j in range(1, nf + 1)] for sq in lst] for key, lst in seqs.items()}
    fins = {key: [[P.frame_input(f)[0] for f in fl] for fl in lst] for key, lst in frames.items()}
    torch.cuda.synchronize()
    log(f"[stress] generated {sum(len(v) for v in seqs.values())} sequences x {nf} frames in {time.time() - t:.1f}s "
        f"({flags['holes']} hole frames, {flags['low_texture']} low-texture of {flags['frames']})")
    ctx = P.Context(0)
    tuned = ctx.autotune([seqs[(w, h)][0]["camera"] for w, h, _ in STRESS_MIX], levels=3, jac="fp16")
    log("[stress] autotuned pixels per thread: " +
        ", ".join(f"{e['width']}x{e['height']} L{e['level']}: {e['ppt']} ({e['us']:.1f} us)" for e in tuned))
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

    server = P.Server(ctx, max_batch=len(sess), pipeline_depth=2)
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
    # ---- pose error of sampled sessions (first frame from the initial state) against the oracle
    from oracle import track
    pose = {}
    for w, h in ((320, 240), (640, 480)):
        i = next(n for n, sp in enumerate(specs) if sp[:2] == (w, h))
        sq = seqs[(w, h)][specs[i][2]]
        f = frames[(w, h)][specs[i][2]][0]
        params = track.default_params(levels=3, iters=(10, 5, 4), mode="rgbdi")
        o = track.track_frame(f["depth"].cpu().numpy(), f["intensity"].cpu().numpy(),
                              f["model_depth"].cpu().numpy(), f["model_intensity"].cpu().numpy(), f["T_WM"],
                              sq["camera"], f["imu"], f["t0"], f["t1"], sq["x0"], sq["q_IW"], sq["prior"], params)
        g = first[i]
        from oracle import lie
        pose[f"{w}x{h}"] = {"m": float(np.linalg.norm(g["x1"]["r"] - o["x1"]["r"])),
                            "rad": float(np.linalg.norm(lie.quat_boxminus(g["x1"]["q"], o["x1"]["q"])))}
    log(f"[stress] pose vs oracle (fp16): {pose}")
    return {
        "workload": "256 sessions: 64 each at 1920x1080, 1280x720, 640x480, 320x240; RGB-D-inertial, 3 levels "
                    "10/5/4, FP16 Jacobian rows on MFMA, float64 solve; 5% of frames with 80% zero-depth holes, "
                    "10% low-texture; Markov-modulated Poisson arrivals (30 Hz mean, x3 / x0.33 states)",
        "frames": total, "hole_frames": flags["holes"], "low_texture_frames": flags["low_texture"],
        "distinct_sequences_per_resolution": nseq, "hbm_bytes_admitted": hbm,
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


def cpu_baseline(seq, n_frames):
    """The oracle as it stands, single-threaded, on the first frames of the same sequence."""
    from threadpoolctl import threadpool_limits

    from oracle import track
    params = track.default_params(levels=3, iters=(10, 5, 4), mode="rgbdi")
    x0, q, prior = seq["x0"], seq["q_IW"], seq["prior"]
    t_total = 0.0
    with threadpool_limits(limits=1):
        for j in range(1, n_frames + 1):
            md, mi, T, d, i, imu, t0, t1 = frame_inputs(seq, j)
            args = [d.cpu().numpy(), i.cpu().numpy(), md.cpu().numpy(), mi.cpu().numpy()]
            t = time.perf_counter()
            o = track.track_frame(*args, T, seq["camera"], imu, t0, t1, x0, q, prior, params)
            t_total += time.perf_counter() - t
            x0, q, prior = o["x1"], o["q_IW"], o["prior"]
    return {"value": n_frames / t_total, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_frames} tracked frames of the 640x480 sequence, 3 levels 10/5/4 iterations, "
                      f"numpy float64 value layer + float32 mask layer, BLAS limited to 1 thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=279)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-frames", type=int, default=100)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-frames", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-frames", type=int, default=40, help="frames per session of the serving workload")
    ap.add_argument("--serving-sequences", type=int, default=6,
                    help="distinct seeded sequences per resolution of the serving workload")
    ap.add_argument("--serving-warmup", type=float, default=0.25, help="seconds of arrivals left out of latency")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--stress-frames", type=int, default=12, help="frames per session of the stress workload")
    ap.add_argument("--stress-sequences", type=int, default=4,
                    help="distinct seeded sequences per resolution of the stress workload")
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
    cpu = None
    if not args.no_cpu_baseline and args.cpu_frames > 0:
        t = time.time()
        cpu = cpu_baseline(g["seq"], args.cpu_frames)
        log(f"[bench] cpu baseline {cpu['value']:.3f} frames/s in {time.time() - t:.1f}s")
    out = {
        "metric": METRIC, "value": g["value"], "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": g["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "single-session 640x480 RGB-D-inertial sequence, 3 levels 10/5/4 GN iterations, "
                               "IMU 200 Hz, procedural 3-plane/4-sphere scene", "width": 640, "height": 480,
                   "levels": 3, "iters": [10, 5, 4], "jac_format": "fp32", "frames": args.steps},
        "latency_ms": g["latency_ms"], "pose_err_final_m": g["pose_err_final_m"], "accuracy": g["accuracy"],
        "launch_modes": g["launch_modes"], "roofline": g["roofline"], "cpu_baseline": cpu, "serving": serving, "stress": stress,
        "robustness": robust, "mapping": mapping,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
