#!/usr/bin/env python3
"""Throughput of the stereo VIO frontend on one MI355X.

One step = one frame through the whole frontend (pyramid, FAST grid
detection, temporal tracking of every live keypoint with the forward-backward
check, stereo matching of the new detections, records back on the host). The
default workload is the learned-initialisation comparison's: 1280x720 stereo,
a seeded synthetic 200-frame sequence with 4x texture density, smooth
SE(2)+scale motion and a planar 5..60 px disparity, <= 300 keypoints per
camera, run twice:

* plain: 4 pyramid levels, 5 Gauss-Newton iterations per level from the
  constant-velocity start (the paper's standard configuration);
* learned: the trained network's guess refined with 2 levels and 3
  iterations, falling back to the plain tracker when the short track is not
  kept or its residual is above the network's threshold.

Each leg's sequence is resident in HBM before timing starts. A step stages
one frame's device images of every stream through the C ABI, submits it and
reads the records back. The first timed region of a leg is the production
path: pipelined submission (frame t is submitted before frame t-2's records
are waited for and read, three frames in flight) with the kernels launched one
by one (`--launch graph`: captured graphs; `--no-pipeline`: one frame at a
time). A second region runs the same steps one frame at a time with each
kernel's HIP start/stop events attached to its own dispatch: it gives the
kernel durations behind the roofline figures, with a check that both regions
give identical records. A host-image leg pushes the frames from host memory
one at a time (upload, kernels, fence, readback: the paper's frontend time).
`value` is the frames/s of the faster leg that meets the accuracy bar (median
per-step error against the synthetic ground truth <= 0.1 px, survival within
0.5 points of plain). Prints one JSON line.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3
# FP32 vector without packed (two-per-lane) math, the form the tracker is built in:
# 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_VECTOR_UNPACKED_TFLOPS = 78.6


def copy_peak_gbs(nbytes=1 << 29, reps=10):
    """Achievable device bandwidth on this GPU: a device-to-device copy of nbytes, timed with HIP
    events over reps copies; each copy moves 2 nbytes (read + write). GB/s."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    e.synchronize()
    gbs = 2.0 * nbytes * reps / (s.elapsed_time(e) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs
# Algorithmic FP32 work of the tracker, per level and pass of one keypoint:
# the template (52 samples, gradients, normalisation, J, H, its inverse, G,
# c) about 4.6 kFLOP, one Gauss-Newton iteration (warp, bilinear samples,
# the sums, the update) about 1.25 kFLOP.
F_TEMPLATE = 4600.0
F_ITERATION = 1250.0
MLP_FLOP_PER_ROW = 2 * (32 * 128 + 128 * 128 + 128 * 3)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def track_flops_per_call(levels, iters):
    """Algorithmic FP32 operations of one forward-backward track: two passes of
    `levels` levels, each a template and `iters` iterations (L = 4, N = 5:
    86.8 kFLOP)."""
    return 2 * levels * (F_TEMPLATE + iters * F_ITERATION)


def pyramid_bytes(width, height, levels, cams):
    """Algorithmic HBM bytes of the pyramid+detector launch: level 0 read once
    and levels 1..L-1 written once (the device push's copy of level 0 into the
    frontend's own pyramid is not counted)."""
    a0 = width * height * cams
    p1 = sum((width >> l) * (height >> l) for l in range(1, levels)) * cams
    return a0 + p1


def kernel_source_hash(source):
    """First 16 hex digits of the SHA-256 of a kernel's source file followed by
    every header of the kernel sources (sorted by name), so that a change to a
    shared header counts as a change of the kernel."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2609_30459_amd", "csrc")
    h = hashlib.sha256()
    for path in [os.path.join(csrc, source)] + sorted(glob.glob(os.path.join(csrc, "*.h"))):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed counter profile of this workload,
    or None when the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    k = prof.get("kernels", {}).get(kernel)
    if not k or k.get("traffic_bytes") is None:
        return None
    if kernel_source_hash(k["source"]) != k["source_sha256_16"]:
        return None
    return k["traffic_bytes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps per leg (default 150, batch16 and rig4 80)")
    ap.add_argument("--warmup", type=int, default=10, help="untimed steps before each leg's timed steps (at least 10)")
    ap.add_argument("--workload", default="stereo1280",
                    help="stereo1280 (default), stereo752, rig4, star752, mono320 or batch16")
    ap.add_argument("--seq", type=int, default=0)
    ap.add_argument("--init", choices=["both", "const_vel", "learned"], default="both",
                    help="legs to run: the plain tracker (const_vel), the learned initialisation, or both")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle CPU-baseline budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-host-leg", action="store_true", help="skip the host-image leg")
    ap.add_argument("--launch", choices=["plain", "graph", "eager"], default="plain",
                    help="first timed region: kernels launched one by one without timestamps (default), captured "
                         "graphs, or one by one with HIP events attached to each dispatch")
    ap.add_argument("--in-flight", type=int, choices=[2, 3], default=3,
                    help="frames in flight on the pipelined path (the library allows up to three)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="one frame at a time (no frame submitted before the last one's records are read)")
    ap.add_argument("--no-second-launch", "--no-graph-replay", dest="no_second", action="store_true",
                    help="skip the second timed region (one frame at a time with per-kernel events)")
    ap.add_argument("--weights", default=None, help="learned-init weights (default: the package's for the workload)")
    ap.add_argument("--zero-network", action="store_true",
                    help="ablation: the learned leg with the network's parameters set to zero (guess: no motion), "
                         "same threshold and budgets")
    ap.add_argument("--levels", type=int, default=None, help="override the pyramid levels")
    ap.add_argument("--iters", type=int, default=None, help="override the Gauss-Newton iterations per level")
    ap.add_argument("--k-per-cell", type=int, default=None, help="keypoints per detection cell (default 1)")
    ap.add_argument("--preset", choices=["standard", "lite"], default="standard",
                    help="lite: minimum FAST threshold 20, cells of 82 px, 3 Gauss-Newton iterations (Sec. IV-D)")
    ap.add_argument("--motion", choices=["none", "truth"], default="none",
                    help="truth: each frame's synthetic camera motion as the predicted pose of the camera-model "
                         "start (Sec. III-E), pinhole model of focal --focal over a scene at inverse depth 0.5")
    ap.add_argument("--motion-noise", type=float, default=0.0, metavar="PX",
                    help="Gaussian error (px, per axis) added to the predicted image translation")
    ap.add_argument("--focal", type=float, default=450.0)
    ap.add_argument("--camera", choices=["pinhole", "kb4"], default="pinhole",
                    help="camera model of --motion truth: kb4 = the Kannala-Brandt fisheye model with the first "
                         "four Taylor coefficients of tan (within a fraction of a pixel of the rendered pinhole "
                         "scene near the centre), which takes the fisheye start path")
    ap.add_argument("--pred-levels", type=int, default=0,
                    help="short budget (levels) of tracks with a camera-model start; 0 = the full budget")
    ap.add_argument("--pred-iters", type=int, default=3)
    ap.add_argument("--pred-rho", type=float, default=None,
                    help="residual RMS above which a short predicted track falls back (default: none)")
    ap.add_argument("--learned-levels", type=int, default=2)
    ap.add_argument("--learned-iters", type=int, default=3)
    ap.add_argument("--learned-fb-levels", type=int, default=2,
                    help="learned leg: budget of the fallback from the constant-velocity start (0 = the full one)")
    ap.add_argument("--learned-fb-iters", type=int, default=5)
    ap.add_argument("--learned-stereo", choices=["prior", "neighbour"], default="neighbour",
                    help="learned leg: stereo matches start from the nearest paired keypoint's offset (neighbour) "
                         "or from the disparity prior")
    ap.add_argument("--parallel-fallback", type=int, choices=[0, 1], default=None,
                    help="learned leg: fallbacks computed beside the short attempts (1) or after them (0); "
                         "default: the autotuned choice, else 1 for one stream and 0 for batches")
    ap.add_argument("--stereo-levels", type=int, default=2, help="budget of neighbour-started stereo matches")
    ap.add_argument("--stereo-iters", type=int, default=3)
    ap.add_argument("--waves-per-cu", type=int, default=None,
                    help="tracker grid: 0 = one wave per keypoint, N = persistent N waves per CU "
                         "(default: the autotuned choice, else 0)")
    ap.add_argument("--block-waves", type=int, default=None, help="tracker waves per workgroup (1, 2, 4)")
    ap.add_argument("--learned-block-waves", type=int, choices=[4, 8, 16], default=None,
                    help="keypoints per learned-stage workgroup")
    ap.add_argument("--pyramid-stream", type=int, choices=[0, 1, 2], default=0,
                    help="pyramid beside the tracking, waited for by a signal (0) or an event (1), or in order on "
                         "the launch stream (2)")
    ap.add_argument("--learned-fused", type=int, choices=[0, 1], default=None,
                    help="learned stage inside the tracker launch (default: on for one stream, off when batched)")
    ap.add_argument("--kp-per-wave", type=int, choices=[1, 2], default=None,
                    help="keypoints per tracking wavefront (default: the autotuned choice, else 1); 2 needs the "
                         "learned stage in its own launch")
    ap.add_argument("--tile", type=int, default=None, help="pyramid/detector tile edge (32, 64)")
    ap.add_argument("--stereo-mode", type=int, default=None, help="0 speculative, 1 deferred stereo matching")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run device-to-device copies of BYTES bytes (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": args.calibrate_copy, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the frontend's streams are "
              "independent and would shard across GPUs without communication", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2609_30459_amd as vf
    import synthgen
    from synthgen.workloads import BATCH16

    batched = args.workload == "batch16"
    if args.steps is None:
        from paper_2609_30459_amd.autotune import bench_steps
        args.steps = bench_steps(args.workload)
    warmup = max(args.warmup, 10)
    if batched:
        ws = list(BATCH16)
    else:
        ws = [synthgen.WORKLOADS[args.workload]]
    over = {}
    if args.preset == "lite":
        over.update(thresholds=(40, 20), cell_size=82, gn_iters=3)
    if args.k_per_cell:
        over["k_per_cell"] = args.k_per_cell
    if args.levels:
        over["levels"] = args.levels
    if args.iters:
        over["gn_iters"] = args.iters
    ws = [w.with_(**over) for w in ws]
    w0 = ws[0]
    n_frames = warmup + args.steps
    log(f"rendering {n_frames} frames of {args.workload}: {len(ws)} stream(s), "
        f"{sum(w.n_cams * w.width * w.height for w in ws) / 1e6:.2f} MP per step")
    seqs = [synthgen.sequence(w, seq=args.seq, stream=i, n_frames=n_frames) for i, w in enumerate(ws)]
    devs = [torch.from_numpy(q.frames).cuda() for q in seqs]
    torch.cuda.synchronize()
    streams = [(w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size) for w in ws]
    inits = ["const_vel", "learned"] if args.init == "both" else [args.init]
    short_pred = args.motion != "none" and args.pred_levels > 0
    profiled_config = (args.motion == "none" and args.preset == "standard" and not args.k_per_cell and
                       not args.levels and not args.iters)

    def launch_choice(init):
        """Launch parameters (never change the records): explicit flags, else the autotuned choice."""
        wpc, bw, tile, smode = args.waves_per_cu, args.block_waves, args.tile, args.stereo_mode
        pfb, lbw, lfu, kpw = args.parallel_fallback, args.learned_block_waves, args.learned_fused, args.kp_per_wave
        tuned = None
        if wpc is None and bw is None and tile is None and smode is None:
            from paper_2609_30459_amd import autotune
            tuned = autotune.lookup(args.workload, init)
            if tuned:
                wpc, bw = tuned["track_waves_per_cu"], tuned["track_block_waves"]
                tile, smode = tuned.get("pyr_tile", 64), tuned.get("stereo_mode", 0)
                if pfb is None and "track_parallel_fallback" in tuned:
                    pfb = tuned["track_parallel_fallback"]
                if lbw is None and "learned_block_waves" in tuned:
                    lbw = tuned["learned_block_waves"]
                if lfu is None and "learned_fused" in tuned:
                    lfu = tuned["learned_fused"]
                if kpw is None and "track_kp_per_wave" in tuned:
                    kpw = tuned["track_kp_per_wave"]
        if pfb is None:
            pfb = 0 if batched else 1
        if kpw == 2 and args.learned_fused is None:
            lfu = 0  # the fused learned stage runs one keypoint per wave
        if lfu is None:
            lfu = 0 if batched else 1
        return dict(track_waves_per_cu=wpc or 0, track_block_waves=bw or 4, pyr_tile=tile or 64,
                    stereo_mode=smode or 0, track_parallel_fallback=pfb if init == "learned" else 0,
                    learned_block_waves=(lbw or 0) if init == "learned" else 0,
                    learned_fused=lfu if init == "learned" else 0, pyramid_stream=args.pyramid_stream,
                    track_kp_per_wave=kpw or 1), \
            tuned is not None

    mlp = None
    if "learned" in inits:
        from paper_2609_30459_amd.train_mlp import load_weights
        # the workload's own trained network when there is one, else the stereo1280 one
        wdir = os.path.join(ROOT, "paper_2609_30459_amd", "weights")
        own = os.path.join(wdir, f"mlp_{args.workload}.bin")
        path = args.weights or (own if os.path.exists(own) else os.path.join(wdir, "mlp_stereo1280.bin"))
        params_, rho_, meta = load_weights(path)
        if args.zero_network:
            params_ = np.zeros_like(params_)
        mlp = (params_, rho_, os.path.basename(path) + (" (zeroed)" if args.zero_network else ""))
        log(f"learned init: {path} ({meta}), rho {rho_:.4f}")

    ids = list(range(len(ws)))
    # each frame's device images (views into the resident sequences), all
    # cameras stream by stream, made once before any timed region
    frame_imgs = [[devs[i][t, c] for i, w in enumerate(ws) for c in range(w.n_cams)] for t in range(n_frames)]
    # the push/staging call's pointer and pipelined arrays, built once per frame
    frame_imgs = [vf.Frontend.device_images(f) for f in frame_imgs]
    # camera-model start: the motion of frame t-1 -> t per stream (every camera of a stream takes its
    # first camera's motion), made before any timed region
    motions, K_of = None, None
    if args.motion == "truth":
        inv_depth = 0.5
        rng = np.random.default_rng(1234)
        K_of = [seqs[i].camera_motion(0, args.focal, inv_depth)[0] for i in ids]
        if args.camera == "kb4":
            K_of = [(*K, 1 / 3, 2 / 15, 17 / 315, 62 / 2835) for K in K_of]
        motions = [[None] * n_frames for _ in ws]
        for i, w in enumerate(ws):
            for t in range(1, n_frames):
                _, R, tr = seqs[i].camera_motion(t - 1, args.focal, inv_depth)
                if args.motion_noise > 0:
                    tr = tr.copy()
                    tr[:2] += rng.normal(0.0, args.motion_noise, 2) / (args.focal * inv_depth)
                motions[i][t] = vf.Frontend.motion_array([(c, R, tr, inv_depth) for c in range(w.n_cams)])

    def leg_params(init):
        extra, tuned = launch_choice(init)
        if short_pred:
            extra.update(pred_levels=args.pred_levels, pred_iters=args.pred_iters,
                         pred_rho=args.pred_rho if args.pred_rho is not None else 3.0e38)
        if init == "learned":
            extra.update(init_mode=1, learned_levels=args.learned_levels, learned_iters=args.learned_iters,
                         learned_rho=mlp[1], learned_fb_levels=args.learned_fb_levels,
                         learned_fb_iters=args.learned_fb_iters)
            if args.learned_stereo == "neighbour":
                extra.update(stereo_init=1, stereo_levels=args.stereo_levels, stereo_iters=args.stereo_iters)
        return extra, tuned

    def new_frontend(init, eager=False, plain=False):
        extra, _ = leg_params(init)
        # the streams share one parameter block; per-stream sizes and caps come with the stream
        fe = vf.Frontend(streams, vf.params_for(w0, eager=eager, plain=plain, **extra))
        if init == "learned":
            fe.set_mlp(mlp[0], mlp[1])
        if motions is not None:
            for i, w in enumerate(ws):
                for c in range(w.n_cams):
                    fe.set_camera_model(i, c, K_of[i])
        return fe

    def timed_run(init, eager):
        """Warmup, then the timed steps: (records per stream, wall s per step, stats per step, elapsed s)."""
        fe = new_frontend(init, eager=eager, plain=args.launch == "plain" and not eager)
        records = [[] for _ in ws]
        wall, stats = [], []
        pipelined = not eager and not args.no_pipeline
        depth = args.in_flight
        t_sub = {}

        def submit(t):
            if motions is not None and t > 0:
                for i in ids:
                    fe.set_motion(i, motions[i][t])
            t_sub[t] = time.perf_counter()
            if pipelined:
                fe.stage_frames_device(ids, [t + 1] * len(ws), frame_imgs[t])
                fe.step_async()
            elif batched:
                fe.stage_frames_device(ids, [t + 1] * len(ws), frame_imgs[t])
                fe.step()
            else:
                fe.push_stereo_frame_device(0, t + 1, frame_imgs[t])

        def collect(t):
            if pipelined:
                fe.wait()
            if batched or pipelined:
                for i, r in enumerate(fe.get_tracks_many(ids)):
                    records[i].append(r)
            else:
                records[0].append(fe.get_tracks(0))
            return time.perf_counter() - t_sub.pop(t)

        # no garbage-collector pause inside the warmup or the timed steps, and
        # no idle gap between them (the device would lower its clocks in one)
        gc.collect()
        gc.disable()
        log(f"{init}: warmup {warmup} steps ({'eager' if eager else args.launch}"
            f"{f', {depth} frames in flight' if pipelined else ''}), then {args.steps} timed steps")
        # the warmup runs the timed region's own loop (pipelined when it is), so
        # the first timed frames find its code paths and buffers warm
        for t in range(warmup):
            submit(t)
            if not pipelined:
                collect(t)
            elif t >= depth - 1:
                collect(t - depth + 1)
        if pipelined:
            for t in range(max(0, warmup - depth + 1), warmup):
                collect(t)
        torch.cuda.synchronize()
        # the production region reads only the records; the eager region also
        # each frame's statistics (kernel times, device time, fallbacks)
        t0 = time.perf_counter()
        for t in range(warmup, n_frames):
            submit(t)
            if pipelined:
                # frame t - depth + 1 is read while the later ones run
                if t - warmup >= depth - 1:
                    wall.append(collect(t - depth + 1))
            else:
                wall.append(collect(t))
                if eager:
                    stats.append(fe.stats())
        if pipelined:
            for t in range(max(warmup, n_frames - depth + 1), n_frames):
                wall.append(collect(t))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        gc.enable()
        fe.close()
        return records, wall, stats, elapsed

    def host_run(init):
        """The paper's frontend time: host images pushed one frame at a time (H2D upload, kernels, fence,
        records back), host wall clock per frame."""
        fe = new_frontend(init)
        host = [q.frames for q in seqs]
        wall = []
        log(f"{init}: host-image leg, {warmup} + {args.steps} frames")
        for t in range(n_frames):
            if motions is not None and t > 0:
                for i in ids:
                    fe.set_motion(i, motions[i][t])
            t0 = time.perf_counter()
            if batched:
                for i, w in enumerate(ws):
                    fe.stage_frame(i, t + 1, list(host[i][t]))
                fe.step()
                fe.get_tracks_many(ids)
            else:
                fe.push_stereo_frame(0, t + 1, list(host[0][t]))
                fe.get_tracks(0)
            if t >= warmup:
                wall.append(time.perf_counter() - t0)
        fe.close()
        ms = np.array(wall) * 1e3
        return {"value": len(ws) * 1e3 / ms.mean(), "unit": "stream-frames/s" if batched else "frames/s",
                "ms_per_frame": float(ms.mean()), "p50_ms": float(np.percentile(ms, 50)),
                "p99_ms": float(np.percentile(ms, 99)),
                "h2d_bytes_per_frame": sum(w.n_cams * w.width * w.height for w in ws)}

    TR, DET, MAT = vf.VIO_TRACKED, vf.VIO_DETECTED, vf.VIO_MATCHED

    def leg(init):
        first_eager = args.launch == "eager"
        records, wall, stats, elapsed = timed_run(init, first_eager)
        steps_per_s = args.steps / elapsed
        second, eager_stats = None, stats if first_eager else None
        if not args.no_second:
            rec2, wall2, stats2, elapsed2 = timed_run(init, not first_eager)
            same = all(a.tobytes() == b.tobytes() for ra, rb in zip(records, rec2) for a, b in zip(ra, rb))
            second = {"launch": "graph" if first_eager else "eager",
                      "value": args.steps * len(ws) / elapsed2, "ms_per_step": 1000.0 * elapsed2 / args.steps,
                      "gpu_ms_per_step": float(np.mean([s_["last_gpu_ms"] for s_ in stats2])) if stats2 else None,
                      "latency_p50_ms": float(np.percentile(np.array(wall2) * 1e3, 50)),
                      "latency_p99_ms": float(np.percentile(np.array(wall2) * 1e3, 99)),
                      "records_identical": bool(same)}
            if not first_eager:
                eager_stats = stats2
        # per-frame statistics of the eager region (the same records as the
        # first region, so the same fallbacks); [steps, 6]: pyramid+detector,
        # tracker, selection, learned stage, (unused), whole frame
        kstats = eager_stats or [{"last_stage_ms": [-1.0] * 3, "last_learned_ms": [-1.0] * 2, "last_gpu_ms": -1.0,
                                  "last_fallback": 0}]
        fallbacks = np.array([s_["last_fallback"] for s_ in kstats], np.float64)
        sm = np.array([s_["last_stage_ms"] + s_["last_learned_ms"] + [s_["last_gpu_ms"]] for s_ in kstats])
        mean_ms = sm.mean(0)
        have_times = bool((sm[:, :3] >= 0).all())

        # tracked keypoints and accuracy against the synthetic ground truth
        tracked = np.zeros(args.steps)
        n_temporal = np.zeros(args.steps)
        n_stereo = np.zeros(args.steps)
        errs, serrs, n_tr, n_lost = [], [], 0, 0
        for i, (w, seq) in enumerate(zip(ws, seqs)):
            rec = records[i]
            # records[i] holds the warmup frames too: frame t is rec[t]
            for k, t in enumerate(range(warmup, n_frames)):
                tracked[k] += int((rec[t]["status"] == TR).sum())
                n_temporal[k] += int(np.isin(rec[t - 1]["status"], [TR, DET, MAT]).sum())
                # each detection is matched into the pair's right camera, or a star's three other cameras
                n_stereo[k] += int((rec[t]["status"] == DET).sum()) * (3 if w.star else 1) if w.stereo else 0
            e, se, tr, lo = accuracy(w, seq, rec, TR, DET, MAT)
            errs += e
            serrs += se
            n_tr += tr
            n_lost += lo
        err = np.concatenate(errs) if errs else np.zeros(1)
        serr = np.concatenate(serrs) if serrs else np.zeros(1)
        survival = n_tr / max(1, n_tr + n_lost)

        L, N = w0.levels, w0.gn_iters
        if init == "learned":
            # every temporal track runs the short tracker, fallbacks the fallback budget; stereo matches
            # run the neighbour budget (every match after the first frame has a paired neighbour) or the full one
            fbl = args.learned_fb_levels or L
            fbi = args.learned_fb_iters if args.learned_fb_levels else N
            stereo_f = (track_flops_per_call(args.stereo_levels, args.stereo_iters)
                        if args.learned_stereo == "neighbour" else track_flops_per_call(L, N))
            flops_step = (n_temporal * track_flops_per_call(args.learned_levels, args.learned_iters) +
                          fallbacks * track_flops_per_call(fbl, fbi) + n_stereo * stereo_f)
        elif short_pred:
            flops_step = (n_temporal * track_flops_per_call(args.pred_levels, args.pred_iters) +
                          (fallbacks + n_stereo) * track_flops_per_call(L, N))
        else:
            flops_step = (n_temporal + n_stereo) * track_flops_per_call(L, N)
        pyr_b = sum(pyramid_bytes(w.width, w.height, L, w.n_cams) for w in ws)
        pyr_gbs = pyr_b / (mean_ms[0] * 1e-3) / 1e9 if have_times else None
        trk_tf = float(flops_step.mean()) / (mean_ms[1] * 1e-3) / 1e12 if have_times else None
        kernels = {
            "k_pyr_detect": {"bound": "hbm", "avg_ms": float(mean_ms[0]), "bytes_per_launch": pyr_b,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "achieved": pyr_gbs,
                             "copy_peak": copy_gbs,
                             "frac_of_copy": pyr_gbs / copy_gbs if pyr_gbs is not None else None},
            "k_track": {"bound": "alu", "avg_ms": float(mean_ms[1]),
                        "calls_per_launch": float((n_temporal + n_stereo).mean()),
                        "flops_per_launch": float(flops_step.mean()), "peak": FP32_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "achieved": trk_tf, "peak_unpacked": FP32_VECTOR_UNPACKED_TFLOPS,
                        "frac_unpacked": trk_tf / FP32_VECTOR_UNPACKED_TFLOPS if trk_tf is not None else None},
            "k_select": {"bound": "latency", "avg_ms": float(mean_ms[2])},
        }
        if init == "learned":
            rows = n_temporal.mean()
            kernels["learned_stage"] = {"bound": "latency", "avg_ms": float(sm[:, 3].mean() + max(0.0, sm[:, 4].mean())),
                                        "rows_per_launch": float(rows), "mfma_flops_per_launch": MLP_FLOP_PER_ROW * rows}
        roof = None
        if have_times:
            dom = ["k_pyr_detect", "k_track"][int(np.argmax(mean_ms[:2]))]
            kd = kernels[dom]
            roof = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                    "unit": kd["unit"], "frac": kd["achieved"] / kd["peak"],
                    "traffic": measured_traffic(f"{args.workload}_{'plain' if init == 'const_vel' else init}", dom)
                    if profiled_config else None,
                    "avg_ms": kd["avg_ms"]}
        wall_ms = np.array(wall) * 1e3
        extra, tuned = leg_params(init)
        return {
            "value": steps_per_s * len(ws), "ms_per_step": 1000.0 / steps_per_s,
            "tracked_kpts_per_s": float(tracked.mean()) * steps_per_s,
            "gpu_ms_per_step": float(mean_ms[5]),
            "latency_ms": {"p50": float(np.percentile(wall_ms, 50)), "p99": float(np.percentile(wall_ms, 99)),
                           "gpu_p50": float(np.percentile(sm[:, 5], 50)),
                           "gpu_p99": float(np.percentile(sm[:, 5], 99))},
            "accuracy": {"temporal_median_px": float(np.median(err)),
                         "temporal_p90_px": float(np.percentile(err, 90)),
                         "stereo_median_px": float(np.median(serr)), "survival": survival},
            "fallback_per_step": float(fallbacks.mean()) if init == "learned" or short_pred else None,
            "budget": ({"levels": args.learned_levels, "iters": args.learned_iters,
                        "fallback_levels": args.learned_fb_levels or L,
                        "fallback_iters": args.learned_fb_iters if args.learned_fb_levels else N,
                        "stereo_start": args.learned_stereo,
                        **({"stereo_levels": args.stereo_levels, "stereo_iters": args.stereo_iters}
                           if args.learned_stereo == "neighbour" else {}),
                        "rho": mlp[1], "weights": mlp[2]} if init == "learned"
                       else {"levels": L, "iters": N, "stereo_start": "prior"}),
            "launch": {**{k: v for k, v in extra.items() if k in ("track_waves_per_cu", "track_block_waves",
                                                                   "pyr_tile", "stereo_mode",
                                                                   "track_parallel_fallback", "learned_block_waves",
                                                                   "learned_fused", "pyramid_stream",
                                                                   "track_kp_per_wave")},
                       "autotuned": tuned},
            "roofline": roof, "second_launch": second, "kernels": kernels,
            "host_image": None if args.no_host_leg else host_run(init),
        }

    # the achievable device bandwidth beside the vendor figure (before the legs: nothing else runs)
    copy_gbs = copy_peak_gbs()
    log(f"device copy: {copy_gbs:.0f} GB/s")
    legs = {init: leg(init) for init in inits}

    # value: the faster leg that meets the accuracy bar (median <= 0.1 px; survival within 0.5 points of plain)
    base_surv = legs["const_vel"]["accuracy"]["survival"] if "const_vel" in legs else None
    ok = {k: v["accuracy"]["temporal_median_px"] <= 0.1 and
          (base_surv is None or v["accuracy"]["survival"] >= base_surv - 0.005) for k, v in legs.items()}
    for k, v in legs.items():
        v["meets_accuracy_bar"] = ok[k]
    cand = [k for k in legs if ok[k]] or list(legs)
    best = max(cand, key=lambda k: legs[k]["value"])
    if "const_vel" in legs and "learned" in legs:
        legs["learned"]["speedup_vs_plain"] = legs["learned"]["value"] / legs["const_vel"]["value"]
        if legs["learned"]["host_image"] and legs["const_vel"]["host_image"]:
            legs["learned"]["host_image"]["speedup_vs_plain"] = (legs["learned"]["host_image"]["value"] /
                                                                 legs["const_vel"]["host_image"]["value"])

    # ---- CPU baseline: the oracle on a bounded sample of the same workload (plain tracker) ----
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nproc = os.cpu_count() or 1
        model = cpu_model_name()
        unit = "stream-frames/s" if batched else "frames/s"

        def new_oracles():
            return [oracle.Frontend([w.width] * w.n_cams, [w.height] * w.n_cams, w.stereo, oracle.params_for(w))
                    for w in ws]

        log(f"cpu baseline: oracle for up to {args.cpu_seconds:.0f} s (one thread)")
        fos = new_oracles()
        n, c0 = 0, time.perf_counter()
        while n < n_frames and (time.perf_counter() - c0 < args.cpu_seconds or n < 3):
            for fo, q in zip(fos, seqs):
                fo.push(list(q.frames[n]))
                fo.records()
            n += 1
        cpu_s = time.perf_counter() - c0
        for fo in fos:
            fo.close()
        cpu = {"value": n * len(ws) / cpu_s, "unit": unit, "cores": 1, "kind": "oracle",
               "sample": f"first {n} frames of the same {args.workload} sequence(s), plain tracker, single-threaded "
                         f"C++ oracle (-O2), {cpu_s:.1f} s", "nproc": nproc, "cpu_model": model}
        if batched:
            from concurrent.futures import ThreadPoolExecutor
            threads = min(len(ws), nproc)
            log(f"cpu baseline: oracle, one thread per stream ({threads} threads), {n} frames")
            fos = new_oracles()

            def run_stream(i):
                for t in range(n):
                    fos[i].push(list(seqs[i].frames[t]))
                    fos[i].records()

            c0 = time.perf_counter()
            with ThreadPoolExecutor(max_workers=threads) as ex:
                list(ex.map(run_stream, range(len(ws))))
            thr_s = time.perf_counter() - c0
            for fo in fos:
                fo.close()
            cpu["threaded"] = {"value": n * len(ws) / thr_s, "unit": unit, "threads": threads,
                               "sample": f"the same {n} frames, one thread per stream, {thr_s:.1f} s"}

    vb = legs[best]
    out = {
        "metric": "stereo frames/s + tracked kpts/s, plain vs learned-init KLT at <=0.1px err",
        "value": vb["value"],
        "unit": "stream-frames/s" if batched else "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": vb["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "value_leg": best, "legs": inits, "streams": len(ws),
                   "cameras": sum(w.n_cams for w in ws),
                   "sizes": sorted({f"{w.width}x{w.height}x{w.n_cams}" for w in ws}),
                   "levels": w0.levels, "gn_iters": w0.gn_iters, "max_keypoints": sorted({w.max_keypoints for w in ws}),
                   "preset": args.preset, "k_per_cell": w0.k_per_cell,
                   "motion": args.motion, **({"motion_noise_px": args.motion_noise, "focal": args.focal,
                                              "camera": args.camera} if args.motion != "none" else {}),
                   **({"pred_levels": args.pred_levels, "pred_iters": args.pred_iters, "pred_rho": args.pred_rho}
                      if short_pred else {}),
                   "cell_size": sorted({w.cell_size for w in ws}), "thresholds": list(w0.thresholds),
                   "launch": args.launch, "pipelined": args.launch != "eager" and not args.no_pipeline,
                   "in_flight": args.in_flight if args.launch != "eager" and not args.no_pipeline else 1,
                   "parallelism": "single_gpu"},
        "tracked_kpts_per_s": vb["tracked_kpts_per_s"],
        "gpu_ms_per_step": vb["gpu_ms_per_step"],
        "latency_ms": vb["latency_ms"],
        "accuracy": vb["accuracy"],
        "roofline": vb["roofline"],
        "hbm_copy": {"gbs": copy_gbs, "vendor_peak_gbs": HBM_PEAK_GBS, "frac_of_vendor": copy_gbs / HBM_PEAK_GBS,
                     "bytes_per_copy": 2 * (1 << 29)},
        "legs": legs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def accuracy(w, seq, rec, TR, DET, MAT):
    """Temporal and stereo errors against the ground truth, tracked and lost counts."""
    errs, serrs, n_tr, lost = [], [], 0, 0
    for t in range(1, len(rec)):
        prev, cur = rec[t - 1], rec[t]
        live = np.isin(prev["status"], [TR, DET, MAT])
        n_tr += int((cur["status"] == TR).sum())
        for c in range(w.n_cams):
            pc = prev[live & (prev["camera"] == c)]
            pos = {int(i): (x, y) for i, x, y in zip(pc["id"], pc["x"], pc["y"])}
            cc = cur[(cur["camera"] == c) & (cur["status"] == TR)]
            if len(cc):
                px = np.array([pos[int(i)][0] for i in cc["id"]])
                py = np.array([pos[int(i)][1] for i in cc["id"]])
                gx, gy = seq.gt_temporal(t - 1, c, px, py)
                errs.append(np.hypot(cc["x"] - gx, cc["y"] - gy))
            lost += int(((cur["camera"] == c) & (cur["age"] > 0) & ~np.isin(cur["status"], [TR, DET, MAT])).sum())
        if w.stereo:
            # groups: stereo pairs, or a star rig whose first camera's detections go to the other three
            group = 4 if w.star else 2
            for c in range(0, w.n_cams, group):
                dl = cur[(cur["camera"] == c) & (cur["status"] == DET)]
                lpos = {int(i): (x, y) for i, x, y in zip(dl["id"], dl["x"], dl["y"])}
                for tc in range(c + 1, c + group):
                    mr = cur[(cur["camera"] == tc) & (cur["status"] == MAT)]
                    if len(mr):
                        lx = np.array([lpos[int(i)][0] for i in mr["id"]])
                        ly = np.array([lpos[int(i)][1] for i in mr["id"]])
                        gx, gy = seq.gt_stereo(c, lx, ly, tc)
                        serrs.append(np.hypot(mr["x"] - gx, mr["y"] - gy))
    return errs, serrs, n_tr, lost


if __name__ == "__main__":
    main()
