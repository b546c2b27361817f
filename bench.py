#!/usr/bin/env python3
"""Throughput of the stereo VIO frontend on one MI355X.

One step = one frame through the whole frontend (pyramid, FAST grid
detection, temporal tracking of every live keypoint with the forward-backward
check, stereo matching of the new detections, records back on the host). The
default workload is 752x480 stereo: a seeded synthetic 200-frame sequence with
4x texture density, smooth SE(2)+scale motion and a planar 5..60 px disparity,
4 pyramid levels, 5 Gauss-Newton iterations per level, <= 300 keypoints per
camera.

The sequences are resident in HBM before timing starts. A step stages one
frame's device images of every stream of the workload through the C ABI,
submits it, and reads the records back. The first timed region is the
production path and gives `value`: pipelined submission (frame t is submitted
before frame t-1's records are waited for and read, two frames in flight) with
the kernels launched one by one without timestamps (`--launch graph`:
captured graphs; `--no-pipeline`: one frame at a time, the paper's
submit-and-wait). A second timed region runs the same steps one frame at a
time with each kernel's HIP start/stop events attached to its own dispatch: it
gives the kernel durations behind the roofline figures and is reported beside
the first (`second_launch`, with a check that both give identical records).
Prints one JSON line.
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
PATTERN = 52


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
    """Algorithmic FP32 operations of one forward-backward track.

    Counting convention (per pattern point, multiply and add counted
    separately): template per level 122 (5 bilinear samples at 13, sample
    positions 4, gradients 4, normalisation 7, Hessian 18, gains 15, c 9);
    iteration 32 (warp 8, bilinear 13, the four sums 11). Wave-uniform scalar
    work (3x3 inverse, SE(2) exponential) is not counted.
    """
    return 2 * levels * PATTERN * (122 + 32 * iters)


def pyramid_bytes(width, height, levels, cams, copy_l0=True):
    """Algorithmic HBM bytes of the pyramid+detector launch: level 0 read once,
    written once into the own pyramid (device push), levels 1..L-1 written."""
    a0 = width * height * cams
    p1 = sum((width >> l) * (height >> l) for l in range(1, levels)) * cams
    return a0 * (2 if copy_l0 else 1) + p1


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed counter profile of this workload,
    or None when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    k = prof.get("kernels", {}).get(kernel)
    if not k or k.get("traffic_bytes") is None:
        return None
    with open(os.path.join(ROOT, "paper_2609_30459_amd", "csrc", k["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != k["source_sha256_16"]:
            return None
    return k["traffic_bytes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 190, batch16 and rig4 100)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="stereo752",
                    help="stereo752, stereo1280, rig4, star752, mono320 or batch16")
    ap.add_argument("--seq", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle CPU-baseline budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", choices=["plain", "graph", "eager"], default="plain",
                    help="first timed region (`value`): the kernels launched one by one without timestamps "
                         "(default; the fewest host calls per pipelined frame), captured graphs, or one by one "
                         "with HIP events attached to each dispatch (gives kernel durations)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="graph launches one frame at a time (no frame submitted before the last one's records are read)")
    ap.add_argument("--no-second-launch", "--no-graph-replay", dest="no_second", action="store_true",
                    help="skip the second timed region, which runs the same steps with the other launch mode")
    ap.add_argument("--init", choices=["const_vel", "learned"], default="const_vel")
    ap.add_argument("--weights", default=None, help="learned-init weights (default: the package's for the workload)")
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
    ap.add_argument("--waves-per-cu", type=int, default=None,
                    help="tracker grid: 0 = one wave per keypoint, N = persistent N waves per CU "
                         "(default: the autotuned choice, else 0)")
    ap.add_argument("--block-waves", type=int, default=None, help="tracker waves per workgroup (1, 2, 4)")
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
        args.steps = 100 if args.workload in ("batch16", "rig4") else 190
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
    n_frames = args.warmup + args.steps
    log(f"rendering {n_frames} frames of {args.workload}: {len(ws)} stream(s), "
        f"{sum(w.n_cams * w.width * w.height for w in ws) / 1e6:.2f} MP per step")
    seqs = [synthgen.sequence(w, seq=args.seq, stream=i, n_frames=n_frames) for i, w in enumerate(ws)]
    devs = [torch.from_numpy(q.frames).cuda() for q in seqs]
    torch.cuda.synchronize()
    streams = [(w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size) for w in ws]

    wpc, bw, tile, smode = args.waves_per_cu, args.block_waves, args.tile, args.stereo_mode
    tuned = None
    if wpc is None and bw is None and tile is None and smode is None:
        from paper_2609_30459_amd import autotune
        tuned = autotune.lookup(args.workload, args.init)
        if tuned:
            wpc, bw = tuned["track_waves_per_cu"], tuned["track_block_waves"]
            tile, smode = tuned.get("pyr_tile", 64), tuned.get("stereo_mode", 0)
    wpc = wpc or 0
    bw = bw or 4
    tile = tile or 64
    smode = smode or 0
    extra = dict(track_waves_per_cu=wpc, track_block_waves=bw, pyr_tile=tile, stereo_mode=smode)
    short_pred = args.motion != "none" and args.pred_levels > 0
    profiled_config = (args.init == "const_vel" and args.motion == "none" and args.preset == "standard" and
                       not args.k_per_cell and not args.levels and not args.iters)
    if short_pred:
        extra.update(pred_levels=args.pred_levels, pred_iters=args.pred_iters,
                     pred_rho=args.pred_rho if args.pred_rho is not None else 3.0e38)
    rho = None
    if args.init == "learned":
        from paper_2609_30459_amd.train_mlp import load_weights
        # the workload's own trained network when there is one, else the stereo1280 one
        wdir = os.path.join(ROOT, "paper_2609_30459_amd", "weights")
        own = os.path.join(wdir, f"mlp_{args.workload}.bin")
        path = args.weights or (own if os.path.exists(own) else os.path.join(wdir, "mlp_stereo1280.bin"))
        mlp_params, rho, meta = load_weights(path)
        log(f"learned init: {path} ({meta}), rho {rho:.4f}")
        extra.update(init_mode=1, learned_levels=args.learned_levels, learned_iters=args.learned_iters,
                     learned_rho=rho)
    ids = list(range(len(ws)))
    # each frame's device images (views into the resident sequences), all
    # cameras stream by stream, made once before any timed region
    frame_imgs = [[devs[i][t, c] for i, w in enumerate(ws) for c in range(w.n_cams)] for t in range(n_frames)]
    # the push/staging call's pointer and pitch arrays, built once per frame
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

    def timed_run(eager):
        """Warmup, then the timed steps: (records per stream, wall s per step, stats per step, elapsed s)."""
        # the streams share one parameter block; per-stream sizes and caps come with the stream
        fe = vf.Frontend(streams, vf.params_for(w0, eager=eager, plain=args.launch == "plain" and not eager, **extra))
        if args.init == "learned":
            fe.set_mlp(mlp_params, rho)
        if motions is not None:
            for i, w in enumerate(ws):
                for c in range(w.n_cams):
                    fe.set_camera_model(i, c, K_of[i])
        records = [[] for _ in ws]
        wall, stats = [], []

        pipelined = not eager and not args.no_pipeline
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

        # pipelined (graph launches): frame t is submitted before frame t-1's
        # records are read, so the host's work overlaps the device's; the
        # latency of a frame runs from its submission to its records
        log(f"warmup {args.warmup} steps ({'eager' if eager else 'graph'}{', pipelined' if pipelined else ''})")
        for t in range(args.warmup):
            submit(t)
            collect(t)
        torch.cuda.synchronize()
        log(f"timing {args.steps} steps")
        # no garbage-collector pause inside the timed steps
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        for t in range(args.warmup, n_frames):
            submit(t)
            if pipelined:
                if t > args.warmup:
                    wall.append(collect(t - 1))
                    stats.append(fe.stats())
            else:
                wall.append(collect(t))
                stats.append(fe.stats())
        if pipelined:
            wall.append(collect(n_frames - 1))
            stats.append(fe.stats())
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        gc.enable()
        fe.close()
        return records, wall, stats, elapsed

    first_eager = args.launch == "eager"
    records, wall, stats, elapsed = timed_run(first_eager)
    steps_per_s = args.steps / elapsed
    fallbacks = [s_["last_fallback"] for s_ in stats]
    second, eager_stats = None, stats if first_eager else None
    if not args.no_second:
        rec2, wall2, stats2, elapsed2 = timed_run(not first_eager)
        same = all(a.tobytes() == b.tobytes() for ra, rb in zip(records, rec2) for a, b in zip(ra, rb))
        second = {"launch": "graph" if first_eager else "eager",
                  "value": args.steps * len(ws) / elapsed2, "ms_per_step": 1000.0 * elapsed2 / args.steps,
                  "gpu_ms_per_step": float(np.mean([s_["last_gpu_ms"] for s_ in stats2])),
                  "latency_p50_ms": float(np.percentile(np.array(wall2) * 1e3, 50)),
                  "latency_p99_ms": float(np.percentile(np.array(wall2) * 1e3, 99)),
                  "records_identical": bool(same)}
        if not first_eager:
            eager_stats = stats2
    # kernel durations from the eager pass (a graph replay gives the frame's device time only);
    # the whole-frame device time from the first timed region
    kstats = eager_stats if eager_stats is not None else stats
    stage_ms = [s_["last_stage_ms"] + s_["last_learned_ms"] + [f_["last_gpu_ms"]] for s_, f_ in zip(kstats, stats)]

    # ---- tracked keypoints and accuracy against the synthetic ground truth ---
    TR, DET, MAT = vf.VIO_TRACKED, vf.VIO_DETECTED, vf.VIO_MATCHED
    tracked = np.zeros(args.steps)
    errs, serrs, n_tr, n_lost = [], [], 0, 0
    n_temporal = np.zeros(args.steps)
    n_stereo = np.zeros(args.steps)
    for i, (w, seq) in enumerate(zip(ws, seqs)):
        rec = records[i]
        for k, t in enumerate(range(args.warmup, n_frames)):
            tracked[k] += int((rec[t]["status"] == TR).sum())
            prev = rec[t - 1] if t > 0 else rec[t][:0]
            n_temporal[k] += int(np.isin(prev["status"], [TR, DET, MAT]).sum())
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

    # ---- roofline of the dominant kernel (HIP events on the launch stream) ----
    # [steps, 6]: pyramid+detector, tracker, selection, features, network, whole frame
    sm = np.array(stage_ms)
    mean_ms = sm.mean(0)
    mean_ms[3] = sm[:, 3].mean() if args.init == "learned" else -1.0
    mean_ms[4] = sm[:, 4].mean() if args.init == "learned" else -1.0
    have_times = bool((sm[:, :3] >= 0).all())
    L, N = w0.levels, w0.gn_iters
    fb = np.array(fallbacks, np.float64)
    if args.init == "learned" or short_pred:
        # every temporal track runs the short tracker; fallbacks rerun the full one
        sl, si = (args.learned_levels, args.learned_iters) if args.init == "learned" else (args.pred_levels,
                                                                                          args.pred_iters)
        flops_step = n_temporal * track_flops_per_call(sl, si) + (fb + n_stereo) * track_flops_per_call(L, N)
    else:
        flops_step = (n_temporal + n_stereo) * track_flops_per_call(L, N)
    pyr_b = sum(pyramid_bytes(w.width, w.height, L, w.n_cams) for w in ws)
    total_rows = sum(w.max_keypoints * w.n_cams for w in ws)
    kernels = {
        "k_pyr_detect": {"bound": "hbm", "avg_ms": float(mean_ms[0]), "bytes_per_launch": pyr_b,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "achieved": pyr_b / (mean_ms[0] * 1e-3) / 1e9 if have_times else None},
        "k_track": {"bound": "alu", "avg_ms": float(mean_ms[1]), "calls_per_launch": float((n_temporal + n_stereo).mean()),
                    "flops_per_launch": float(flops_step.mean()), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "achieved": float(flops_step.mean()) / (mean_ms[1] * 1e-3) / 1e12 if have_times else None,
                    },
        "k_select": {"bound": "latency", "avg_ms": float(mean_ms[2])},
    }
    if args.init == "learned":
        kernels["k_features"] = {"bound": "latency", "avg_ms": float(mean_ms[3])}
        kernels["k_mlp_fwd"] = {"bound": "mfma", "avg_ms": float(mean_ms[4]),
                                "flops_per_launch": 2 * (32 * 128 + 128 * 128 + 128 * 3) * total_rows}
    roof = None
    if have_times:
        dom = ["k_pyr_detect", "k_track", "k_select"][int(np.argmax(mean_ms[:2]))]
        kd = kernels[dom]
        roof = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                "unit": kd["unit"], "frac": kd["achieved"] / kd["peak"],
                # counters were taken on the default configuration only
                "traffic": measured_traffic(args.workload, dom) if profiled_config else None,
                "avg_ms": kd["avg_ms"]}

    # ---- CPU baseline: the oracle on a bounded sample of the same workload ---
    cpu = None
    if not args.no_cpu_baseline and args.init == "const_vel":
        import oracle
        nproc = os.cpu_count() or 1
        model = cpu_model_name()
        unit = "stream-frames/s" if batched else "frames/s"

        def new_oracles():
            return [oracle.Frontend([w.width] * w.n_cams, [w.height] * w.n_cams, w.stereo, oracle.params_for(w))
                    for w in ws]

        # (i) one thread, stream after stream, frame by frame
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
               "sample": f"first {n} frames of the same {args.workload} sequence(s), single-threaded C++ oracle "
                         f"(-O2), {cpu_s:.1f} s", "nproc": nproc, "cpu_model": model}
        if batched:
            # (ii) one thread per stream (the oracle's calls release the GIL), the same frames
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

    wall_ms = np.array(wall) * 1e3
    value = steps_per_s * len(ws)
    out = {
        "metric": "stereo frames/s + tracked kpts/s, plain vs learned-init KLT at <=0.1px err",
        "value": value,
        "unit": "stream-frames/s" if batched else "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 / steps_per_s,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "streams": len(ws),
                   "cameras": sum(w.n_cams for w in ws),
                   "sizes": sorted({f"{w.width}x{w.height}x{w.n_cams}" for w in ws}),
                   "levels": L, "gn_iters": N, "max_keypoints": sorted({w.max_keypoints for w in ws}),
                   "preset": args.preset, "k_per_cell": w0.k_per_cell,
                   "motion": args.motion, **({"motion_noise_px": args.motion_noise, "focal": args.focal,
                                              "camera": args.camera} if args.motion != "none" else {}),
                   **({"pred_levels": args.pred_levels, "pred_iters": args.pred_iters, "pred_rho": args.pred_rho}
                      if short_pred else {}),
                   "cell_size": sorted({w.cell_size for w in ws}), "thresholds": list(w0.thresholds),
                   "init": args.init, "launch": args.launch,
                   "pipelined": args.launch != "eager" and not args.no_pipeline, "track_waves_per_cu": wpc, "track_block_waves": bw, "pyr_tile": tile,
                   "stereo_mode": ["speculative", "deferred"][smode],
                   "autotuned": tuned is not None, "parallelism": "single_gpu",
                   **({"learned_levels": args.learned_levels, "learned_iters": args.learned_iters, "rho": rho}
                      if args.init == "learned" else {})},
        "tracked_kpts_per_s": float(tracked.mean()) * steps_per_s,
        "gpu_ms_per_step": float(mean_ms[5]),
        "latency_ms": {"p50": float(np.percentile(wall_ms, 50)), "p99": float(np.percentile(wall_ms, 99)),
                       "gpu_p50": float(np.percentile(sm[:, 5], 50)), "gpu_p99": float(np.percentile(sm[:, 5], 99))},
        "accuracy": {"temporal_median_px": float(np.median(err)), "temporal_p90_px": float(np.percentile(err, 90)),
                     "stereo_median_px": float(np.median(serr)), "survival": survival},
        "fallback_per_step": float(fb.mean()) if args.init == "learned" or short_pred else None,
        "roofline": roof,
        "second_launch": second,
        "kernels": kernels,
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
