"""Picks the kernels' launch shapes per workload and device by measurement.

Four choices are free and leave the records bit for bit the same:
  * the tracker's launch shape: one wave64 per work item in workgroups of 1, 2
    or 4 waves, or a persistent grid of 1..16 waves per compute unit popping
    items from a shared queue;
  * keypoints per tracking wavefront: one (a lane per pattern point) or two
    (one per 32-lane half, two pattern points per lane);
  * the pyramid/detector tile: 64x64 level-0 pixels per 1024-thread workgroup
    or 32x32 per 256-thread workgroup (more, smaller workgroups, at the cost
    of a larger share of recomputed apron);
  * the stereo mode: match every cell winner speculatively in the tracking
    launch (fewest dependent launches) or only the selected detections after
    selection (least work).
Which is fastest depends on the image sizes, the item count, the levels and
iterations, and the chip. The tracker grid is chosen first, on the same frames
of the workload with the kernels launched one by one and HIP events attached
to their dispatches, by the tracker kernel's mean duration (one keypoint per
wave over all grids, then two per wave with the best grid and with one launch
per item). Then, with that grid, the tile, the stereo mode and keypoints per
wave are decided together in the production setting -- the benchmark's
pipelined loop, three frames in flight, the next frames' pyramids running
beside this frame's tracking, one process per candidate -- by its time per
step: kernels alone on the chip and kernels sharing it favour different
choices (two keypoints per wave are faster alone on batch16, and slower in
the benchmark's loop). The winners go into a JSON cache keyed by the device's
architecture and compute-unit count, which the benchmark reads.

    python -m paper_2609_30459_amd.autotune --workload batch16 --init const_vel
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned", "launch.json")

# tracker shapes (waves_per_cu, block_waves); waves_per_cu 0 = one wave per item
SHAPES = [(0, 1), (0, 2), (0, 4), (1, 4), (2, 4), (4, 4), (8, 4), (16, 4), (2, 1), (4, 2), (8, 2)]


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{p.gcnArchName.split(':')[0]}_{p.multi_processor_count}cu"


def _load_cache(path=CACHE):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(workload: str, init: str, path=CACHE):
    """The cached choice for this device, workload and init mode, or None."""
    entry = _load_cache(path).get(device_key(), {}).get(f"{workload}:{init}")
    return entry


def _workloads(name):
    import synthgen
    from synthgen.workloads import BATCH16
    return list(BATCH16) if name == "batch16" else [synthgen.WORKLOADS[name]]


def measure(workload: str, init: str, shapes, frames=40, warmup=8, weights=None, learned_levels=2,
            learned_iters=3, log=print):
    """Mean pyramid, tracker, all-kernel and frame device times (ms) of each
    (waves_per_cu, block_waves, tile, stereo_mode, kp_per_wave) candidate."""
    import torch

    import paper_2609_30459_amd as vf
    import synthgen
    from paper_2609_30459_amd.train_mlp import load_weights

    ws = _workloads(workload)
    n = warmup + frames
    seqs = [synthgen.sequence(w, seq=0, stream=i, n_frames=n) for i, w in enumerate(ws)]
    devs = [torch.from_numpy(q.frames).cuda() for q in seqs]
    streams = [(w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size) for w in ws]
    extra = {}
    if init == "learned":
        params, rho, _ = load_weights(weights or os.path.join(HERE, "weights", "mlp_stereo1280.bin"))
        extra = dict(init_mode=1, learned_levels=learned_levels, learned_iters=learned_iters, learned_rho=rho)
    ids = list(range(len(ws)))
    out = []
    for wpc, bw, tile, smode, kpw in shapes:
        p = vf.params_for(ws[0], eager=True, track_waves_per_cu=wpc, track_block_waves=bw, pyr_tile=tile,
                          stereo_mode=smode, track_kp_per_wave=kpw, **extra)
        pyr, track, total, frame = [], [], [], []
        with vf.Frontend(streams, p) as fe:
            if init == "learned":
                fe.set_mlp(params, rho)
            for t in range(n):
                imgs = [devs[i][t, c] for i, w in enumerate(ws) for c in range(w.n_cams)]
                fe.stage_frames_device(ids, [t + 1] * len(ws), imgs)
                fe.step()
                if t >= warmup:
                    st = fe.stats()
                    pyr.append(st["last_stage_ms"][0])
                    track.append(st["last_stage_ms"][1])
                    total.append(sum(st["last_stage_ms"]) + sum(max(0.0, m) for m in st["last_learned_ms"]))
                    frame.append(st["last_gpu_ms"])
        r = {"track_waves_per_cu": wpc, "track_block_waves": bw, "pyr_tile": tile, "stereo_mode": smode,
             "track_kp_per_wave": kpw, "pyr_ms": float(np.mean(pyr)), "track_ms": float(np.mean(track)), "kernels_ms": float(np.mean(total)),
             "frame_ms": float(np.mean(frame))}
        log(f"  waves/CU {wpc:2d}  waves/block {bw}  keypoints/wave {kpw}  tile {tile}  stereo {smode}: "
            f"pyramid {r['pyr_ms'] * 1e3:7.1f} "
            f"us, tracker {r['track_ms'] * 1e3:7.1f} us, kernels {r['kernels_ms'] * 1e3:7.1f} us, frame "
            f"{r['frame_ms'] * 1e3:7.1f} us")
        out.append(r)
    return out


def bench_steps(workload: str) -> int:
    """The benchmark's default timed steps for the workload."""
    return 80 if workload in ("batch16", "rig4") else 150


def pipelined_ms(workload: str, init: str, shape, extra=(), **_):
    """Time per step (ms) of the benchmark's pipelined production loop (bench.py at the repository
    root: plain launches, three frames in flight, records read every frame, its own frames), in a
    process of its own, with shape = (waves_per_cu, block_waves, tile, stereo_mode, kp_per_wave).
    Measured in one long-lived process one after another, the choices ranked differently from the
    benchmark's fresh process per run; the benchmark's ranking is the one that counts."""
    import subprocess
    wpc, bw, tile, smode, kpw = shape
    root = os.path.dirname(HERE)
    cmd = [sys.executable, os.path.join(root, "bench.py"), "--workload", workload, "--init", init,
           "--no-cpu-baseline", "--no-host-leg", "--no-second-launch", "--waves-per-cu", str(wpc),
           "--block-waves", str(bw), "--tile", str(tile), "--stereo-mode", str(smode), "--kp-per-wave", str(kpw)]
    cmd += list(extra)
    out = subprocess.run(cmd, cwd=root, check=True, capture_output=True, text=True).stdout
    return float(json.loads(out.strip().splitlines()[-1])["ms_per_step"])


def tune(workload: str, init: str, frames=40, path=CACHE, log=print, **kw):
    """Measures every candidate, stores the fastest in the cache and returns it."""
    t0 = time.time()
    res = measure(workload, init, [(w, b, 64, 0, 1) for w, b in SHAPES], frames=frames, log=log, **kw)
    best = min(res, key=lambda r: r["track_ms"])
    wpc, bw = best["track_waves_per_cu"], best["track_block_waves"]
    # keypoints per wavefront: two per wave with the best grid, and with the
    # one-launch-per-item grid
    res += measure(workload, init, sorted({(wpc, bw, 64, 0, 2), (0, 4, 64, 0, 2)}), frames=frames, log=log, **kw)
    best = min(res, key=lambda r: r["track_ms"])
    wpc, bw = best["track_waves_per_cu"], best["track_block_waves"]
    cache = _load_cache(path)
    old = cache.get(device_key(), {}).get(f"{workload}:{init}", {})
    # the final pick in the pipelined production loop, over tile, stereo mode
    # and keypoints per wave with the chosen grid; a learned stage fused into
    # the tracker (a choice kept from the benchmark sweeps) runs one keypoint
    # per wave
    kps = (1,) if init == "learned" and old.get("learned_fused") else (1, 2)
    extra = []
    if init == "learned":  # the learned stage's own choices, as the benchmark runs them
        extra = ["--learned-fused", str(old.get("learned_fused", 0))]
        if "track_parallel_fallback" in old:
            extra += ["--parallel-fallback", str(old["track_parallel_fallback"])]
    # two passes over the choices, each keeping its faster pass (a pass now
    # and then catches a slow moment of the machine)
    piped = {}
    for _ in range(2):
        for t in (32, 64):
            for sm in (0, 1):
                for k in kps:
                    ms = pipelined_ms(workload, init, (wpc, bw, t, sm, k), extra)
                    piped[(t, sm, k)] = min(ms, piped.get((t, sm, k), ms))
                    log(f"  pipelined: tile {t}  stereo {sm}  keypoints/wave {k}: {ms * 1e3:7.1f} us/frame")
    tile, smode, kpw = min(piped, key=piped.get)
    entry = {"track_waves_per_cu": wpc, "track_block_waves": bw, "track_kp_per_wave": kpw, "pyr_tile": tile,
             "stereo_mode": smode, "track_ms": best["track_ms"], "pipelined_ms": piped[(tile, smode, kpw)],
             "pipelined": [{"pyr_tile": t, "stereo_mode": sm, "track_kp_per_wave": k, "ms": v}
                           for (t, sm, k), v in piped.items()],
             "frames": frames, "candidates": res}
    # the learned stage's choices (its own launch or fused into the tracker,
    # parallel fallbacks, keypoints per workgroup) are set from pipelined
    # benchmark sweeps, not by this kernel-time tuner: kept across re-tuning
    for k in ("learned_fused", "track_parallel_fallback", "learned_block_waves"):
        if k in old:
            entry[k] = old[k]
    cache.setdefault(device_key(), {})[f"{workload}:{init}"] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path + ".tmp", "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(path + ".tmp", path)
    log(f"{workload}:{init} -> waves/CU {wpc}, waves/block {bw}, keypoints/wave {kpw}, tile {tile}, "
        f"stereo mode {entry['stereo_mode']} "
        f"({time.time() - t0:.1f} s)")
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", action="append", help="repeatable; default stereo752, stereo1280, batch16")
    ap.add_argument("--init", choices=["const_vel", "learned", "both"], default="both")
    ap.add_argument("--frames", type=int, default=40)
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))

    def log(m):
        print(m, file=sys.stderr, flush=True)

    inits = ["const_vel", "learned"] if args.init == "both" else [args.init]
    for wl in args.workload or ["stereo752", "stereo1280", "batch16"]:
        for init in inits:
            log(f"tuning {wl} ({init})")
            tune(wl, init, frames=args.frames, path=args.cache, log=log)


if __name__ == "__main__":
    main()
