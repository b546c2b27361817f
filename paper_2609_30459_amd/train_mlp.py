"""Trains the learned-initialisation network on tracks of the plain tracker.

Data: seeded training sequences (disjoint seeds from the evaluation ones) of a
stereo workload are run through the GPU frontend with the plain tracker; for
every keypoint kept by temporal tracking, its network inputs at frame t-1
(computed by the frontend's own feature kernel) are paired with the plain
tracker's displacement to frame t. Adam with a cosine learning-rate decay.

The fallback threshold rho is then calibrated on the short tracker itself: the
trained network drives the learned frontend (with no residual fallback) over
the training sequences again, and rho is a high percentile of the residual RMS
of its kept tracks, so that only the tail of the short tracker's own
distribution -- where it settled in a wrong basin -- falls back.

Training runs on the GPU with the library's BF16-MFMA forward/backward and
Adam kernels (vio_mlp.h); nothing here computes the network.

    python -m paper_2609_30459_amd.train_mlp --out weights.bin
"""
from __future__ import annotations

import argparse
import os
import struct
import sys
import time

import numpy as np

MAGIC = b"VIOMLP01"


def save_weights(path, params, rho, meta=""):
    params = np.ascontiguousarray(params, np.float32)
    meta_b = meta.encode()
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<ifI", len(params), float(rho), len(meta_b)))
        f.write(meta_b)
        f.write(params.tobytes())


def load_weights(path):
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a weights file")
        n, rho, lm = struct.unpack("<ifI", f.read(12))
        meta = f.read(lm).decode()
        params = np.frombuffer(f.read(4 * n), np.float32).copy()
    if len(params) != n:
        raise ValueError(f"{path}: truncated")
    return params, rho, meta


def collect(workload, n_seq=20, n_frames=6, max_samples=50000, log=print):
    """(X [S,32], T [S,2], resid [R]) from the plain tracker on training seeds."""
    import paper_2609_30459_amd as vf
    import synthgen
    from synthgen.workloads import train_seed

    w = workload
    X, T, R = [], [], []
    zero = np.zeros(vf.MLP_NPARAM, np.float32)
    for s in range(n_seq):
        seq = synthgen.sequence(w, n_frames=n_frames, seed=train_seed(s))
        params = vf.params_for(w, init_mode=1, learned_levels=min(2, w.levels), learned_iters=3, learned_rho=-1.0)
        stream = (w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size)
        with vf.Frontend([stream], params) as fe:
            fe.set_mlp(zero, rho=-1.0)  # rho < 0: every track is the plain tracker's
            prev = None
            for t in range(n_frames):
                fe.push_stereo_frame(0, t + 1, list(seq.frames[t]))
                recs = fe.get_tracks(0)
                if t > 0:
                    for c in range(w.n_cams):
                        feats = fe.get_features(0, c)
                        rc = recs[recs["camera"] == c][: len(feats)]
                        kp = prev[c]
                        assert len(kp) == len(feats) and (rc["id"] == kp["id"]).all()
                        ok = rc["status"] == vf.VIO_TRACKED
                        X.append(feats[ok])
                        T.append(np.stack([rc["x"][ok] - kp["x"][ok], rc["y"][ok] - kp["y"][ok]], 1))
                        R.append(rc["resid_rms"][ok])
                prev = [fe.get_keypoints(0, c) for c in range(w.n_cams)]
        log(f"  sequence {s}: {sum(len(x) for x in X)} samples")
    X = np.concatenate(X).astype(np.float32)
    T = np.concatenate(T).astype(np.float32)
    R = np.concatenate(R).astype(np.float32)
    if len(X) > max_samples:
        idx = np.random.default_rng(0).choice(len(X), max_samples, replace=False)
        idx.sort()
        X, T = X[idx], T[idx]
    return X, T, R


def train(X, T, epochs=60, batch=1024, lr=1e-3, lr_end=1e-5, seed=0, log=print):
    """Adam on the GPU with a cosine decay from lr to lr_end; returns (params, per-epoch mean losses)."""
    import math

    import torch

    import paper_2609_30459_amd as vf

    rng = np.random.default_rng(seed)
    params0 = _init_params(seed)
    dx = torch.from_numpy(X).cuda()
    dt = torch.from_numpy(T).cuda()
    n = len(X)
    losses = []
    with vf.Mlp(batch) as net:
        net.set_params(params0)
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).cuda()
            xs, ts = dx[perm].contiguous(), dt[perm].contiguous()
            tot, nb = 0.0, 0
            lr_ep = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * ep / max(1, epochs - 1)))
            for b0 in range(0, n - batch + 1, batch):
                loss = net.train_step(xs[b0:b0 + batch], ts[b0:b0 + batch], lr=lr_ep, want_loss=True)
                tot += loss
                nb += 1
            losses.append(tot / max(1, nb))
            log(f"  epoch {ep}: loss {losses[-1]:.4f}")
        params = net.get_params()
    return params, losses


def calibrate_rho(params, workload, n_seq=20, n_frames=6, percentile=99.5, learned_levels=2, learned_iters=3):
    """rho: the percentile of the short tracker's residual RMS over its kept tracks (training seeds)."""
    import paper_2609_30459_amd as vf
    import synthgen
    from synthgen.workloads import train_seed

    w = workload
    R = []
    for s in range(n_seq):
        seq = synthgen.sequence(w, n_frames=n_frames, seed=train_seed(s))
        p = vf.params_for(w, init_mode=1, learned_levels=learned_levels, learned_iters=learned_iters,
                          learned_rho=1e9)
        with vf.Frontend([(w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size)], p) as fe:
            fe.set_mlp(params, rho=1e9)
            for t in range(n_frames):
                fe.push_stereo_frame(0, t + 1, list(seq.frames[t]))
                rec = fe.get_tracks(0)
                if t > 0:
                    R.append(rec["resid_rms"][rec["status"] == vf.VIO_TRACKED])
    return float(np.percentile(np.concatenate(R), percentile))


def _init_params(seed):
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    P = np.zeros(21123, np.float32)
    o = 0
    for fan_out, fan_in in ((128, 32), (128, 128), (3, 128)):
        lim = np.sqrt(6.0 / fan_in)
        P[o:o + fan_out * fan_in] = rng.uniform(-lim, lim, fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    return P


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="stereo1280")
    ap.add_argument("--sequences", type=int, default=20)
    ap.add_argument("--frames", type=int, default=6)
    ap.add_argument("--samples", type=int, default=50000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--rho-percentile", type=float, default=99.5)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synthgen

    def log(m):
        print(m, file=sys.stderr, flush=True)

    w = synthgen.WORKLOADS[args.workload]
    t0 = time.time()
    log(f"collecting plain-tracker samples from {args.sequences} training sequences of {w.name}")
    X, T, R = collect(w, args.sequences, args.frames, args.samples, log)
    log(f"{len(X)} samples, plain-tracker residual {args.rho_percentile}th percentile "
        f"{np.percentile(R, args.rho_percentile):.4f}, {time.time() - t0:.1f} s")
    params, losses = train(X, T, epochs=args.epochs, log=log)
    rho = calibrate_rho(params, w, args.sequences, args.frames, args.rho_percentile)
    log(f"rho = {rho:.4f} ({args.rho_percentile}th percentile of the short tracker's residuals)")
    save_weights(args.out, params, rho, meta=f"{w.name} samples={len(X)} epochs={args.epochs} "
                                            f"final_loss={losses[-1]:.5f}")
    log(f"saved {args.out} (loss {losses[0]:.4f} -> {losses[-1]:.4f}, {time.time() - t0:.1f} s)")


if __name__ == "__main__":
    main()
