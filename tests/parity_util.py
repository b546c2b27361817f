"""Helpers that run the oracle and the GPU library side by side and compare them."""
from __future__ import annotations

import numpy as np

import oracle

TOL_PX = 1e-3      # track positions, FP32 (the workloads' stated bound)
# patch rotation, radians: a rotation error d moves the pattern's outermost
# point (radius sqrt(3.5^2 + 1.5^2) = 3.81 px) by 3.81 d, held to TOL_PX
TOL_THETA = TOL_PX / 3.81
MARGIN = 1e-3      # decisions closer than this to their threshold are reported, not failed
# A track outside the tolerance may go to the FP64 referee only when its
# Gauss-Newton system is near singular: the ratio of the smallest to the
# largest eigenvalue of H at the level-0 template of either pass, with the
# rotation measured as the displacement it causes at the pattern's RMS radius
# (so all three parameters are in pixels; 1 for an isotropic corner, about
# 0.06-0.1 for the median corner of the synthetic workloads), below
# RATIO_BOUND. Along that weak direction the FP32 summation order moves the
# fixed point by more than the tolerance on both FP32 sides.
RATIO_BOUND = 1e-2
# Referrals allowed per run: with one keypoint per cell (every track a cell's
# strongest corner) at most one, and only for a corner whose rotation is all
# but unobservable (ratio below RATIO_BOUND_K1: a strong FAST corner can still
# be nearly symmetric under rotation -- rig4's keypoint 2823 has 2.8e-4 at its
# level-0 target template); with k > 1 per cell, where the weaker corners of a
# cell are tracked too, at most this fraction of the compared tracks.
RATIO_BOUND_K1 = 1e-3
REFER_CAP = 0.005
# Both sides lost a track and only the reason differs (a diverged backward
# pass): the tracked/lost set is the same; at most this fraction per run.
DIVERGED_CAP = 0.005

# every run's tally, printed at the end of the pytest session (tests/conftest.py)
SESSION_TALLIES = []


class Tally:
    """Counts of one parity run: compared tracks and every excuse taken."""

    def __init__(self, where, register=True):
        self.where = where
        self.compared = 0      # tracked or matched records with equal status, positions compared
        self.margin = []       # status differs, forward-backward distance within MARGIN of the threshold
        self.diverged = []     # both lost, reasons differ (backward pass diverged)
        self.referred = []     # outside the tolerance, decided by the FP64 referee
        if register:
            SESSION_TALLIES.append(self)

    def line(self):
        worst = max((r[2] for r in self.referred), default=None)
        return (f"{self.where}: compared {self.compared}, margin {len(self.margin)}, diverged {len(self.diverged)}, "
                f"referred {len(self.referred)}" +
                (f" (weakest-direction ratios up to {worst:.2e})" if worst is not None else ""))

    def check(self, k_per_cell):
        """The run's excuses against the caps."""
        assert len(self.margin) <= 1, f"{self.line()}: {self.margin}"
        assert len(self.diverged) <= max(1, DIVERGED_CAP * self.compared), f"{self.line()}: {self.diverged[:5]}"
        if k_per_cell == 1:
            assert len(self.referred) <= 1 and all(r[2] < RATIO_BOUND_K1 for r in self.referred), \
                f"{self.line()}: {self.referred[:5]}"
        else:
            assert len(self.referred) <= REFER_CAP * self.compared, f"{self.line()}: {self.referred[:5]}"


def _pattern_rms_radius():
    u, v = oracle.pattern()
    return float(np.sqrt(np.mean(u.astype(np.float64) ** 2 + v.astype(np.float64) ** 2)))


def weak_ratio(img, x, y):
    """lambda_min / lambda_max of the level-0 template's Gauss-Newton matrix at
    (x, y), rotation scaled to pixels at the pattern's RMS radius; 0 when the
    template does not fit."""
    H, _, fits, _ = oracle.template(img, float(x), float(y))
    if not fits:
        return 0.0
    D = np.diag([1.0, 1.0, 1.0 / _pattern_rms_radius()])
    ev = np.linalg.eigvalsh(D @ H @ D)
    return float(ev[0] / ev[-1]) if ev[-1] > 0 else 0.0


def oracle_state(fe_orc, cam):
    """The oracle's live keypoints of camera `cam` as vio_keypoint records."""
    from paper_2609_30459_amd import KEYPOINT_DTYPE
    ids, xy, pxy, age = fe_orc.keypoints(cam)
    out = np.zeros(len(ids), KEYPOINT_DTYPE)
    out["id"], out["x"], out["y"] = ids, xy[:, 0], xy[:, 1]
    out["px"], out["py"], out["age"] = pxy[:, 0], pxy[:, 1], age
    return out


def inject(fe_gpu, fe_orc, stream, n_cams):
    for c in range(n_cams):
        fe_gpu.set_keypoints(stream, c, oracle_state(fe_orc, c))


def compare_records(gpu, orc, fb_threshold, where="", referee=None, tally=None):
    """Element-by-element comparison; returns the list of excused margin cases.

    Identifiers, cameras and statuses must agree, tracked and matched positions
    lie within TOL_PX (rotations within TOL_THETA), detections agree exactly.
    Every excuse is counted in `tally` (a Tally, whose caps the caller checks
    after the run; without one, this call's excuses are checked against them):

    * a status disagreement where the forward-backward distance of either side
      lies within MARGIN of the threshold (an FP32 tie the two summation orders
      may break differently; also returned to the caller);
    * both sides lost the track and only the reason differs because the
      backward pass diverged (one left the image, the other returned more than
      1 px away);
    * a position outside the tolerance on a near-singular Gauss-Newton system
      (eigenvalue ratio below RATIO_BOUND), where the GPU is no further from
      the FP64 track than the FP32 oracle is, plus the tolerance.
      referee(indices) returns the FP64 (x, y, theta, fb) and the eigenvalue
      ratio of the given records.
    """
    one_off = tally is None
    tally = Tally(where, register=False) if one_off else tally
    assert len(gpu) == len(orc), f"{where}: {len(gpu)} GPU records vs {len(orc)} oracle records"
    assert (gpu["camera"] == orc["camera"]).all(), where
    assert (gpu["id"] == orc["id"]).all(), where
    excused = []
    bad = []
    for i in np.nonzero(gpu["status"] != orc["status"])[0]:
        sg, so = int(gpu["status"][i]), int(orc["status"][i])
        near = (abs(gpu["fb_err"][i] - fb_threshold) < MARGIN or abs(orc["fb_err"][i] - fb_threshold) < MARGIN)
        diverged = ({sg, so} == {oracle.LOST_FB, oracle.LOST_OOB} and
                    max(gpu["fb_err"][i], orc["fb_err"][i]) > 1.0)
        if {sg, so} <= {oracle.TRACKED, oracle.LOST_FB, oracle.MATCHED} and near:
            excused.append((int(gpu["id"][i]), sg, so, float(orc["fb_err"][i])))
            tally.margin.append((where,) + excused[-1])
        elif diverged:
            tally.diverged.append((where, int(gpu["id"][i]), sg, so, float(gpu["fb_err"][i]), float(orc["fb_err"][i])))
        else:
            bad.append((int(gpu["camera"][i]), int(gpu["id"][i]), sg, so, float(gpu["fb_err"][i]),
                        float(orc["fb_err"][i]), float(gpu["x"][i]), float(orc["x"][i]), float(gpu["y"][i]),
                        float(orc["y"][i])))
    assert not bad, f"{where}: status mismatches (cam, id, gpu, oracle, fb_g, fb_o, xg, xo, yg, yo): {bad[:10]}"
    same = gpu["status"] == orc["status"]
    pos = same & np.isin(orc["status"], [oracle.TRACKED, oracle.MATCHED])
    tally.compared += int(pos.sum())
    if pos.any():
        fields, tols = ("x", "y", "theta", "fb_err"), np.array([TOL_PX, TOL_PX, TOL_THETA, TOL_PX])
        d = np.stack([np.abs(gpu[f][pos].astype(np.float64) - orc[f][pos]) for f in fields], 1)
        off = np.nonzero(pos)[0][(d > tols).any(1)]
        if len(off):
            worst = off[int(np.argmax((d[(d > tols).any(1)] / tols).max(1)))]
            msg = (f"{where}: id {int(gpu['id'][worst])} differs by "
                   f"{[float(abs(gpu[f][worst] - orc[f][worst])) for f in fields]} (x, y, theta, fb)")
            assert referee is not None, msg
            ref = referee(off)
            eg = np.stack([np.abs(gpu[f][off].astype(np.float64) - ref[:, j]) for j, f in enumerate(fields)], 1)
            eo = np.stack([np.abs(orc[f][off].astype(np.float64) - ref[:, j]) for j, f in enumerate(fields)], 1)
            bad_ref = (eg > eo + tols).any(1)
            assert not bad_ref.any(), \
                f"{msg}; against FP64 the GPU is off by {eg[bad_ref][0].tolist()}, the oracle by {eo[bad_ref][0].tolist()}"
            well = ref[:, 4] >= RATIO_BOUND
            assert not well.any(), (f"{msg}; {int(well.sum())} of them well conditioned (eigenvalue ratio "
                                    f"{ref[well, 4].min():.3g} >= {RATIO_BOUND}), not referable")
            for n, i in enumerate(off):
                tally.referred.append((where, int(gpu["id"][i]), float(ref[n, 4]),
                                       float(max(abs(gpu["x"][i] - orc["x"][i]), abs(gpu["y"][i] - orc["y"][i])))))
    det = orc["status"] == oracle.DETECTED
    assert (gpu["x"][det] == orc["x"][det]).all() and (gpu["y"][det] == orc["y"][det]).all(), where
    assert (gpu["score"][det] == orc["score"][det]).all(), where
    if one_off:
        tally.check(1)
    return excused


def _track_fp64(frames, t, orc, prev, idx, L, N, fb, d0, motion=None, short=None):
    """FP64 (x, y, theta, fb, eigenvalue ratio) of the tracked/matched records `idx` of frame t: temporal
    tracks from the previous state with the constant-velocity start (or the
    camera-model start where motion[camera] = (K, R, t, rho, {id: rho}) is
    given), stereo matches from the same frame's detection in the detecting
    camera (with the extrinsics start where motion[("ext", camera)] =
    (Ks, Kt, R, t, rho) is given). short = (levels, iters, rho): a track with
    a camera-model start first runs that budget and keeps it when tracked with
    a residual RMS <= rho, else the full budget from the same start."""
    out = np.zeros((len(idx), 5))
    for n, i in enumerate(idx):
        c, kid = int(orc["camera"][i]), int(orc["id"][i])
        if orc["status"][i] == oracle.TRACKED:
            kp = prev[c][prev[c]["id"] == kid][0]
            src, dst = frames[t - 1][c], frames[t][c]
            pt, init = (kp["x"], kp["y"]), (2.0 * kp["x"] - kp["px"], 2.0 * kp["y"] - kp["py"])
            th0 = 0.0
            predicted = False
            if motion and c in motion:
                K, R, tr, rho, own = motion[c]
                st, ok = oracle.motion_start(K, R, tr, np.array([pt], np.float64), own.get(kid, rho))
                if ok[0]:
                    init, th0 = (st[0, 0], st[0, 1]), st[0, 2]
                    predicted = True
        else:
            th0 = 0.0
            # the keypoint's detection, in the camera whose matches this one receives
            det = orc[(orc["id"] == kid) & (orc["status"] == oracle.DETECTED)][0]
            src, dst = frames[t][int(det["camera"])], frames[t][c]
            pt, init = (det["x"], det["y"]), (det["x"] - d0, det["y"])
            if motion and ("ext", c) in motion:
                Ks, Kt, R, tr, rho = motion[("ext", c)]
                st, ok = oracle.motion_start(Ks, R, tr, np.array([pt], np.float64), rho, Kq=Kt)
                if ok[0]:
                    init, th0 = (st[0, 0], st[0, 1]), st[0, 2]
        r = None
        if short is not None and orc["status"][i] == oracle.TRACKED and predicted:
            rs, st = oracle.track(src, dst, np.array([pt], np.float64), np.array([init], np.float64), short[0],
                                  short[1], fb, double=True, theta0=th0)
            if st[0] == oracle.TRACKED and rs[0, 4] <= short[2]:
                r = rs
        if r is None:
            r, _ = oracle.track(src, dst, np.array([pt], np.float64), np.array([init], np.float64), L, N, fb,
                                double=True, theta0=th0)
        out[n, :4] = r[0, :4]
        # the weaker of the two passes' level-0 systems: the forward template on
        # the source at p, the backward one on the target at p'
        out[n, 4] = min(weak_ratio(src, *pt), weak_ratio(dst, orc["x"][i], orc["y"][i]))
    return out


def run_pair(workload, seq, n_frames, inject_state=True, params_overrides=None, stream_overrides=None,
             push_device=False, launch=None, before_push=None):
    """Runs the oracle and the GPU frontend over the first n_frames of `seq`.

    params_overrides apply to both sides; launch: GPU-only launch parameters
    (tiles, tracker shape, stereo mode), which must not change the records;
    before_push(t, fe_gpu, fe_oracle) runs before each frame's push and
    returns the camera motions it set ({camera: (K, R, t, rho, {id: rho})}) or
    None.
    Yields (t, gpu_records, oracle_records, excused) per frame.
    """
    import paper_2609_30459_amd as vf
    po = params_overrides or {}
    fe_o = oracle.Frontend([workload.width] * workload.n_cams, [workload.height] * workload.n_cams,
                           workload.stereo, oracle.params_for(workload, **po))
    stream = (workload.n_cams, workload.width, workload.height, workload.max_keypoints, workload.cell_size)
    if stream_overrides:
        stream = stream_overrides
    fe_g = vf.Frontend([stream], vf.params_for(workload, **po, **(launch or {})))
    dev = None
    if push_device:
        import torch
        dev = torch.from_numpy(seq.frames[:n_frames]).cuda()
    L, N = po.get("levels", workload.levels), po.get("gn_iters", workload.gn_iters)
    fb, d0 = po.get("fb_threshold", workload.fb_threshold), po.get("disparity0", workload.disparity0)
    k = po.get("k_per_cell", workload.k_per_cell)
    tally = Tally(f"{workload.name} k={k} {n_frames} frames" + (f" {po}" if po else "") +
                  (f" {launch}" if launch else ""))
    try:
        for t in range(n_frames):
            if inject_state and t > 0:
                inject(fe_g, fe_o, 0, workload.n_cams)
            prev = [oracle_state(fe_o, c) for c in range(workload.n_cams)]
            motion = before_push(t, fe_g, fe_o) if before_push else None
            fe_o.push(list(seq.frames[t]))
            if push_device:
                fe_g.push_stereo_frame_device(0, t + 1, [dev[t, c] for c in range(workload.n_cams)])
            else:
                fe_g.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            g, o = fe_g.get_tracks(0), fe_o.records()

            short = ((po["pred_levels"], po.get("pred_iters", N), po.get("pred_rho", 0.0))
                     if po.get("pred_levels", 0) > 0 else None)

            def referee(idx, t=t, o=o, prev=prev, motion=motion, short=short):
                return _track_fp64(seq.frames, t, o, prev, idx, L, N, fb, d0, motion, short)

            # the FP64 referee rebuilds constant-velocity and camera-model starts
            # and the short budget of camera-model starts (not the learned
            # guess, nor the neighbour stereo start)
            learned = po.get("init_mode", 0) != 0 or po.get("stereo_init", 0) != 0
            exc = compare_records(g, o, workload.fb_threshold, where=f"{workload.name} frame {t}",
                                  referee=None if learned else referee, tally=tally)
            yield t, g, o, exc, fe_g, fe_o
        print(tally.line(), flush=True)
        tally.check(k)
    finally:
        fe_g.close()
        fe_o.close()
