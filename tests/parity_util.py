"""Helpers that run the oracle and the GPU library side by side and compare them."""
from __future__ import annotations

import numpy as np

import oracle

TOL_PX = 1e-3      # track positions, FP32 (the workloads' stated bound)
# patch rotation, radians: a rotation error d moves the pattern's outermost
# point (radius sqrt(3.5^2 + 1.5^2) = 3.81 px) by 3.81 d, held to TOL_PX
TOL_THETA = TOL_PX / 3.81
MARGIN = 1e-3      # decisions closer than this to their threshold are reported, not failed


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


def compare_records(gpu, orc, fb_threshold, where="", referee=None):
    """Element-by-element comparison; returns the list of excused margin cases.

    Identifiers, cameras and statuses must agree, tracked and matched positions
    lie within TOL_PX, detections agree exactly. A status disagreement is
    excused only when the forward-backward distance of either side lies within
    MARGIN of the threshold (an FP32 tie the two summation orders may break
    differently, returned to the caller), or when both sides lost the track and
    only the reason differs because the backward pass diverged (one left the
    image, the other returned more than 1 px away).

    Positions and forward-backward distances within TOL_PX and rotations
    within TOL_THETA, or, for a track
    that is barely observable (a weak corner or an edge, where the Gauss-Newton
    system is near singular and the FP32 summation order moves its fixed
    point), no further from the FP64 track than the FP32 oracle is, plus the
    same tolerance. referee(indices) returns the FP64 (x, y, theta, fb) of
    the given records.
    """
    assert len(gpu) == len(orc), f"{where}: {len(gpu)} GPU records vs {len(orc)} oracle records"
    assert (gpu["camera"] == orc["camera"]).all(), where
    assert (gpu["id"] == orc["id"]).all(), where
    excused = []
    bad = []
    for i in np.nonzero(gpu["status"] != orc["status"])[0]:
        sg, so = int(gpu["status"][i]), int(orc["status"][i])
        near = (abs(gpu["fb_err"][i] - fb_threshold) < MARGIN or abs(orc["fb_err"][i] - fb_threshold) < MARGIN)
        # Both sides lost the track, one because the backward pass left the
        # image, the other because it came back far away: a diverged backward
        # pass, where FP32 rounding differences are amplified without bound.
        diverged = ({sg, so} == {oracle.LOST_FB, oracle.LOST_OOB} and
                    max(gpu["fb_err"][i], orc["fb_err"][i]) > 1.0)
        if {sg, so} <= {oracle.TRACKED, oracle.LOST_FB, oracle.MATCHED} and near:
            excused.append((int(gpu["id"][i]), sg, so, float(orc["fb_err"][i])))
        elif diverged:
            continue
        else:
            bad.append((int(gpu["camera"][i]), int(gpu["id"][i]), sg, so, float(gpu["fb_err"][i]),
                        float(orc["fb_err"][i]), float(gpu["x"][i]), float(orc["x"][i]), float(gpu["y"][i]),
                        float(orc["y"][i])))
    assert not bad, f"{where}: status mismatches (cam, id, gpu, oracle, fb_g, fb_o, xg, xo, yg, yo): {bad[:10]}"
    same = gpu["status"] == orc["status"]
    pos = same & np.isin(orc["status"], [oracle.TRACKED, oracle.MATCHED])
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
    det = orc["status"] == oracle.DETECTED
    assert (gpu["x"][det] == orc["x"][det]).all() and (gpu["y"][det] == orc["y"][det]).all(), where
    assert (gpu["score"][det] == orc["score"][det]).all(), where
    return excused


def _track_fp64(frames, t, orc, prev, idx, L, N, fb, d0, motion=None):
    """FP64 (x, y, theta, fb) of the tracked/matched records `idx` of frame t: temporal
    tracks from the previous state with the constant-velocity start (or the
    camera-model start where motion[camera] = (K, R, t, rho, {id: rho}) is
    given), stereo matches from the same frame's detection in the detecting
    camera (with the extrinsics start where motion[("ext", camera)] =
    (Ks, Kt, R, t, rho) is given)."""
    out = np.zeros((len(idx), 4))
    for n, i in enumerate(idx):
        c, kid = int(orc["camera"][i]), int(orc["id"][i])
        if orc["status"][i] == oracle.TRACKED:
            kp = prev[c][prev[c]["id"] == kid][0]
            src, dst = frames[t - 1][c], frames[t][c]
            pt, init = (kp["x"], kp["y"]), (2.0 * kp["x"] - kp["px"], 2.0 * kp["y"] - kp["py"])
            th0 = 0.0
            if motion and c in motion:
                K, R, tr, rho, own = motion[c]
                st, ok = oracle.motion_start(K, R, tr, np.array([pt], np.float64), own.get(kid, rho))
                if ok[0]:
                    init, th0 = (st[0, 0], st[0, 1]), st[0, 2]
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
        r, _ = oracle.track(src, dst, np.array([pt], np.float64), np.array([init], np.float64), L, N, fb,
                            double=True, theta0=th0)
        out[n] = r[0, :4]
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

            def referee(idx, t=t, o=o, prev=prev, motion=motion):
                return _track_fp64(seq.frames, t, o, prev, idx, L, N, fb, d0, motion)

            # the FP64 referee rebuilds constant-velocity and camera-model starts
            # (not the short budgets of learned or predicted tracks)
            learned = po.get("init_mode", 0) != 0 or po.get("pred_levels", 0) > 0
            exc = compare_records(g, o, workload.fb_threshold, where=f"{workload.name} frame {t}",
                                  referee=None if learned else referee)
            yield t, g, o, exc, fe_g, fe_o
    finally:
        fe_g.close()
        fe_o.close()
