"""The FP64 referee of the record comparison rebuilds each track's
inputs (frames, start point, initial guess) from the oracle's state; on
well-conditioned tracks its position, rotation and forward-backward
distance must agree with the FP32 oracle's."""
import numpy as np
import pytest

import oracle
import synthgen
from parity_util import _track_fp64, oracle_state


def test_referee_rebuilds_temporal_and_stereo_tracks():
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=3, n_frames=3)
    fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w))
    try:
        for t in range(3):
            prev = [oracle_state(fe, c) for c in range(2)]
            fe.push(list(seq.frames[t]))
            o = fe.records()
            for st in (oracle.TRACKED, oracle.MATCHED):
                idx = np.nonzero(o["status"] == st)[0][:40]
                # frame 0 has no temporal tracks; later frames add few detections
                want = 0 if (t == 0) == (st == oracle.TRACKED) else 10
                assert len(idx) >= want, (t, st, len(idx))
                if len(idx) < 10:
                    continue
                th = _track_fp64(seq.frames, t, o, prev, idx, w.levels, w.gn_iters, w.fb_threshold, w.disparity0)
                d = np.abs(th[:, :4] - np.stack([o["x"][idx], o["y"][idx], o["theta"][idx], o["fb_err"][idx]], 1)).max(1)
                assert np.median(d) < 1e-4 and (d < 1e-3).mean() > 0.9, (t, st, np.sort(d)[-5:])
    finally:
        fe.close()


def test_referee_rebuilds_camera_model_starts():
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=3, n_frames=3)
    fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w))
    try:
        for t in range(3):
            prev = [oracle_state(fe, c) for c in range(2)]
            motion = None
            if t == 2:
                K, R, tr = seq.camera_motion(1, 400.0, 0.5)
                ids = prev[0]["id"]
                own = {int(i): 0.5 for i in ids[::3]}
                fe.set_motion(0, K, R, tr, 0.5, depths=list(own.items()))
                motion = {0: (K, R, tr, 0.5, own)}
            fe.push(list(seq.frames[t]))
        o = fe.records()
        idx = np.nonzero((o["status"] == oracle.TRACKED) & (o["camera"] == 0))[0][:40]
        assert len(idx) > 10
        ref = _track_fp64(seq.frames, 2, o, prev, idx, w.levels, w.gn_iters, w.fb_threshold, w.disparity0, motion)
        d = np.abs(ref[:, :4] - np.stack([o["x"][idx], o["y"][idx], o["theta"][idx], o["fb_err"][idx]], 1)).max(1)
        assert np.median(d) < 1e-4 and (d < 1e-3).mean() > 0.9, np.sort(d)[-5:]
    finally:
        fe.close()


def test_weak_ratio_separates_corners_from_edges():
    """lambda_min / lambda_max of the Gauss-Newton matrix: a ramp (aperture
    problem) has a singular system, a textured corner region a well-conditioned
    one; a one-dimensional texture (vertical stripes) leaves y unconstrained."""
    from parity_util import RATIO_BOUND, weak_ratio
    yy, xx = np.mgrid[0:48, 0:48]
    ramp = (2 * xx + 3 * yy + 10).astype(np.uint8)
    assert abs(weak_ratio(ramp, 24, 24)) < 1e-9
    stripes = (120 + 60 * np.sin(xx * 0.9)).astype(np.uint8)
    assert weak_ratio(stripes, 24.3, 24) < 1e-6
    img = synthgen.sequence(synthgen.WORKLOADS["stereo752"], n_frames=1).frames[0, 0]
    d = oracle.detect(img, 32)[:, 0]
    pts = d[d[:, 2] >= 20, :2][:50]
    r = np.array([weak_ratio(img, x, y) for x, y in pts])
    assert np.median(r) > 3 * RATIO_BOUND and (r <= 1).all()
    assert weak_ratio(img, 2.0, 2.0) == 0.0  # the template does not fit


def test_tally_caps():
    from parity_util import Tally
    t = Tally("unit", register=False)
    t.compared = 1000
    t.check(1)
    t.referred.append(("unit", 7, 1e-3, 2e-3))
    with pytest.raises(AssertionError):
        t.check(1)          # one keypoint per cell: only a ratio below 1e-3
    t.referred[0] = ("unit", 7, 5e-4, 2e-3)
    t.check(1)              # ... and only one per run
    t.referred.append(("unit", 8, 5e-4, 2e-3))
    with pytest.raises(AssertionError):
        t.check(1)
    t.referred.pop()
    t.check(3)              # k > 1: up to 0.5 % of the compared tracks
    t.referred += [("unit", i, 1e-3, 2e-3) for i in range(5)]
    with pytest.raises(AssertionError):
        t.check(3)
    t.referred.clear()
    t.margin += [1, 2]
    with pytest.raises(AssertionError):
        t.check(1)          # at most one FP32 tie at the threshold per run
