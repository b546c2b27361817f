"""The FP64 referee of the record comparison rebuilds each track's
inputs (frames, start point, initial guess) from the oracle's state; on
well-conditioned tracks its position, rotation and forward-backward
distance must agree with the FP32 oracle's."""
import numpy as np

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
                d = np.abs(th - np.stack([o["x"][idx], o["y"][idx], o["theta"][idx], o["fb_err"][idx]], 1)).max(1)
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
        d = np.abs(ref - np.stack([o["x"][idx], o["y"][idx], o["theta"][idx], o["fb_err"][idx]], 1)).max(1)
        assert np.median(d) < 1e-4 and (d < 1e-3).mean() > 0.9, np.sort(d)[-5:]
    finally:
        fe.close()
