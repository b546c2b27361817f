"""Pins of the oracle's star topology (a four-camera rig whose first camera
detects and whose new keypoints are matched into the other three, as the
paper runs the four-camera headset of its dataset, Sec. IV-A)."""
import numpy as np

import oracle
import synthgen

STAR = synthgen.WORKLOADS["stereo752"].with_(star=True, name="star752", n_frames=4)


def _run(n_cams, frames, topology, stereo=True):
    w = STAR
    fe = oracle.Frontend([w.width] * n_cams, [w.height] * n_cams, stereo, oracle.params_for(w, topology=topology))
    out = []
    try:
        for f in frames:
            fe.push(list(f))
            out.append(fe.records())
    finally:
        fe.close()
    return out


def _cam(rec, c):
    return rec[rec["camera"] == c]


def test_star_first_pair_equals_a_stereo_pair():
    """Only camera 0 detects, so cameras 0 and 1 of the star see exactly what
    a stereo pair of the same two images sees."""
    seq = synthgen.sequence(STAR, seq=1, n_frames=4)
    star = _run(4, seq.frames, 1)
    pair = _run(2, seq.frames[:, :2], 0)
    for t in range(4):
        for c in (0, 1):
            assert _cam(star[t], c).tobytes() == _cam(pair[t], c).tobytes(), (t, c)
        assert len(_cam(star[t], 2)) > 0 and len(_cam(star[t], 3)) > 0


def test_star_targets_follow_one_procedure():
    """With cameras 2 and 3 given camera 1's images, their records are
    camera 1's with the camera index changed."""
    seq = synthgen.sequence(STAR, seq=2, n_frames=3)
    f = seq.frames.copy()
    f[:, 2] = f[:, 1]
    f[:, 3] = f[:, 1]
    out = _run(4, f, 1)
    for t in range(3):
        r1 = _cam(out[t], 1).copy()
        for c in (2, 3):
            rc = _cam(out[t], c).copy()
            assert len(rc) == len(r1) > 0
            rc["camera"] = 1
            assert rc.tobytes() == r1.tobytes(), (t, c)


def test_star_matches_land_on_the_ground_truth():
    seq = synthgen.sequence(STAR, seq=3, n_frames=1)
    rec = _run(4, seq.frames, 1)[0]
    det = _cam(rec, 0)
    det = det[det["status"] == oracle.DETECTED]
    pos = {int(i): (x, y) for i, x, y in zip(det["id"], det["x"], det["y"])}
    for c in (1, 2, 3):
        m = _cam(rec, c)
        m = m[m["status"] == oracle.MATCHED]
        assert len(m) > 0.8 * len(det)
        src = np.array([pos[int(i)] for i in m["id"]], np.float64)
        gx, gy = seq.gt_stereo(0, src[:, 0], src[:, 1], c)
        err = np.hypot(m["x"] - gx, m["y"] - gy)
        assert np.median(err) < 0.1, (c, np.median(err))
