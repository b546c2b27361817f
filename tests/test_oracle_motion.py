"""Pins of the oracle's camera-model start (Sec. III-E: the forward warp starts
from the pattern projected through the camera model with the predicted pose
and the keypoint's inverse depth), against closed forms and an independent
statement through 3D points, and of its wiring into the frame pipeline."""
import numpy as np
import pytest

import oracle
import synthgen

K = np.array([460.0, 460.0, 375.5, 239.5])


def _rot(axis, ang):
    a = np.asarray(axis, np.float64) / np.linalg.norm(axis)
    x = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * x + (1 - np.cos(ang)) * (x @ x)


def _pts(n=50, seed=0):
    r = np.random.default_rng(seed)
    return np.stack([r.uniform(0, 751, n), r.uniform(0, 479, n)], 1)


def test_identity_motion_starts_at_the_keypoint():
    p = _pts()
    out, ok = oracle.motion_start(K, np.eye(3), np.zeros(3), p, np.linspace(0.1, 3.0, len(p)))
    assert ok.all()
    assert np.abs(out[:, :2] - p).max() < 1e-9 and np.abs(out[:, 2]).max() < 1e-12


def test_roll_rotates_about_the_principal_point():
    a = 0.07
    p = _pts()
    out, ok = oracle.motion_start(K, _rot([0, 0, 1], a), np.zeros(3), p, 0.5)
    c, s = np.cos(a), np.sin(a)
    d = p - K[2:]
    want = K[2:] + np.stack([c * d[:, 0] - s * d[:, 1], s * d[:, 0] + c * d[:, 1]], 1)
    assert ok.all() and np.abs(out[:, :2] - want).max() < 1e-9
    assert np.abs(out[:, 2] - a).max() < 1e-12


def test_sideways_and_forward_translation():
    p = _pts()
    rho = 0.25
    out, _ = oracle.motion_start(K, np.eye(3), [0.1, -0.2, 0.0], p, rho)
    assert np.abs(out[:, 0] - (p[:, 0] + K[0] * 0.1 * rho)).max() < 1e-9
    assert np.abs(out[:, 1] - (p[:, 1] - K[1] * 0.2 * rho)).max() < 1e-9
    # moving back by tz scales about the principal point by 1 / (1 + tz rho)
    out, _ = oracle.motion_start(K, np.eye(3), [0.0, 0.0, 0.8], p, rho)
    want = K[2:] + (p - K[2:]) / (1 + 0.8 * rho)
    assert np.abs(out[:, :2] - want).max() < 1e-9 and np.abs(out[:, 2]).max() < 1e-12


def test_general_motion_against_3d_points():
    """Independent statement: scene points in 3D, projected before and after
    the rigid motion; the rotation is that of the image of the point one
    pixel to the right (one pixel = Z / fx in X at depth Z)."""
    r = np.random.default_rng(3)
    Kx = np.array([410.0, 395.0, 300.2, 210.7])
    R = _rot(r.normal(size=3), 0.3)
    t = np.array([0.3, -0.1, 0.2])
    P = np.stack([r.uniform(-2, 2, 40), r.uniform(-1.5, 1.5, 40), r.uniform(2, 8, 40)], 1)

    def proj(Q):
        return np.stack([Kx[0] * Q[:, 0] / Q[:, 2] + Kx[2], Kx[1] * Q[:, 1] / Q[:, 2] + Kx[3]], 1)

    p = proj(P)
    Pn = P @ R.T + t
    P1 = P + np.stack([P[:, 2] / Kx[0], np.zeros(40), np.zeros(40)], 1)
    d = proj(P1 @ R.T + t) - proj(Pn)
    out, ok = oracle.motion_start(Kx, R, t, p, 1.0 / P[:, 2])
    assert ok.all()
    assert np.abs(out[:, :2] - proj(Pn)).max() < 1e-8
    assert np.abs(out[:, 2] - np.arctan2(d[:, 1], d[:, 0])).max() < 1e-10


def test_point_behind_the_new_camera_is_rejected():
    p = _pts(4)
    rho = 0.5  # depth 2: moving 3 forward puts the scene behind the camera
    _, ok = oracle.motion_start(K, np.eye(3), [0, 0, -3.0], p, rho)
    assert not ok.any()
    _, ok = oracle.motion_start(K, np.eye(3), [0, 0, -1.0], p, rho)
    assert ok.all()


@pytest.mark.parametrize("name", ["stereo752", "mono320"])
def test_synthetic_motion_as_a_camera_predicts_the_ground_truth(name):
    w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, n_frames=2)
    p = _pts(30, seed=5) * [w.width / 752, w.height / 480]
    for f, rho in ((300.0, 0.2), (900.0, 1.7)):
        Km, R, t = seq.camera_motion(0, f, rho)
        out, ok = oracle.motion_start(Km, R, t, p, rho)
        gx, gy = seq.gt_temporal(0, 0, p[:, 0], p[:, 1])
        assert ok.all() and max(np.abs(out[:, 0] - gx).max(), np.abs(out[:, 1] - gy).max()) < 1e-9


def _pipeline(motion=None, preds=None, frames=4, at=2):
    """Runs the oracle, setting `motion` / `preds` before frame `at` only
    (not frame 1: new keypoints have no velocity yet, so constant velocity
    starts them at the keypoint as well)."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=6, n_frames=frames)
    fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w))
    out = []
    try:
        for t in range(frames):
            if t == at and motion:
                motion(fe)
            fe.push(list(seq.frames[t]), predictions=preds(fe) if t == at and preds else None)
            out.append(fe.records())
    finally:
        fe.close()
    return out


def test_pipeline_identity_motion_equals_predictions_at_the_keypoints():
    """R = I, t = 0 starts every temporal track at its keypoint with no
    rotation, as a caller prediction at the keypoint does; only the camera
    given the motion is affected, and only for one frame."""
    def motion(fe):
        fe.set_motion(1, K, np.eye(3), np.zeros(3), 0.5)

    def preds(fe):
        ids, xy, _, _ = fe.keypoints(1)
        return [(int(i), 1, float(x), float(y)) for i, (x, y) in zip(ids, xy)]

    a, b, plain = _pipeline(motion), _pipeline(preds=preds), _pipeline()
    for t in range(4):
        assert a[t].tobytes() == b[t].tobytes(), t
    # camera 0 is untouched by camera 1's motion
    cam0 = a[2]["camera"] == 0
    assert a[2][cam0].tobytes() == plain[2][cam0].tobytes()
    assert a[2].tobytes() != plain[2].tobytes()


def test_pipeline_per_keypoint_depth_behind_the_camera_keeps_constant_velocity():
    """A keypoint whose own inverse depth puts it behind the new camera keeps
    the constant-velocity start; the others take the camera-model start."""
    state = {}

    def motion(fe):
        ids, _, _, _ = fe.keypoints(0)
        state["ids"] = ids
        # every keypoint at depth 0.5 (behind after moving 1 forward) except those with their own depth 0.1
        fe.set_motion(0, K, np.eye(3), [0, 0, -1.0], 2.0, depths=[(int(i), 0.1) for i in ids[::2]])

    a, plain = _pipeline(motion), _pipeline()
    ids = state["ids"]
    def temporal(rec, sel):
        m = (rec["camera"] == 0) & (rec["status"] != oracle.DETECTED) & np.isin(rec["id"], sel)
        return rec[m]

    behind, own = ids[1::2], ids[::2]
    assert len(behind) > 10 and len(own) > 10
    assert temporal(a[2], behind).tobytes() == temporal(plain[2], behind).tobytes()
    ra, rp = temporal(a[2], own), temporal(plain[2], own)
    assert len(ra) == len(own) and (ra["x"] != rp["x"]).mean() > 0.5


def _motion_run(params_over, frames=4):
    """stereo752 with the synthetic camera motion from frame 2 on; returns
    every frame's records, the oracle's fallback counts and the number of
    live keypoints (temporal tracks) before each frame."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=6, n_frames=frames)
    fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w, **params_over))
    out, fb, live = [], [], []
    try:
        for t in range(frames):
            live.append(sum(len(fe.keypoints(c)[0]) for c in range(2)))
            if t >= 2:
                K, R, tr = seq.camera_motion(t - 1, 420.0, 0.4)
                for c in range(2):
                    fe.set_motion(c, K, R, tr, 0.4)
            fe.push(list(seq.frames[t]))
            out.append(fe.records())
            fb.append(fe.last_fallback)
    finally:
        fe.close()
    return out, fb, live


def test_short_budget_for_predicted_tracks_reduces_to_the_full_one():
    """The predicted tracks' short budget: equal to the full budget it is the
    full run (no fallback); with a residual limit below every residual each
    predicted track falls back to the full run from the same start. Either way
    the records equal those of the full budget alone."""
    w = synthgen.WORKLOADS["stereo752"]
    full, fb0, live = _motion_run({})
    same, fb1, _ = _motion_run(dict(pred_levels=w.levels, pred_iters=w.gn_iters, pred_rho=1e9))
    back, fb2, _ = _motion_run(dict(pred_levels=2, pred_iters=3, pred_rho=-1.0))
    for t in range(4):
        assert same[t].tobytes() == full[t].tobytes(), t
        assert back[t].tobytes() == full[t].tobytes(), t
    assert fb0 == [0] * 4 and fb1 == [0] * 4
    # every temporal track of frames 2 and 3 had a camera-model start and fell back
    assert fb2[:2] == [0, 0] and fb2[2:] == live[2:] and live[2] > 100


def test_short_budget_keeps_the_predicted_tracks():
    """With the exact motion a 2-level, 3-iteration budget keeps nearly every
    predicted track without falling back."""
    short, fb, _ = _motion_run(dict(pred_levels=2, pred_iters=3, pred_rho=1e9))
    n_tr = int((short[3]["status"] == oracle.TRACKED).sum())
    assert n_tr > 200 and fb[3] < 0.02 * n_tr, (n_tr, fb)


def test_projection_into_another_camera():
    """Identity motion between two cameras of different intrinsics maps p to
    Kt Ks^-1 p (a pure change of pixel coordinates, no rotation)."""
    Ks = np.array([400.0, 380.0, 300.0, 200.0])
    Kt = np.array([800.0, 760.0, 350.5, 240.25])
    p = _pts(30, seed=9)
    out, ok = oracle.motion_start(Ks, np.eye(3), np.zeros(3), p, 0.7, Kq=Kt)
    want = np.stack([Kt[2] + Kt[0] * (p[:, 0] - Ks[2]) / Ks[0], Kt[3] + Kt[1] * (p[:, 1] - Ks[3]) / Ks[1]], 1)
    assert ok.all() and np.abs(out[:, :2] - want).max() < 1e-9
    assert np.abs(out[:, 2]).max() < 1e-12


def _stereo_run(set_ext, frames=3):
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=8, n_frames=frames)
    fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w))
    out = []
    try:
        set_ext(fe, seq)
        for t in range(frames):
            fe.push(list(seq.frames[t]))
            out.append(fe.records())
    finally:
        fe.close()
    return out, seq


def test_stereo_extrinsics_that_equal_the_disparity_prior():
    """A sideways baseline of d0 / (f rho) with equal intrinsics starts every
    match at p - (d0, 0), as the disparity prior does."""
    w = synthgen.WORKLOADS["stereo752"]
    rho, f = 0.5, 450.0
    Kc = np.array([f, f, 375.5, 239.5])

    def ext(fe, seq):
        fe.set_stereo(1, Kc, Kc, np.eye(3), [-w.disparity0 / (f * rho), 0.0, 0.0], rho)

    a, _ = _stereo_run(ext)
    b, _ = _stereo_run(lambda fe, seq: None)
    for ra, rb in zip(a, b):
        assert len(ra) == len(rb) and (ra["status"] == rb["status"]).all() and (ra["id"] == rb["id"]).all()
        assert np.abs(ra["x"] - rb["x"]).max() < 1e-4 and np.abs(ra["y"] - rb["y"]).max() < 1e-4


def test_stereo_extrinsics_from_the_rig_land_on_the_ground_truth():
    """Baselines from each synthetic rig's disparity plane (its constant term)
    start the matches closer than the fixed prior; they still land on the
    ground truth, and the cleared extrinsics give the prior's records back."""
    rho, f = 0.5, 450.0
    Kc = np.array([f, f, 375.5, 239.5])

    def ext(fe, seq):
        c = seq.planes[0][0][2]
        fe.set_stereo(1, Kc, Kc, np.eye(3), [-c / (f * rho), 0.0, 0.0], rho)

    out, seq = _stereo_run(ext, frames=1)
    rec = out[0]
    det = rec[(rec["camera"] == 0) & (rec["status"] == oracle.DETECTED)]
    m = rec[(rec["camera"] == 1) & (rec["status"] == oracle.MATCHED)]
    pos = {int(i): (x, y) for i, x, y in zip(det["id"], det["x"], det["y"])}
    src = np.array([pos[int(i)] for i in m["id"]])
    gx, gy = seq.gt_stereo(0, src[:, 0], src[:, 1])
    assert len(m) > 0.8 * len(det) and np.median(np.hypot(m["x"] - gx, m["y"] - gy)) < 0.1

    def cleared(fe, seq):
        ext(fe, seq)
        fe.set_stereo(1)

    a, _ = _stereo_run(cleared, frames=2)
    b, _ = _stereo_run(lambda fe, seq: None, frames=2)
    assert all(x.tobytes() == y.tobytes() for x, y in zip(a, b))
