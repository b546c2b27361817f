"""Camera-model start of the temporal tracks (Sec. III-E: the forward warp
starts from the pattern projected through the camera model with the predicted
pose and the keypoint's inverse depth) against the CPU oracle, through the C
ABI, and its argument checks."""
import numpy as np
import pytest

import oracle
import synthgen
from parity_util import run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_30459_amd  # noqa: F401  (raises when the library is missing)


def _motion_hook(w, seq, f=420.0, rho=0.4, from_frame=2, per_keypoint=True, cams=None):
    """Sets both sides' camera models once and, from `from_frame` on, the
    synthetic motion of frame t-1 -> t as every camera's predicted motion
    (exact for the left cameras; the right ones see the left's), with
    per-keypoint inverse depths for a third of the keypoints."""
    cams = list(range(w.n_cams)) if cams is None else cams

    def hook(t, fe_g, fe_o):
        if t == 0:
            for c in cams:
                K, _, _ = seq.camera_motion(0, f, rho)
                fe_g.set_camera_model(0, c, K)
        if t < from_frame:
            return None
        K, R, tr = seq.camera_motion(t - 1, f, rho)
        K32, R32, t32 = (np.asarray(a, np.float32).astype(np.float64) for a in (K, R, tr))
        motions, depths, out = [], [], {}
        for c in cams:
            own = {}
            if per_keypoint:
                ids, _, _, _ = fe_o.keypoints(c)
                r = np.random.default_rng(100 * t + c)
                own = {int(i): float(np.float32(rho * r.uniform(0.8, 1.25))) for i in ids[::3]}
            fe_o.set_motion(c, K32, R32, t32, float(np.float32(rho)), depths=list(own.items()))
            motions.append((c, R32, t32, rho))
            depths += [(i, c, d) for i, d in own.items()]
            out[c] = (K32, R32, t32, float(np.float32(rho)), own)
        fe_g.set_motion(0, motions, depths)
        return out

    return hook


@pytest.mark.parametrize("name,frames", [("stereo752", 6), ("rig4", 4), ("mono320_free", 5)])
def test_camera_model_start_parity(name, frames):
    if name == "mono320_free":
        w = synthgen.WORKLOADS["mono320"].with_(warp_second=False, name="mono320_free")
    else:
        w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, seq=7, n_frames=frames)
    print(f"case {name} frames={frames}", flush=True)
    excused, n_tr = [], 0
    for t, g, o, exc, _, _ in run_pair(w, seq, frames, before_push=_motion_hook(w, seq)):
        excused += exc
        n_tr += int((o["status"] == oracle.TRACKED).sum())
        print(f"  frame {t}: {len(g)} records, statuses {np.bincount(g['status'], minlength=7).tolist()}", flush=True)
    assert n_tr > 0
    assert len(excused) <= 1, excused


def test_camera_model_start_only_on_named_cameras_and_one_frame():
    """Motion for the right camera only, at frame 2 only: the parity run
    covers which camera takes it and that the next frame goes back to the
    constant-velocity start."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=8, n_frames=5)
    hook = _motion_hook(w, seq, cams=[1], per_keypoint=False)

    def once(t, fe_g, fe_o):
        return hook(t, fe_g, fe_o) if t <= 2 else None

    for t, g, o, exc, _, _ in run_pair(w, seq, 5, before_push=once):
        assert len(exc) <= 1, (t, exc)


def test_learned_mode_skips_the_network_for_camera_model_starts():
    import paper_2609_30459_amd as vf
    from paper_2609_30459_amd.train_mlp import load_weights
    import os
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=2, n_frames=4)
    path = os.path.join(os.path.dirname(vf.__file__), "weights", "mlp_stereo1280.bin")
    params, _, _ = load_weights(path)
    # rho = 0: every learned track falls back, so the fallback count shows which tracks tried the network
    p = vf.params_for(w, init_mode=1, learned_levels=2, learned_iters=3, learned_rho=0.0)
    fb = []
    with vf.Frontend([(2, w.width, w.height, w.max_keypoints, w.cell_size)], p) as fe:
        fe.set_mlp(params, 0.0)
        for c in range(2):
            fe.set_camera_model(0, c, seq.camera_motion(0, 420.0, 0.4)[0])
        for t in range(4):
            if t == 3:
                _, R, tr = seq.camera_motion(2, 420.0, 0.4)
                fe.set_motion(0, [(0, R, tr, 0.4), (1, R, tr, 0.4)])
            fe.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            fb.append(fe.stats()["last_fallback"])
    assert fb[2] > 100 and fb[3] == 0, fb


def test_set_motion_rejects_bad_arguments_and_keeps_nothing():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=3, n_frames=4)
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    K, R, tr = seq.camera_motion(1, 420.0, 0.4)
    with vf.Frontend([stream], vf.params_for(w)) as a, vf.Frontend([stream], vf.params_for(w)) as b:
        with pytest.raises(vf.VioError):
            a.set_motion(0, [(0, R, tr, 0.4)])                      # no camera model yet
        with pytest.raises(vf.VioError):
            a.set_camera_model(0, 0, (0.0, 420.0, 1.0, 1.0))         # fx <= 0
        with pytest.raises(vf.VioError):
            a.set_camera_model(0, 2, K)                               # camera out of range
        a.set_camera_model(0, 0, K)
        bad = [
            ([(0, R, tr, 0.4), (0, R, tr, 0.4)], []),                # camera twice
            ([(0, R, tr, 0.0)], []),                                  # inverse depth 0
            ([(0, R, tr, float("nan"))], []),                         # not finite
            ([(1, R, tr, 0.4)], []),                                  # camera without a model
            ([(0, R, tr, 0.4)], [(5, 1, 0.3)]),                       # depth for a camera without motion
            ([(0, R, tr, 0.4)], [(5, 0, 0.3), (5, 0, 0.2)]),          # repeated depth
            ([(0, R, tr, 0.4)], [(5, 0, -1.0)]),                      # negative depth
            ([(0, R, tr, 0.4)], [(i, 0, 0.3) for i in range(w.max_keypoints + 1)]),  # too many depths
        ]
        for m, d in bad:
            with pytest.raises(vf.VioError):
                a.set_motion(0, m, d)
        # nothing was kept: both handles give the same records
        for t in range(4):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            assert a.get_tracks(0).tobytes() == b.get_tracks(0).tobytes(), t


def test_staged_batch_with_motion_equals_single_pushes():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    seqs = [synthgen.sequence(w, seq=5, stream=i, n_frames=4) for i in range(3)]
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    with vf.Frontend([stream] * 3, vf.params_for(w)) as batch, vf.Frontend([stream] * 3, vf.params_for(w)) as single:
        for fe in (batch, single):
            for s in range(3):
                for c in range(2):
                    fe.set_camera_model(0 + s, c, seqs[s].camera_motion(0, 420.0, 0.4)[0])
        for t in range(4):
            for s in range(3):
                for fe in (batch, single):
                    if t >= 2 and s != 1:  # stream 1 runs without motion
                        _, R, tr = seqs[s].camera_motion(t - 1, 420.0, 0.4)
                        fe.set_motion(s, [(0, R, tr, 0.4), (1, R, tr, 0.5)])
                batch.stage_frame(s, t + 1, list(seqs[s].frames[t]))
                single.push_stereo_frame(s, t + 1, list(seqs[s].frames[t]))
            batch.step()
            for s in range(3):
                assert batch.get_tracks(s).tobytes() == single.get_tracks(s).tobytes(), (t, s)


@pytest.mark.parametrize("pred_rho", [3.0e38, 0.03])
def test_short_budget_of_predicted_tracks_parity(pred_rho):
    """Predicted tracks first run 2 levels x 3 iterations; rho = 0.03 makes a
    part of them fall back to the full budget. Records and fallback counts
    equal the oracle's."""
    w = synthgen.WORKLOADS["rig4"]
    seq = synthgen.sequence(w, seq=3, n_frames=4)
    over = dict(pred_levels=2, pred_iters=3, pred_rho=pred_rho)
    n_fb = []
    for t, g, o, exc, fe_g, fe_o in run_pair(w, seq, 4, params_overrides=over,
                                              before_push=_motion_hook(w, seq, per_keypoint=False)):
        assert len(exc) <= 1, (t, exc)
        assert fe_g.stats()["last_fallback"] == fe_o.last_fallback, t
        n_fb.append(fe_o.last_fallback)
    if pred_rho < 1.0:
        assert n_fb[3] > 0, n_fb


def _ext_hook(w, seq, f=450.0, rho=0.5, clear_at=None):
    """Both sides: every target camera's matches start from extrinsics built
    from its synthetic disparity plane (a sideways baseline of c / (f rho)),
    the two cameras with different principal points."""
    Ks = np.array([f, f, 375.5, 239.5], np.float32)
    Kt = np.array([f, f, 371.0, 241.0], np.float32)
    views = seq.views

    def hook(t, fe_g, fe_o):
        if t == 0:
            for c in range(w.n_cams):
                fe_g.set_camera_model(0, c, Ks if c % views == 0 else Kt)
            for c in range(w.n_cams):
                if c % views == 0:
                    continue
                cc = float(seq._plane(c)[2])
                # x_t = cx_t + f (a + rho tx) = x_s - c  =>  tx = (cx_s - cx_t - c) / (f rho)
                tr = np.array([(Ks[2] - Kt[2] - cc) / (f * rho), (Ks[3] - Kt[3]) / (f * rho), 0.0], np.float32)
                fe_g.set_stereo_extrinsics(0, c, np.eye(3), tr, rho)
                fe_o.set_stereo(c, Ks.astype(np.float64), Kt.astype(np.float64), np.eye(3),
                                tr.astype(np.float64), float(np.float32(rho)))
        if clear_at is not None and t == clear_at:
            for c in range(w.n_cams):
                if c % views:
                    fe_g.set_stereo_extrinsics(0, c, None)
                    fe_o.set_stereo(c)
        return None

    return hook


@pytest.mark.parametrize("name", ["stereo752", "star752"])
def test_stereo_extrinsics_start_parity(name):
    w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, seq=4, n_frames=4)
    print(f"case {name}", flush=True)
    matched = 0
    for t, g, o, exc, _, _ in run_pair(w, seq, 4, before_push=_ext_hook(w, seq, clear_at=3)):
        assert len(exc) <= 1, (t, exc)
        matched += int((o["status"] == oracle.MATCHED).sum())
    assert matched > 100


def test_stereo_extrinsics_arguments():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    with vf.Frontend([(2, w.width, w.height, 300, 32)], vf.params_for(w)) as fe:
        with pytest.raises(vf.VioError):
            fe.set_stereo_extrinsics(0, 1, np.eye(3), [0.1, 0, 0], 0.5)  # no camera models yet
        fe.set_camera_model(0, 0, (450.0, 450.0, 375.5, 239.5))
        fe.set_camera_model(0, 1, (450.0, 450.0, 375.5, 239.5))
        with pytest.raises(vf.VioError):
            fe.set_stereo_extrinsics(0, 0, np.eye(3), [0.1, 0, 0], 0.5)  # camera 0 detects
        with pytest.raises(vf.VioError):
            fe.set_stereo_extrinsics(0, 1, np.eye(3), [0.1, 0, 0], 0.0)  # inverse depth 0
        fe.set_stereo_extrinsics(0, 1, np.eye(3), [0.1, 0, 0], 0.5)
        fe.set_stereo_extrinsics(0, 1, None)
