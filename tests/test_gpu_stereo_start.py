"""The neighbour stereo start (VIO_STEREO_INIT_NEIGHBOUR) and the learned
fallback budget on the GPU against the CPU oracle, through the C ABI. The pair
tables come from the selection kernel after each frame, or are rebuilt after
a host upload of keypoints (the state-injected runs exercise both: frame 0's
table comes from the kernel, later ones from the injection)."""
import numpy as np
import pytest

import oracle
import synthgen
from parity_util import run_pair

pytestmark = pytest.mark.gpu

NB = dict(stereo_init=1, stereo_levels=2, stereo_iters=3)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_30459_amd  # noqa: F401  (raises when the library is missing)


@pytest.mark.parametrize("stereo_mode", [0, 1])
@pytest.mark.parametrize("name,frames,inject", [("stereo752", 6, True), ("stereo752", 8, False),
                                                ("star752", 5, True), ("stereo1280", 5, False)])
def test_neighbour_stereo_start_parity(name, frames, inject, stereo_mode):
    w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, seq=6, n_frames=frames)
    print(f"case {name} frames={frames} inject={inject} stereo_mode={stereo_mode}", flush=True)
    matched = 0
    for t, g, o, exc, _, _ in run_pair(w, seq, frames, inject_state=inject, params_overrides=NB,
                                       launch={"stereo_mode": stereo_mode}):
        if t > 0:
            matched += int(((o["status"] == oracle.MATCHED) & (o["age"] == 0)).sum())
    assert matched > 0


def test_neighbour_stereo_start_deferred_equals_speculative_bitwise():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"].with_(n_canvases=2)
    seq = synthgen.sequence(w, seq=9, n_frames=6)
    stream = (4, w.width, w.height, w.max_keypoints, w.cell_size)
    with vf.Frontend([stream], vf.params_for(w, **NB)) as a, \
            vf.Frontend([stream], vf.params_for(w, stereo_mode=1, **NB)) as b:
        for t in range(6):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            ra, rb = a.get_tracks(0), b.get_tracks(0)
            assert len(ra) > 0 and ra.tobytes() == rb.tobytes(), t


def test_stereo_init_arguments():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    for bad in (dict(stereo_init=2), dict(stereo_init=1, stereo_levels=0), dict(stereo_init=1, stereo_levels=5),
                dict(stereo_init=1, stereo_iters=0), dict(learned_fb_levels=5), dict(learned_fb_levels=2,
                                                                                     learned_fb_iters=0)):
        with pytest.raises(vf.VioError):
            vf.Frontend([stream], vf.params_for(w, **bad))


@pytest.mark.parametrize("name,extra", [
    ("stereo752", dict(init_mode=1, learned_levels=2, learned_iters=3, learned_rho=0.03)),
    ("stereo1280", dict(init_mode=1, learned_levels=2, learned_iters=3, learned_rho=0.03, learned_fb_levels=2,
                        learned_fb_iters=5, stereo_init=1)),
    ("stereo752", dict(init_mode=1, learned_levels=2, learned_iters=3, learned_rho=-1.0, learned_fb_levels=3,
                       learned_fb_iters=4))])
@pytest.mark.parametrize("launch", [{}, {"stereo_mode": 1}, {"track_waves_per_cu": 4}])
def test_parallel_fallback_equals_serial_bitwise(name, extra, launch):
    """The parallel fallbacks (a second wave per short attempt) give the records
    of the serial ones, bit for bit, and the same fallback counts."""
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, seq=8, n_frames=5)
    P = oracle.mlp_init(13) * 0.05
    P[-3:] = 0.0
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    fbs = 0
    with vf.Frontend([stream], vf.params_for(w, **extra, **launch)) as a, \
            vf.Frontend([stream], vf.params_for(w, track_parallel_fallback=1, **extra, **launch)) as b:
        a.set_mlp(P)
        b.set_mlp(P)
        for t in range(5):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            ra, rb = a.get_tracks(0), b.get_tracks(0)
            assert len(ra) > 0 and ra.tobytes() == rb.tobytes(), t
            sa, sb = a.stats(), b.stats()
            assert sa["last_fallback"] == sb["last_fallback"], t
            fbs += sa["last_fallback"]
    assert fbs > 0


def test_parallel_fallback_of_predicted_tracks_equals_serial():
    """Predicted (camera-model) starts with a short budget: parallel = serial."""
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=2, n_frames=5)
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    over = dict(pred_levels=2, pred_iters=3, pred_rho=0.02)
    fbs = 0
    with vf.Frontend([stream], vf.params_for(w, **over)) as a, \
            vf.Frontend([stream], vf.params_for(w, track_parallel_fallback=1, **over)) as b:
        for t in range(5):
            if t > 0:
                K, R, tr = seq.camera_motion(t - 1, 450.0, 0.5)
                for fe in (a, b):
                    if t == 1:
                        fe.set_camera_model(0, 0, K)
                        fe.set_camera_model(0, 1, K)
                    fe.set_motion(0, [(0, R, tr, 0.5), (1, R, tr, 0.5)])
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            assert a.get_tracks(0).tobytes() == b.get_tracks(0).tobytes(), t
            fbs += a.stats()["last_fallback"]
    assert fbs > 0
