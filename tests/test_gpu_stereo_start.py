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
