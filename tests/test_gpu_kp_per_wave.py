"""Two keypoints per tracking wave (vio_frontend_params.track_kp_per_wave = 2:
one keypoint per 32-lane half, two pattern points per lane) is a launch
choice: its records are those of one keypoint per wave, bit for bit. The
cases reach every path of the two-per-wave driver: both halves in one pass,
a half without an item (odd counts), halves of two cameras or two stereo
targets (a pair across segment or target boundaries runs its halves one after
the other), halves with different budgets (predicted and learned starts side
by side), short attempts kept by one half and not the other, parallel
fallbacks, the neighbour stereo start, the persistent grid and an odd level
count. The records also meet the CPU oracle directly.
"""
import os

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


# uneven mix with odd keypoint caps, so that pairs of items straddle cameras
MIX = [
    synthgen.Workload("k320", 3, 320, 240, n_frames=5, cell_size=16, max_keypoints=121),
    synthgen.Workload("k752", 3, 752, 480, stereo=True, n_frames=5, cell_size=32, max_keypoints=301),
    synthgen.Workload("k400", 3, 400, 304, stereo=True, n_frames=5, cell_size=24, max_keypoints=77),
]


def _lockstep(streams, seqs, frames, params, mlp=None, preds=None):
    """Steps two handles, one keypoint per wave and two, over the same frames
    and compares every stream's records and the fallback counts; returns the
    number of records and of fallbacks."""
    import paper_2609_30459_amd as vf
    n_rec = n_fb = 0
    with vf.Frontend(streams, vf.make_params(**params)) as a, \
            vf.Frontend(streams, vf.make_params(**params, track_kp_per_wave=2)) as b:
        for fe in (a, b):
            if mlp is not None:
                fe.set_mlp(*mlp)
        for t in range(frames):
            print(f"  frame {t}", flush=True)
            for s, seq in enumerate(seqs):
                p = preds(t, a, s) if preds else None
                a.push_stereo_frame(s, t + 1, list(seq.frames[t]), predictions=p)
                b.push_stereo_frame(s, t + 1, list(seq.frames[t]), predictions=p)
            for s in range(len(streams)):
                ra, rb = a.get_tracks(s), b.get_tracks(s)
                assert ra.tobytes() == rb.tobytes(), (t, s)
                n_rec += len(ra)
            sa, sb = a.stats(), b.stats()
            assert sa["last_fallback"] == sb["last_fallback"], t
            n_fb += sa["last_fallback"]
    return n_rec, n_fb


def _base(w, **kw):
    return dict(levels=w.levels, gn_iters=w.gn_iters, cell_size=w.cell_size, k_per_cell=w.k_per_cell,
                thresholds=w.thresholds, edge_margin=w.edge_margin, max_keypoints=w.max_keypoints,
                fb_threshold=w.fb_threshold, disparity0=w.disparity0, topology=1 if w.star else 0, **kw)


@pytest.mark.parametrize("launch", [dict(), dict(stereo_mode=1, track_block_waves=1),
                                    dict(track_waves_per_cu=4, stereo_mode=1), dict(track_waves_per_cu=2,
                                                                                   track_block_waves=2)])
def test_batch_of_uneven_streams(launch):
    import paper_2609_30459_amd as vf
    seqs = [synthgen.sequence(w, seq=30 + i, n_frames=5) for i, w in enumerate(MIX)]
    streams = [(w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size) for w in MIX]
    print(f"case batch {launch}", flush=True)
    p = _base(MIX[1], **launch)
    with vf.Frontend(streams, vf.make_params(**p)) as a, \
            vf.Frontend(streams, vf.make_params(**p, track_kp_per_wave=2)) as b:
        for t in range(5):
            for s, seq in enumerate(seqs):
                a.stage_frame(s, t + 1, list(seq.frames[t]))
                b.stage_frame(s, t + 1, list(seq.frames[t]))
            a.step()
            b.step()
            for s in range(len(MIX)):
                ra, rb = a.get_tracks(s), b.get_tracks(s)
                assert len(ra) > 0 and ra.tobytes() == rb.tobytes(), (t, s)


def _mlp():
    import paper_2609_30459_amd as vf
    from paper_2609_30459_amd.train_mlp import load_weights
    params, rho, _ = load_weights(os.path.join(os.path.dirname(vf.__file__), "weights", "mlp_stereo1280.bin"))
    return params, rho


@pytest.mark.parametrize("extra", [
    dict(),
    dict(track_parallel_fallback=1),
    dict(learned_fb_levels=2, learned_fb_iters=5, stereo_init=1),
    dict(track_waves_per_cu=4, stereo_mode=1, stereo_init=1, track_parallel_fallback=1),
])
def test_learned_initialisation(extra):
    """The learned stage in its own launch, short attempts from the network's
    guess with a residual limit that sends a part of them to the fallback."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=9, n_frames=5)
    params, _ = _mlp()
    p = _base(w, init_mode=1, learned_levels=2, learned_iters=3, learned_rho=0.03, **extra)
    print(f"case learned {extra}", flush=True)
    n_rec, n_fb = _lockstep([(2, w.width, w.height, w.max_keypoints, w.cell_size)], [seq], 5, p,
                            mlp=(params, 0.03))
    assert n_rec > 0 and n_fb > 0


def test_learned_and_predicted_starts_side_by_side():
    """Caller predictions for every third keypoint of the left camera with a
    short predicted budget, the rest from the network's guess with their own
    fallback budget: pairs whose halves run different budgets."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=10, n_frames=5)
    params, _ = _mlp()
    p = _base(w, init_mode=1, learned_levels=2, learned_iters=3, learned_rho=0.03, learned_fb_levels=3,
              learned_fb_iters=4, pred_levels=2, pred_iters=4, pred_rho=0.02)

    def preds(t, fe, s):
        kp = fe.get_keypoints(s, 0)[::3]
        return [(int(k["id"]), 0, 2 * k["x"] - k["px"] + 0.25, 2 * k["y"] - k["py"] - 0.25) for k in kp]

    print("case learned + predicted", flush=True)
    n_rec, n_fb = _lockstep([(2, w.width, w.height, w.max_keypoints, w.cell_size)], [seq], 5, p,
                            mlp=(params, 0.03), preds=preds)
    assert n_rec > 0 and n_fb > 0


@pytest.mark.parametrize("stereo_mode", [0, 1])
def test_star_rig(stereo_mode):
    """Camera 0 matched into cameras 1..3: stereo items of three targets."""
    w = synthgen.WORKLOADS["star752"]
    seq = synthgen.sequence(w, seq=11, n_frames=4)
    print(f"case star stereo_mode={stereo_mode}", flush=True)
    n_rec, _ = _lockstep([(w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size)], [seq], 4,
                         _base(w, stereo_mode=stereo_mode))
    assert n_rec > 0


@pytest.mark.parametrize("name,frames", [("stereo752", 6), ("rig4", 3)])
def test_oracle_parity(name, frames):
    w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, seq=12, n_frames=frames)
    print(f"case oracle {name}", flush=True)
    n_tr = 0
    for t, g, o, exc, _, _ in run_pair(w, seq, frames, launch=dict(track_kp_per_wave=2)):
        assert len(exc) <= 1, (t, exc)
        n_tr += int((o["status"] == oracle.TRACKED).sum())
    assert n_tr > 0


def test_three_levels():
    """The kernels of an odd level count (L = 3: mono320 in free motion, its
    default being a two-frame warp), bitwise against one keypoint per wave on a
    sequence whose keypoint 90 turns by 0.33 rad along a weak direction."""
    w = synthgen.WORKLOADS["mono320"].with_(warp_second=False, name="mono320_free")
    seq = synthgen.sequence(w, seq=12, n_frames=5)
    print("case mono320_free L=3", flush=True)
    n_rec, _ = _lockstep([(1, w.width, w.height, w.max_keypoints, w.cell_size)], [seq], 5, _base(w))
    assert n_rec > 0


def test_arguments():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    for bad in (dict(track_kp_per_wave=3), dict(track_kp_per_wave=-1),
                dict(track_kp_per_wave=2, init_mode=1, learned_fused=1)):
        with pytest.raises(vf.VioError):
            vf.Frontend([stream], vf.params_for(w, **bad))
    # learned_fused only matters with learned initialisation
    with vf.Frontend([stream], vf.params_for(w, track_kp_per_wave=2, learned_fused=1)):
        pass
