"""Batched stepping of many uneven streams (one submit, persistent tracking grid).

Invariants: a batched step gives exactly the records of stepping each stream
on its own, for the one-wave-per-item and the persistent tracking grids alike;
and each stream of a batch matches its own CPU oracle.
"""
import numpy as np
import pytest

import oracle
import synthgen
from parity_util import Tally, compare_records

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# small uneven mix: mono 320x240, stereo 752x480, stereo 400x300 with 5 levels' worth of size
MIX = [
    synthgen.Workload("b320", 3, 320, 240, n_frames=4, cell_size=16, max_keypoints=120),
    synthgen.Workload("b752", 3, 752, 480, stereo=True, n_frames=4, cell_size=32, max_keypoints=300),
    synthgen.Workload("b400", 3, 400, 304, stereo=True, n_frames=4, cell_size=24, max_keypoints=80),
]


def _seqs(n_frames):
    return [synthgen.sequence(w, seq=20 + i, n_frames=n_frames) for i, w in enumerate(MIX)]


def _streams():
    return [(w.n_cams, w.width, w.height, w.max_keypoints, w.cell_size) for w in MIX]


@pytest.mark.parametrize("waves_per_cu,block_waves,tile,stereo_mode",
                         [(0, 4, 64, 0), (0, 1, 32, 1), (4, 4, 64, 1), (2, 2, 32, 0)])
def test_batched_step_equals_per_stream_push(waves_per_cu, block_waves, tile, stereo_mode):
    import paper_2609_30459_amd as vf
    seqs = _seqs(4)
    params = vf.params_for(MIX[1], track_waves_per_cu=waves_per_cu, track_block_waves=block_waves, pyr_tile=tile,
                           stereo_mode=stereo_mode)
    with vf.Frontend(_streams(), params) as a, vf.Frontend(_streams(), vf.params_for(MIX[1])) as b:
        for t in range(4):
            for s, seq in enumerate(seqs):
                a.stage_frame(s, t + 1, list(seq.frames[t]))
            a.step()
            for s, seq in enumerate(seqs):
                b.push_stereo_frame(s, t + 1, list(seq.frames[t]))
            for s in range(len(MIX)):
                ra, rb = a.get_tracks(s), b.get_tracks(s)
                assert len(ra) > 0 and ra.tobytes() == rb.tobytes(), (t, s)


def test_batched_streams_match_their_oracles():
    import paper_2609_30459_amd as vf
    seqs = _seqs(4)
    orcs = [oracle.Frontend([w.width] * w.n_cams, [w.height] * w.n_cams, w.stereo,
                            oracle.params_for(MIX[1], max_keypoints=w.max_keypoints, cell_size=w.cell_size))
            for w in MIX]
    tally = Tally("batch of three streams, 4 frames, persistent grid")
    with vf.Frontend(_streams(), vf.params_for(MIX[1], track_waves_per_cu=8)) as fe:
        for t in range(4):
            for s, seq in enumerate(seqs):
                fe.stage_frame(s, t + 1, list(seq.frames[t]))
                orcs[s].push(list(seq.frames[t]))
            fe.step()
            for s in range(len(MIX)):
                compare_records(fe.get_tracks(s), orcs[s].records(), MIX[1].fb_threshold,
                                where=f"batch stream {s} frame {t}", tally=tally)
    for o in orcs:
        o.close()
    tally.check(1)


def test_partial_staging_leaves_other_streams_alone():
    import paper_2609_30459_amd as vf
    seqs = _seqs(3)
    with vf.Frontend(_streams(), vf.params_for(MIX[1], track_waves_per_cu=2)) as fe, \
            vf.Frontend(_streams()[:1], vf.params_for(MIX[1])) as solo:
        # stream 0 steps every time, stream 2 only in the first step
        fe.stage_frame(0, 1, list(seqs[0].frames[0]))
        fe.stage_frame(2, 1, list(seqs[2].frames[0]))
        fe.step()
        r2 = fe.get_tracks(2)
        for t in range(1, 3):
            fe.stage_frame(0, t + 1, list(seqs[0].frames[t]))
            fe.step()
        for t in range(3):
            solo.push_stereo_frame(0, t + 1, list(seqs[0].frames[t]))
        assert fe.get_tracks(0).tobytes() == solo.get_tracks(0).tobytes()
        assert fe.get_tracks(2).tobytes() == r2.tobytes()
        with pytest.raises(vf.VioError):
            fe.step()  # nothing staged
        with pytest.raises(vf.VioError):
            fe.get_tracks(1)  # stream 1 never ran


def test_multi_stream_staging_call_equals_single_stagings():
    import torch

    import paper_2609_30459_amd as vf
    seqs = _seqs(3)
    devs = [torch.from_numpy(q.frames).cuda() for q in seqs]
    with vf.Frontend(_streams(), vf.params_for(MIX[1], eager=True)) as a, \
            vf.Frontend(_streams(), vf.params_for(MIX[1])) as b:
        for t in range(3):
            imgs = [devs[s][t, c] for s, w in enumerate(MIX) for c in range(w.n_cams)]
            a.stage_frames_device([0, 1, 2], [t + 1] * 3, imgs)
            a.step()
            for s, w in enumerate(MIX):
                b.stage_frame_device(s, t + 1, [devs[s][t, c] for c in range(w.n_cams)])
            b.step()
            for s in range(3):
                assert a.get_tracks(s).tobytes() == b.get_tracks(s).tobytes(), (t, s)
            assert all(m > 0 for m in a.stats()["last_stage_ms"])
            # one readback call for several streams, in any order
            for order in ([0, 1, 2], [2, 0], [1]):
                many = a.get_tracks_many(order)
                assert len(many) == len(order)
                for s, r in zip(order, many):
                    assert r.tobytes() == a.get_tracks(s).tobytes(), (t, order, s)


@pytest.mark.parametrize("stereo_mode", [0, 1])
def test_step_counts_equal_the_records(stereo_mode):
    """The per-frame counts the selection kernel reports (vio_stats) agree with
    the records: tracked, detected and matched records by status, and lost =
    the previous frame's live keypoints that were not tracked."""
    import paper_2609_30459_amd as vf
    TR, DET, MAT = vf.VIO_TRACKED, vf.VIO_DETECTED, vf.VIO_MATCHED
    seqs = _seqs(5)
    with vf.Frontend(_streams(), vf.params_for(MIX[1], stereo_mode=stereo_mode)) as fe:
        prev_live = None
        for t in range(5):
            for s, seq in enumerate(seqs):
                fe.stage_frame(s, t + 1, list(seq.frames[t]))
            fe.step()
            recs = np.concatenate([fe.get_tracks(s) for s in range(len(MIX))])
            st = fe.stats()
            n_tr = int((recs["status"] == TR).sum())
            assert st["last_tracked"] == n_tr, t
            assert st["last_detected"] == int((recs["status"] == DET).sum()), t
            assert st["last_matched"] == int((recs["status"] == MAT).sum()), t
            assert st["last_lost"] == (prev_live - n_tr if prev_live is not None else 0), t
            prev_live = int(np.isin(recs["status"], [TR, DET, MAT]).sum())


@pytest.mark.parametrize("learned", [False, True])
def test_pipelined_steps_equal_synchronous_steps(learned):
    """Frame t+1 submitted before frame t's records are read (two frames in
    flight, device images, host images staged from the second slot, a stream
    left out of some steps): every frame's records equal synchronous steps'."""
    import torch

    import paper_2609_30459_amd as vf
    n = 6
    seqs = _seqs(n)
    devs = [torch.from_numpy(q.frames).cuda() for q in seqs]
    extra = {}
    if learned:
        import os
        from paper_2609_30459_amd.train_mlp import load_weights
        params, rho, _ = load_weights(os.path.join(os.path.dirname(vf.__file__), "weights", "mlp_stereo1280.bin"))
        extra = dict(init_mode=1, learned_levels=2, learned_iters=3, learned_rho=rho)

    def staged(t):
        return [s for s in range(3) if not (s == 2 and t % 3 == 1)]  # stream 2 skips some frames

    def stage(fe, t):
        for s in staged(t):
            imgs = [devs[s][t, c] for c in range(MIX[s].n_cams)]
            if s == 0:
                fe.stage_frame(s, t + 1, [q.cpu().numpy() for q in imgs])  # host images
            else:
                fe.stage_frame_device(s, t + 1, imgs)

    with vf.Frontend(_streams(), vf.params_for(MIX[1], **extra)) as a, \
            vf.Frontend(_streams(), vf.params_for(MIX[1], **extra)) as b:
        if learned:
            a.set_mlp(params, rho)
            b.set_mlp(params, rho)
        want = []
        for t in range(n):
            stage(b, t)
            b.step()
            want.append({s: b.get_tracks(s).tobytes() for s in staged(t)})
        # three frames in flight: frame t - 2's records are read while t - 1 and t run
        got = []
        depth = 3
        for t in range(n + depth - 1):
            if t < n:
                stage(a, t)
                a.step_async()
                assert a.in_flight == min(t + 1, depth)
                if a.in_flight == depth:
                    with pytest.raises(vf.VioError):
                        a.stage_frame_device(1, 1000 + t, [devs[1][t, c] for c in range(2)])  # a fourth frame
            if t >= depth - 1:
                a.wait()
                got.append({s: a.get_tracks(s).tobytes() for s in staged(t - depth + 1)})
        assert a.in_flight == 0
        with pytest.raises(vf.VioError):
            a.wait()
        for t in range(n):
            assert got[t] == want[t], t
            assert all(len(r) > 0 for r in got[t].values())


def test_calls_during_a_frame_in_flight_wait_for_it():
    import torch

    import paper_2609_30459_amd as vf
    seqs = _seqs(3)
    devs = [torch.from_numpy(q.frames).cuda() for q in seqs]
    with vf.Frontend(_streams(), vf.params_for(MIX[1])) as a, vf.Frontend(_streams(), vf.params_for(MIX[1])) as b:
        for t in range(3):
            for fe in (a, b):
                for s in range(3):
                    fe.stage_frame_device(s, t + 1, [devs[s][t, c] for c in range(MIX[s].n_cams)])
            a.step_async()
            b.step()
            # a keypoint read drains the frame in flight
            assert a.get_keypoints(1, 0).tobytes() == b.get_keypoints(1, 0).tobytes()
            assert a.in_flight == 0
            assert a.get_tracks(1).tobytes() == b.get_tracks(1).tobytes()


def test_push_between_staging_and_step_keeps_the_staged_frame():
    """Stream 1 is staged, stream 0 is pushed on its own, then the step runs
    stream 1: its records equal a handle where nothing came in between."""
    import paper_2609_30459_amd as vf
    seqs = _seqs(3)
    with vf.Frontend(_streams(), vf.params_for(MIX[1])) as a, vf.Frontend(_streams(), vf.params_for(MIX[1])) as b:
        for t in range(3):
            a.stage_frame(1, t + 1, list(seqs[1].frames[t]))
            a.push_stereo_frame(0, t + 1, list(seqs[0].frames[t]))
            a.step()
            b.stage_frame(1, t + 1, list(seqs[1].frames[t]))
            b.step()
            b.push_stereo_frame(0, t + 1, list(seqs[0].frames[t]))
            for s in (0, 1):
                ra = a.get_tracks(s)
                assert len(ra) > 0 and ra.tobytes() == b.get_tracks(s).tobytes(), (t, s)


@pytest.mark.parametrize("learned", [False, True])
def test_pyramid_stream_choices_give_identical_records(learned):
    """The pyramid beside the tracking with a signal or an event, or in order on
    the launch stream: the same records, pipelined three frames deep."""
    import os

    import torch

    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=4, n_frames=6)
    dev = torch.from_numpy(seq.frames).cuda()
    extra = {}
    if learned:
        from paper_2609_30459_amd.train_mlp import load_weights
        params, rho, _ = load_weights(os.path.join(os.path.dirname(vf.__file__), "weights", "mlp_stereo1280.bin"))
        extra = dict(init_mode=1, learned_levels=2, learned_iters=3, learned_rho=rho, learned_fused=1,
                     track_parallel_fallback=1)
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    out = {}
    for mode in (vf.VIO_PYRAMID_SIGNAL, vf.VIO_PYRAMID_EVENT, vf.VIO_PYRAMID_SAME_STREAM):
        got = []
        with vf.Frontend([stream], vf.params_for(w, pyramid_stream=mode, **extra)) as fe:
            if learned:
                fe.set_mlp(params, rho)
            for t in range(6 + 2):
                if t < 6:
                    fe.stage_frame_device(0, t + 1, [dev[t, 0], dev[t, 1]])
                    fe.step_async()
                if t >= 2:
                    fe.wait()
                    got.append(fe.get_tracks(0).tobytes())
        out[mode] = got
    assert all(len(r) > 0 for r in out[0])
    assert out[vf.VIO_PYRAMID_EVENT] == out[vf.VIO_PYRAMID_SIGNAL]
    assert out[vf.VIO_PYRAMID_SAME_STREAM] == out[vf.VIO_PYRAMID_SIGNAL]
