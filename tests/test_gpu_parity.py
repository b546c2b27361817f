"""GPU library against the CPU oracle, through the C ABI.

Pyramid and detector: bit-exact. Tracks: identical tracked/lost sets (FP32 ties
within 1e-3 of the forward-backward threshold are reported) and positions
within 1e-3 px. Sizes span several 64-px tiles with ragged tails, up to the
four-camera 1920x1200 rig.
"""
import numpy as np
import pytest

import oracle
import synthgen
from parity_util import Tally, compare_records, inject, oracle_state, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_30459_amd  # noqa: F401  (raises when the library is missing)


def _vf():
    import paper_2609_30459_amd as vf
    return vf


# (name, width, height, levels, cell, density)
PYR_CASES = [
    ("mono320", 320, 240, 3, 16, 1.0),
    ("stereo752", 752, 480, 4, 32, 4.0),
    ("ragged135x97", 135, 97, 3, 16, 4.0),
    ("odd101x67_L2", 101, 67, 2, 8, 4.0),
    ("tiny40x30_L1", 40, 30, 1, 8, 4.0),
    ("hd1280", 1280, 720, 4, 48, 4.0),
    ("rig1920x1200_L5", 1920, 1200, 5, 32, 4.0),
    ("wide2000x70_L6", 2000, 140, 6, 20, 4.0),
    ("min16x16_L1", 16, 16, 1, 8, 4.0),
]


def _image(w, h, density, seed=5):
    return synthgen.render(seed, w, h, 1, density=density).frames[0, 0]


@pytest.mark.parametrize("tile", [64, 32])
@pytest.mark.parametrize("name,w,h,levels,cell,density", PYR_CASES, ids=[c[0] for c in PYR_CASES])
def test_pyramid_and_cell_winners_bit_exact(name, w, h, levels, cell, density, tile):
    vf = _vf()
    img = _image(w, h, density)
    print(f"case {name} {w}x{h} L={levels} tile {tile}", flush=True)
    with vf.Frontend([(1, w, h, 50, cell)], vf.make_params(levels=levels, cell_size=cell, pyr_tile=tile)) as fe:
        fe.push_stereo_frame(0, 1, [img])
        want = oracle.pyramid(img, levels)
        for l in range(levels):
            got = fe.get_pyramid(0, 0, l)
            assert got.shape == want[l].shape
            assert (got == want[l]).all(), f"level {l}: {(got != want[l]).sum()} pixels differ"
        win = fe.get_cell_winners(0, 0)
        ref = oracle.detect(img, cell)[:, 0]
        assert (win == ref).all(), f"{(win != ref).any(1).sum()} cells differ"
        assert (ref[:, 2] >= 0).sum() > 0 or w < 64


def test_largest_image_winners_and_pyramid_bit_exact():
    """The largest image the boundary takes (width * height < 2^24: 4096 x 4095),
    six levels, 64-px cells (4096 cells): a rendered 1024 x 1024 texture tiled
    with flips, so the tiles' seams are textured too."""
    vf = _vf()
    base = _image(1024, 1024, 4.0, seed=17)
    row = np.concatenate([base, base[:, ::-1], base, base[:, ::-1]], 1)
    img = np.ascontiguousarray(np.concatenate([row, row[::-1], row, row[::-1]], 0)[:4095])
    w, h, L, cell = 4096, 4095, 6, 64
    print(f"case max {w}x{h} L={L}", flush=True)
    with vf.Frontend([(1, w, h, 2000, cell)], vf.make_params(levels=L, cell_size=cell, max_keypoints=2000)) as fe:
        fe.push_stereo_frame(0, 1, [img])
        want = oracle.pyramid(img, L)
        for l in range(L):
            assert (fe.get_pyramid(0, 0, l) == want[l]).all(), l
        win = fe.get_cell_winners(0, 0)
        rec = fe.get_tracks(0)
    ref = oracle.detect(img, cell)[:, 0]
    assert (win == ref).all(), f"{(win != ref).any(1).sum()} cells differ"
    assert (rec["status"] == oracle.DETECTED).sum() == min(2000, (ref[:, 2] >= 0).sum())


@pytest.mark.parametrize("value", [0, 128, 255])
def test_uniform_images_give_no_keypoints(value):
    """A uniform image has no corner (every FAST difference is 0), so nothing
    is detected, matched or tracked, on every frame."""
    vf = _vf()
    w = synthgen.WORKLOADS["stereo752"]
    img = np.full((w.height, w.width), value, np.uint8)
    with vf.Frontend([(2, w.width, w.height, 300, 32)], vf.params_for(w)) as fe:
        for t in range(3):
            fe.push_stereo_frame(0, t + 1, [img, img])
            assert len(fe.get_tracks(0)) == 0
            assert (fe.get_cell_winners(0, 0) == -1).all()
    assert (oracle.detect(img, 32) == -1).all()


def test_device_push_with_unaligned_pitch_matches_oracle():
    """Level 0 read from a caller tensor whose pitch is not a multiple of 4."""
    import torch
    vf = _vf()
    w, h, L, cell = 333, 211, 4, 24
    img = _image(w, h, 4.0, seed=9)
    wide = torch.zeros((h, w + 3), dtype=torch.uint8, device="cuda")
    wide[:, :w] = torch.from_numpy(img).cuda()
    view = wide[:, :w]
    with vf.Frontend([(1, w, h, 50, cell)], vf.make_params(levels=L, cell_size=cell)) as fe:
        fe.push_stereo_frame_device(0, 1, [view])
        want = oracle.pyramid(img, L)
        for l in range(L):
            assert (fe.get_pyramid(0, 0, l) == want[l]).all(), l
        assert (fe.get_cell_winners(0, 0) == oracle.detect(img, cell)[:, 0]).all()


@pytest.mark.parametrize("name,frames", [("mono320", 2), ("stereo752", 8), ("stereo1280", 4), ("rig4", 3)])
def test_pipeline_parity_with_state_injection(name, frames):
    w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, n_frames=frames)
    print(f"case {name} frames={frames}", flush=True)
    n_tracked = 0
    for t, g, o, exc, _, _ in run_pair(w, seq, frames):
        n_tracked += int((o["status"] == oracle.TRACKED).sum())
        print(f"  frame {t}: {len(g)} records, statuses {np.bincount(g['status'], minlength=7).tolist()}", flush=True)
    assert n_tracked > 0 or frames < 2


@pytest.mark.xfail(strict=False, reason=(
    "known deviation, kept in view: keypoint 90 of this sequence turns by 0.33 rad along a near-singular "
    "direction of its Gauss-Newton system; the GPU track lands 3.2e-4 rad from the FP64 track where the FP32 "
    "oracle lands 1.8e-5 rad away, outside the referee's bar. Along a direction this weak the two FP32 "
    "evaluation orders differ by about the FP32 epsilon over the eigenvalue ratio, and which side lands nearer "
    "FP64 depends on rounding (accurate reciprocal and sine/cosine move such failures to other seeds)"))
def test_free_motion_three_levels_near_singular_seed():
    """mono320 in free motion (L = 3), sequence 12: oracle parity on a seed with
    a near-singular track; expected to fail at the position bar until the
    referee scales its allowance with the conditioning."""
    w = synthgen.WORKLOADS["mono320"].with_(warp_second=False, name="mono320_free")
    seq = synthgen.sequence(w, seq=12, n_frames=5)
    print("case mono320_free seq 12", flush=True)
    for t, g, o, exc, _, _ in run_pair(w, seq, 5):
        pass


@pytest.mark.parametrize("name,frames", [("stereo752", 6), ("rig4", 3)])
def test_lite_preset_pipeline_parity(name, frames):
    """The paper's lite preset (Sec. IV-D, Table IV): FAST thresholds down to 20,
    cells of 82 px, 3 Gauss-Newton iterations per level."""
    w = synthgen.WORKLOADS[name].with_(thresholds=(40, 20), cell_size=82, gn_iters=3)
    seq = synthgen.sequence(w, seq=5, n_frames=frames)
    print(f"case {name} lite frames={frames}", flush=True)
    n_tracked = 0
    for t, g, o, exc, _, _ in run_pair(w, seq, frames):
        n_tracked += int((o["status"] == oracle.TRACKED).sum())
        print(f"  frame {t}: {len(g)} records, statuses {np.bincount(g['status'], minlength=7).tolist()}", flush=True)
    assert n_tracked > 0


def test_free_running_stereo_matches_oracle():
    """No state injection: the two pipelines stay in lockstep frame after frame."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=1, n_frames=12)
    for t, g, o, exc, _, _ in run_pair(w, seq, 12, inject_state=False):
        assert not exc, (t, exc)


def test_free_running_deferred_stereo_matches_oracle():
    """Deferred stereo matching (selection first, then only the selected
    detections are matched) keeps lockstep with the oracle."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=1, n_frames=8)
    for t, g, o, exc, _, _ in run_pair(w, seq, 8, inject_state=False, launch={"stereo_mode": 1}):
        assert not exc, (t, exc)


@pytest.mark.parametrize("eager", [False, True])
@pytest.mark.parametrize("name,n_cams", [("stereo", 2), ("two_pairs", 4)])
def test_deferred_stereo_equals_speculative_bitwise(name, n_cams, eager):
    vf = _vf()
    w = synthgen.WORKLOADS["stereo752"].with_(n_canvases=n_cams // 2)
    seq = synthgen.sequence(w, seq=9, n_frames=6)
    stream = (n_cams, w.width, w.height, w.max_keypoints, w.cell_size)
    matched = 0
    with vf.Frontend([stream], vf.params_for(w, eager=eager)) as a, \
            vf.Frontend([stream], vf.params_for(w, eager=eager, stereo_mode=1)) as b:
        for t in range(6):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            ra, rb = a.get_tracks(0), b.get_tracks(0)
            matched += int((ra["status"] == vf.VIO_MATCHED).sum())
            assert len(ra) > 0 and ra.tobytes() == rb.tobytes(), t
            if eager:
                assert all(m > 0 for m in b.stats()["last_stage_ms"])
    assert matched > 0


def test_device_push_equals_host_push_bitwise():
    import torch
    vf = _vf()
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=2, n_frames=5)
    dev = torch.from_numpy(seq.frames).cuda()
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    with vf.Frontend([stream], vf.params_for(w)) as a, vf.Frontend([stream], vf.params_for(w)) as b:
        for t in range(5):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame_device(0, t + 1, [dev[t, 0], dev[t, 1]])
            ra, rb = a.get_tracks(0), b.get_tracks(0)
            assert ra.tobytes() == rb.tobytes(), t


def test_device_push_on_a_caller_stream_waits_for_its_images():
    """Images written on the caller's stream right before the push (a copy
    into a reused buffer), then read by the frontend on that stream: the
    pyramid, on its own stream, starts after the caller's work."""
    import torch
    vf = _vf()
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=3, n_frames=5)
    src = torch.from_numpy(seq.frames).cuda()
    buf = torch.empty_like(src[0])
    torch.cuda.synchronize()
    cs = torch.cuda.Stream()  # default priority
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    with vf.Frontend([stream], vf.params_for(w)) as a, vf.Frontend([stream], vf.params_for(w)) as b:
        for t in range(5):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            with torch.cuda.stream(cs):
                buf.copy_(src[t])
            b.push_stereo_frame_device(0, t + 1, [buf[0], buf[1]], hip_stream=cs)
            ra, rb = a.get_tracks(0), b.get_tracks(0)
            assert len(ra) > 0 and ra.tobytes() == rb.tobytes(), t


def test_runs_are_deterministic():
    vf = _vf()
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=3, n_frames=4)
    outs = []
    for _ in range(2):
        with vf.Frontend([(2, w.width, w.height, w.max_keypoints, w.cell_size)], vf.params_for(w)) as fe:
            recs = []
            for t in range(4):
                fe.push_stereo_frame(0, t + 1, list(seq.frames[t]))
                recs.append(fe.get_tracks(0).tobytes())
            outs.append(recs)
    assert outs[0] == outs[1]


def test_black_frame_loses_tracks_then_refills():
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=4, n_frames=3)
    frames = seq.frames.copy()
    frames[1] = 0  # all-black frame: every patch is degenerate or has zero mean
    for t, g, o, exc, fe_g, _ in run_pair(w, synthgen.Sequence(frames, seq.poses, seq.planes, seq.warp, True, False),
                                          3):
        if t == 1:
            assert len(g) and not np.isin(g["status"], [oracle.TRACKED, oracle.DETECTED, oracle.MATCHED]).any()
        if t == 2:
            assert (g["status"] == oracle.DETECTED).sum() > 100


def test_small_cap_and_predictions():
    vf = _vf()
    w = synthgen.WORKLOADS["stereo752"].with_(max_keypoints=40)
    seq = synthgen.sequence(w, seq=5, n_frames=3)
    fe_o = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w))
    tally = Tally("stereo752 cap 40 with predictions, 3 frames")
    with vf.Frontend([(2, w.width, w.height, 40, w.cell_size)], vf.params_for(w)) as fe_g:
        for t in range(3):
            preds = []
            if t > 0:
                inject(fe_g, fe_o, 0, 2)
                st = oracle_state(fe_o, 0)
                gx, gy = seq.gt_temporal(t - 1, 0, st["x"], st["y"])
                # predict half of the left keypoints at their true new position
                preds = [(int(i), 0, float(x), float(y)) for i, x, y in zip(st["id"][::2], gx[::2], gy[::2])]
            fe_o.push(list(seq.frames[t]), preds)
            fe_g.push_stereo_frame(0, t + 1, list(seq.frames[t]), preds)
            g, o = fe_g.get_tracks(0), fe_o.records()
            compare_records(g, o, w.fb_threshold, where=f"cap40 frame {t}", tally=tally)
            for c in range(2):
                assert len(fe_g.get_keypoints(0, c)) <= 40
    fe_o.close()
    tally.check(1)


def test_abi_errors_on_device():
    vf = _vf()
    from paper_2609_30459_amd import _native as n
    w = synthgen.WORKLOADS["mono320"]
    seq = synthgen.sequence(w)
    with vf.Frontend([(1, 320, 240, 200, 16)], vf.params_for(w)) as fe:
        with pytest.raises(vf.VioError) as e:
            fe.get_tracks(0)
        assert e.value.code == n.VIO_ESTATE
        fe.push_stereo_frame(0, 10, [seq.frames[0, 0]])
        with pytest.raises(vf.VioError) as e:
            fe.push_stereo_frame(0, 10, [seq.frames[1, 0]])  # timestamp not increasing
        assert e.value.code == n.VIO_ESTATE
        with pytest.raises(vf.VioError) as e:
            fe.push_stereo_frame(1, 11, [seq.frames[1, 0]])
        assert e.value.code == n.VIO_EINVAL
        kp = np.zeros(3, vf.KEYPOINT_DTYPE)
        kp["id"] = [5, 4, 6]
        with pytest.raises(vf.VioError) as e:
            fe.set_keypoints(0, 0, kp)  # ids must ascend
        assert e.value.code == n.VIO_EINVAL
        # the handle is still usable after rejected calls
        fe.push_stereo_frame(0, 11, [seq.frames[1, 0]])
        assert len(fe.get_tracks(0)) > 0


def test_graph_replay_equals_eager_launches():
    """The captured per-frame graph and one-by-one launches give identical
    records; eager launches report each kernel's duration."""
    vf = _vf()
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=6, n_frames=5)
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    with vf.Frontend([stream], vf.params_for(w)) as a, vf.Frontend([stream], vf.params_for(w, eager=True)) as b, \
            vf.Frontend([stream], vf.params_for(w, plain=True)) as c:
        for t in range(5):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            c.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            ra, rb = a.get_tracks(0), b.get_tracks(0)
            assert len(ra) > 0 and ra.tobytes() == rb.tobytes(), t
            assert ra.tobytes() == c.get_tracks(0).tobytes(), t  # plain launches, no timing
            assert c.stats()["last_stage_ms"] == [-1.0] * 3
            sa, sb = a.stats(), b.stats()
            assert sa["last_stage_ms"] == [-1.0] * 3 and sa["last_gpu_ms"] > 0
            assert all(m > 0 for m in sb["last_stage_ms"]), sb
            assert sb["last_learned_ms"] == [-1.0] * 2
            # kernel durations lie inside the frame's interval
            assert sum(sb["last_stage_ms"]) <= sb["last_gpu_ms"] * 1.001 + 1e-3
