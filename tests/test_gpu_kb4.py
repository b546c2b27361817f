"""Camera-model start through the Kannala-Brandt equidistant fisheye model
(KB4) against the CPU oracle, through the C ABI: the temporal start
(Sec. III-E, predicted pose and inverse depth through the camera model) and
the stereo extrinsics start with a fisheye target camera, and the setter's
argument checks."""
import numpy as np
import pytest

import oracle
import synthgen
from parity_util import run_pair

pytestmark = pytest.mark.gpu

TAN4 = (1 / 3, 2 / 15, 17 / 315, 62 / 2835)  # Taylor coefficients of tan: KB4 close to the pinhole model
FISH = (-0.02, 0.004, -0.001, 0.0002)         # a mild fisheye
# a KB4 model within 2 px of the rendered (pinhole) scene inside the image
NEAR = (TAN4[0] - 0.01, TAN4[1] + 0.005, TAN4[2], TAN4[3] - 0.003)
# a model whose radius polynomial folds inside the image: r = theta - 0.3 theta^3
# peaks at 0.703 (295 px at f = 420, against 446 px to a 752x480 corner), so
# the outer keypoints have no ray and keep the constant-velocity start, and
# those just inside the fold are refused for a slope below 0.05: both sides
# must draw the same line
FOLD = (-0.3, 0.0, 0.0, 0.0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_30459_amd  # noqa: F401  (raises when the library is missing)


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _kb4_motion_hook(w, seq, k, f=420.0, rho=0.4, from_frame=2):
    """Both sides: every camera a KB4 model (the synthetic camera's pinhole
    intrinsics plus coefficients k) and, from `from_frame` on, the synthetic
    motion with per-keypoint inverse depths for a third of the keypoints."""
    k = tuple(float(np.float32(v)) for v in k)

    def hook(t, fe_g, fe_o):
        K, _, _ = seq.camera_motion(max(t - 1, 0), f, rho)
        Kk = (*_f32(K), *k)
        if t == 0:
            for c in range(w.n_cams):
                fe_g.set_camera_model(0, c, Kk)
        if t < from_frame:
            return None
        _, R, tr = seq.camera_motion(t - 1, f, rho)
        R32, t32 = _f32(R), _f32(tr)
        motions, depths, out = [], [], {}
        for c in range(w.n_cams):
            ids, _, _, _ = fe_o.keypoints(c)
            r = np.random.default_rng(100 * t + c)
            own = {int(i): float(np.float32(rho * r.uniform(0.8, 1.25))) for i in ids[::3]}
            fe_o.set_motion(c, Kk, R32, t32, float(np.float32(rho)), depths=list(own.items()))
            motions.append((c, R32, t32, rho))
            depths += [(i, c, d) for i, d in own.items()]
            out[c] = (Kk, R32, t32, float(np.float32(rho)), own)
        fe_g.set_motion(0, motions, depths)
        return out

    return hook


@pytest.mark.parametrize("k", [TAN4, FISH, FOLD], ids=["tan_series", "fisheye", "fold_in_image"])
@pytest.mark.parametrize("name,frames", [("stereo752", 5), ("mono320_free", 5)])
def test_kb4_temporal_start_parity(name, frames, k):
    if name == "mono320_free":
        w = synthgen.WORKLOADS["mono320"].with_(warp_second=False, name="mono320_free")
    else:
        w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, seq=7, n_frames=frames)
    print(f"case {name} k={k} frames={frames}", flush=True)
    n_tr = 0
    for t, g, o, exc, _, _ in run_pair(w, seq, frames, before_push=_kb4_motion_hook(w, seq, k)):
        n_tr += int((o["status"] == oracle.TRACKED).sum())
        print(f"  frame {t}: {len(g)} records, statuses {np.bincount(g['status'], minlength=7).tolist()}", flush=True)
    assert n_tr > 0


def _kb4_ext_hook(w, seq, ks, kt, f=450.0, rho=0.5):
    """Stereo extrinsics from the detecting camera (pinhole when ks is None,
    else KB4 with coefficients ks) to the target cameras (pinhole when kt is
    None, else KB4 with kt), built from the synthetic disparity planes as for
    the pinhole-to-pinhole case."""
    Ks = np.array([f, f, 375.5, 239.5], np.float32)
    Kt = np.array([f, f, 371.0, 241.0], np.float32)
    ms = tuple(_f32(Ks)) + (() if ks is None else tuple(float(np.float32(v)) for v in ks))
    mt = tuple(_f32(Kt)) + (() if kt is None else tuple(float(np.float32(v)) for v in kt))
    views = seq.views
    ext = {}

    def hook(t, fe_g, fe_o):
        if t == 0:
            for c in range(w.n_cams):
                fe_g.set_camera_model(0, c, ms if c % views == 0 else mt)
            for c in range(w.n_cams):
                if c % views == 0:
                    continue
                cc = float(seq._plane(c)[2])
                tr = np.array([(Ks[2] - Kt[2] - cc) / (f * rho), (Ks[3] - Kt[3]) / (f * rho), 0.0], np.float32)
                fe_g.set_stereo_extrinsics(0, c, np.eye(3), tr, rho)
                ext[("ext", c)] = (ms, mt, np.eye(3), _f32(tr), float(np.float32(rho)))
                fe_o.set_stereo(c, *ext[("ext", c)])
        return ext  # the FP64 referee starts the matches where both sides do

    return hook


@pytest.mark.parametrize("ks,kt", [(None, TAN4), (None, NEAR), (TAN4, None), (NEAR, TAN4),
                                   pytest.param(None, FISH, marks=pytest.mark.skip(
                                       reason="the scene is rendered through pinhole cameras: a fisheye target "
                                              "model puts the starts up to about 20 px off, matches end "
                                              "unconverged after the level budget and the start's FP32 "
                                              "rounding (about 1e-4 px) is amplified past the position "
                                              "tolerance; needs a scene rendered through the fisheye model"))],
                         ids=["pinhole_to_tan", "pinhole_to_near", "tan_to_pinhole", "near_to_tan",
                              "pinhole_to_fisheye"])
@pytest.mark.parametrize("name", ["stereo752", "star752"])
def test_kb4_stereo_extrinsics_start_parity(name, ks, kt):
    """KB4 on either side of the stereo extrinsics start: the detecting
    camera's back-projection and the target camera's projection. The scene is
    rendered through pinhole cameras, so the KB4 models are chosen close to
    it."""
    w = synthgen.WORKLOADS[name]
    seq = synthgen.sequence(w, seq=4, n_frames=3)
    print(f"case {name} ks={ks} kt={kt}", flush=True)
    matched = 0
    for t, g, o, exc, _, _ in run_pair(w, seq, 3, before_push=_kb4_ext_hook(w, seq, ks, kt)):
        matched += int((o["status"] == oracle.MATCHED).sum())
    assert matched > 100


def test_kb4_arguments_and_switching_back_to_pinhole():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    K = (450.0, 450.0, 375.5, 239.5)
    with vf.Frontend([(2, w.width, w.height, 300, 32)], vf.params_for(w)) as fe:
        for bad in [(0.0, 450.0, 375.5, 239.5, *TAN4), (450.0, -1.0, 375.5, 239.5, *TAN4),
                    (*K, np.nan, 0, 0, 0), (*K, 0, np.inf, 0, 0)]:
            with pytest.raises(vf.VioError):
                fe.set_camera_model(0, 0, bad)
        with pytest.raises(vf.VioError):
            fe.set_camera_model(0, 2, (*K, *TAN4))  # camera out of range
        with pytest.raises(ValueError):
            fe.set_camera_model(0, 0, K[:3])
        fe.set_camera_model(0, 0, (*K, *FISH))
        fe.set_camera_model(0, 0, K)  # pinhole again
        fe.set_camera_model(0, 0, None)
        with pytest.raises(vf.VioError):  # a cleared model takes no motion
            fe.set_motion(0, [(0, np.eye(3), np.zeros(3), 0.5)], [])


def test_kb4_then_pinhole_matches_pinhole_only():
    """A camera switched from KB4 back to the pinhole model starts exactly as
    one that only ever had the pinhole model (bit-identical records)."""
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=3, n_frames=4)
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    with vf.Frontend([stream], vf.params_for(w)) as a, vf.Frontend([stream], vf.params_for(w)) as b:
        for t in range(4):
            K, R, tr = seq.camera_motion(max(t - 1, 0), 420.0, 0.4)
            if t == 0:
                a.set_camera_model(0, 0, (*K, *FISH))
                a.set_camera_model(0, 0, K)
                b.set_camera_model(0, 0, K)
            if t >= 2:
                for fe in (a, b):
                    fe.set_motion(0, [(0, R, tr, 0.4)], [])
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            assert a.get_tracks(0).tobytes() == b.get_tracks(0).tobytes(), t
