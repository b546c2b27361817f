"""Pins of the oracle's neighbour stereo start and the learned fallback budget
(project additions on top of the paper's stereo matching, Sec. III-B, and of
the learned initialisation).

Neighbour start: a new keypoint's match into a target camera starts at
p + (x_t - x_s, y_t - y_s) of the previous frame's nearest keypoint (by
squared distance, then id) that lived in both the detecting camera (s) and
the target camera (t); without one, at the disparity prior with the full
budget. The rule is re-derived here from the oracle's keypoint states alone
and the matches are compared with the tracker run from those starts.
"""
import numpy as np

import oracle
import synthgen


def _pairs(fe):
    ids_l, xy_l, _, _ = fe.keypoints(0)
    ids_r, xy_r, _, _ = fe.keypoints(1)
    pos = {int(i): xy_l[k] for k, i in enumerate(ids_l)}
    out = []
    for k, i in enumerate(ids_r):
        if int(i) in pos:
            xl = pos[int(i)]
            out.append((int(i), float(xl[0]), float(xl[1]), np.float32(xy_r[k][0] - xl[0]),
                        np.float32(xy_r[k][1] - xl[1])))
    return out


def test_neighbour_stereo_start_rule():
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=2, n_frames=4)
    SL, SN = 2, 3
    fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True,
                         oracle.params_for(w, stereo_init=1, stereo_levels=SL, stereo_iters=SN))
    # frame 0: no previous frame, so every match starts at the disparity prior
    # with the full budget (4 levels x 5)
    fe.push(list(seq.frames[0]))
    rec = fe.records()
    det = rec[(rec["camera"] == 0) & (rec["status"] == oracle.DETECTED)]
    mat = rec[rec["camera"] == 1]
    pts = np.stack([det["x"], det["y"]], 1).astype(np.float64)
    r0, s0 = oracle.track(seq.frames[0, 0], seq.frames[0, 1], pts, pts - [w.disparity0, 0], w.levels, w.gn_iters)
    assert (mat["id"] == det["id"]).all()
    assert (np.where(s0 == 0, oracle.MATCHED, s0) == mat["status"]).all()
    checked = 0
    for t in range(1, 4):
        # drop two thirds of the left camera's keypoints, so that the frame
        # detects many new ones in the freed cells
        ids, xy, pxy, age = fe.keypoints(0)
        fe.set_keypoints(0, ids[::3], xy[::3], pxy[::3], age[::3])
        # and the right camera's keypoints without a left partner (room for the matches)
        rid, rxy, rpxy, rage = fe.keypoints(1)
        keep = np.isin(rid, ids[::3])
        fe.set_keypoints(1, rid[keep], rxy[keep], rpxy[keep], rage[keep])
        pairs = _pairs(fe)
        assert len(pairs) > 50
        fe.push(list(seq.frames[t]))
        rec = fe.records()
        det = rec[(rec["camera"] == 0) & (rec["status"] == oracle.DETECTED)]
        mat = rec[(rec["camera"] == 1) & (rec["age"] == 0)]
        assert (mat["id"] == det["id"]).all()
        starts = []
        for x, y in zip(det["x"], det["y"]):
            d = [((float(px) - float(x)) ** 2 + (float(py) - float(y)) ** 2, pid, dx, dy)
                 for pid, px, py, dx, dy in pairs]
            _, _, dx, dy = min(d)
            starts.append((np.float32(np.float32(x) + dx), np.float32(np.float32(y) + dy)))
        pts = np.stack([det["x"], det["y"]], 1).astype(np.float64)
        r, st = oracle.track(seq.frames[t, 0], seq.frames[t, 1], pts, np.array(starts, np.float64), SL, SN)
        want = np.where(st == 0, oracle.MATCHED, st)
        # (the right camera has room for every match: no LOST_CAP)
        assert (mat["status"] == want).all(), t
        ok = st == 0
        assert (mat["x"][ok] == r[ok, 0].astype(np.float32)).all() and (mat["y"][ok] == r[ok, 1].astype(np.float32)).all()
        checked += len(det)
    assert checked > 300
    fe.close()


def test_neighbour_stereo_start_off_is_the_disparity_prior():
    """stereo_init = 0 (the default) gives exactly the records of the plain
    frontend; with the neighbour start the short budget matches at least as
    many new keypoints as the disparity prior with the full budget on these
    sequences (the prior is 27.5 px off at the disparity range's ends)."""
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=3, n_frames=5)
    out = {}
    for name, kw in (("plain", {}), ("explicit_off", dict(stereo_init=0)),
                     ("neighbour", dict(stereo_init=1, stereo_levels=2, stereo_iters=3))):
        fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w, **kw))
        matched, recs = 0, []
        for t in range(5):
            fe.push(list(seq.frames[t]))
            r = fe.records()
            recs.append(r.tobytes())
            if t > 0:
                matched += int(((r["camera"] == 1) & (r["status"] == oracle.MATCHED) & (r["age"] == 0)).sum())
        out[name] = (recs, matched)
        fe.close()
    assert out["plain"][0] == out["explicit_off"][0]
    assert out["neighbour"][1] >= out["plain"][1] > 0


def test_learned_fallback_budget():
    """rho < 0 sends every learned track to the fallback: with a fallback
    budget equal to the full one the records are the plain frontend's; with a
    2 x 5 budget each temporal track is the tracker's result from the
    constant-velocity start with that budget."""
    w = synthgen.WORKLOADS["mono320"]
    seq = synthgen.sequence(w)
    P = np.zeros(oracle.MLP_NPARAM, np.float32)
    recs = {}
    for name, kw in (("plain", dict(init_mode=0)),
                     ("fb_full", dict(init_mode=1, learned_rho=-1.0, learned_fb_levels=w.levels,
                                      learned_fb_iters=w.gn_iters)),
                     ("fb_2x5", dict(init_mode=1, learned_rho=-1.0, learned_fb_levels=2, learned_fb_iters=5))):
        fe = oracle.Frontend([w.width], [w.height], False, oracle.params_for(w, **kw))
        if kw["init_mode"]:
            fe.set_mlp(P)
        fe.push([seq.frames[0, 0]])
        ids, xy, pxy, age = fe.keypoints(0)
        fe.push([seq.frames[1, 0]])
        recs[name] = (fe.records(), fe.last_fallback, xy)
        fe.close()
    assert recs["plain"][0].tobytes() == recs["fb_full"][0].tobytes()
    r, n_fb, xy = recs["fb_2x5"]
    assert n_fb == len(xy)
    want, st = oracle.track(seq.frames[0, 0], seq.frames[1, 0], xy, xy, 2, 5)  # age 0: CV start = p
    temporal = r[: len(xy)]
    assert (temporal["status"] == st).all()
    ok = st == oracle.TRACKED
    assert ok.sum() > 0.9 * len(xy)
    assert (temporal["x"][ok] == want[ok, 0].astype(np.float32)).all()
