"""Pins of the oracle's detection mask (the mask buffer the host uploads with
each frame, Fig. 2): a corner on a masked pixel is dropped after non-maximum
suppression, before each cell keeps its k strongest (Sec. III-D)."""
import numpy as np
import pytest

import oracle
import synthgen


def _img(w=320, h=240, seed=4):
    return synthgen.render(seed, w, h, 1, density=4.0).frames[0, 0]


def _block_mask(h, w, seed, n=12):
    r = np.random.default_rng(seed)
    m = np.zeros((h, w), np.uint8)
    for _ in range(n):
        x0, y0 = r.integers(0, w - 8), r.integers(0, h - 8)
        m[y0:y0 + r.integers(4, 60), x0:x0 + r.integers(4, 60)] = r.integers(1, 256)
    return m


@pytest.mark.parametrize("k", [1, 3])
def test_empty_and_full_masks(k):
    img = _img()
    plain = oracle.detect(img, 32, k=k)
    assert (oracle.detect(img, 32, k=k, mask=np.zeros_like(img)) == plain).all()
    full = oracle.detect(img, 32, k=k, mask=np.full_like(img, 7))
    assert (full == -1).all() and (plain[:, 0, 2] >= 0).sum() > 20


@pytest.mark.parametrize("k,seed", [(1, 0), (2, 1), (4, 2)])
def test_mask_equals_filtering_the_survivor_list(k, seed):
    """Brute force: every strict local maximum of the cell at the last
    threshold, in rank order (one pass with room for all of them), minus the
    masked ones, cut to k: the threshold walk with the mask keeps exactly these."""
    img = _img(seed=seed + 10)
    h, w = img.shape
    mask = _block_mask(h, w, seed)
    got = oracle.detect(img, 32, k=k, mask=mask)
    every = oracle.detect(img, 32, k=256, thresholds=(5,))
    assert (every[:, -1, 2] == -1).all()  # room for every survivor
    n_masked = 0
    for cell in range(got.shape[0]):
        surv = [tuple(c) for c in every[cell] if c[2] >= 0]
        keep = [c for c in surv if not mask[c[1], c[0]]][:k]
        n_masked += len(surv) - len([c for c in surv if not mask[c[1], c[0]]])
        want = np.full((k, 3), -1, np.int32)
        if keep:
            want[:len(keep)] = keep
        assert (got[cell] == want).all(), cell
    assert n_masked > 5


def test_masked_maximum_still_suppresses_its_neighbours():
    img = _img(seed=21)
    S = oracle.fast_scores(img)
    win = oracle.detect(img, 32, k=1)[:, 0]
    checked = 0
    for x, y, s in win:
        if s < 0:
            continue
        # a neighbour above the last threshold that only the winner suppresses
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                qx, qy = x + dx, y + dy
                if (dx, dy) == (0, 0) or S[qy, qx] < 5:
                    continue
                nb = S[qy - 1:qy + 2, qx - 1:qx + 2].copy()
                nb[1, 1] = -1
                nb[1 - dy, 1 - dx] = -1  # the winner's own position
                if (nb < S[qy, qx]).all():
                    mask = np.zeros_like(img)
                    mask[y, x] = 1
                    cw = oracle.detect(img, 32, k=4, mask=mask).reshape(-1, 3)
                    assert not ((cw[:, 0] == qx) & (cw[:, 1] == qy)).any()
                    checked += 1
    assert checked > 3


def test_pipeline_mask_blocks_detections_only_where_set():
    # no cap, and a mask edge on a cell edge (384 = 12 cells of 32 px)
    w = synthgen.WORKLOADS["stereo752"].with_(max_keypoints=2000)
    seq = synthgen.sequence(w, seq=2, n_frames=2)
    edge = 384
    mask = np.zeros((w.height, w.width), np.uint8)
    mask[:, :edge] = 255
    out = []
    for m in (None, mask):
        fe = oracle.Frontend([w.width] * 2, [w.height] * 2, True, oracle.params_for(w))
        try:
            if m is not None:
                fe.set_mask(0, m)
            fe.push(list(seq.frames[0]))
            out.append(fe.records())
        finally:
            fe.close()
    plain, masked = out
    det = lambda r: r[(r["status"] == oracle.DETECTED)]
    assert (det(masked)["x"] >= edge).all()
    # the unmasked cells keep the detections they had
    right = det(plain)[det(plain)["x"] >= edge]
    assert len(det(masked)) == len(right) > 50
    assert (np.sort(det(masked)["x"]) == np.sort(right["x"])).all()
