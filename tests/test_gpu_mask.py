"""Detection mask (the host's mask buffer, Fig. 2) against the CPU oracle,
through the C ABI: cell winners bit-exact, pipeline records."""
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


def _block_mask(h, w, seed, n=16):
    r = np.random.default_rng(seed)
    m = np.zeros((h, w), np.uint8)
    for _ in range(n):
        x0, y0 = r.integers(0, w - 8), r.integers(0, h - 8)
        m[y0:y0 + r.integers(4, 90), x0:x0 + r.integers(4, 90)] = r.integers(1, 256)
    return m


@pytest.mark.parametrize("tile", [64, 32])
@pytest.mark.parametrize("name,w,h,levels,cell,k", [("stereo752_k1", 752, 480, 4, 32, 1),
                                                      ("ragged135x97_k3", 135, 97, 3, 16, 3),
                                                      ("rig1920x1200_k2", 1920, 1200, 5, 32, 2)])
def test_masked_cell_winners_bit_exact(name, w, h, levels, cell, k, tile):
    import paper_2609_30459_amd as vf
    img = synthgen.render(13, w, h, 1, density=4.0).frames[0, 0]
    mask = _block_mask(h, w, 3)
    print(f"case {name} tile {tile}", flush=True)
    params = vf.make_params(levels=levels, cell_size=cell, k_per_cell=k, pyr_tile=tile)
    with vf.Frontend([(1, w, h, 50, cell)], params) as fe:
        fe.set_detection_mask(0, 0, mask)
        fe.push_stereo_frame(0, 1, [img])
        got = fe.get_cell_winners(0, 0)
        fe.set_detection_mask(0, 0, None)
        fe.push_stereo_frame(0, 2, [img])
        unmasked = fe.get_cell_winners(0, 0)
    ref = oracle.detect(img, cell, k=k, mask=mask).reshape(-1, 3)
    assert (got == ref).all(), f"{(got != ref).any(1).sum()} slots differ"
    assert (unmasked == oracle.detect(img, cell, k=k).reshape(-1, 3)).all()
    assert (got != unmasked).any()


def test_masked_pipeline_parity():
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=4, n_frames=5)
    mask = _block_mask(w.height, w.width, 8, n=10)

    def hook(t, fe_g, fe_o):
        if t == 0:
            fe_g.set_detection_mask(0, 0, mask)
            fe_o.set_mask(0, mask)
        return None

    n_det = 0
    for t, g, o, exc, _, _ in run_pair(w, seq, 5, before_push=hook):
        assert len(exc) <= 1, (t, exc)
        d = o[o["status"] == oracle.DETECTED]
        n_det += len(d)
        assert not mask[d["y"].astype(int), d["x"].astype(int)].any()
    assert n_det > 100


def test_mask_arguments():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    with vf.Frontend([(2, w.width, w.height, 300, 32)], vf.params_for(w)) as fe:
        m = np.zeros((w.height, w.width), np.uint8)
        with pytest.raises(vf.VioError):
            fe.set_detection_mask(0, 1, m)  # the right camera does not detect
        with pytest.raises(vf.VioError):
            fe.set_detection_mask(1, 0, m)  # no such stream
        with pytest.raises(ValueError):
            fe.set_detection_mask(0, 0, m[:, :-1])
        fe.set_detection_mask(0, 0, m)
        fe.set_detection_mask(0, 0, None)
