"""The handle's device arena from a caller's allocator (torch's caching
allocator here): the frames give the same records as with the library's own
allocation, and the arena goes back through the caller's free."""
import pytest

import synthgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_30459_amd  # noqa: F401  (raises when the library is missing)


def test_arena_from_the_torch_caching_allocator():
    import torch

    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    seq = synthgen.sequence(w, seq=5, n_frames=4)
    stream = (2, w.width, w.height, w.max_keypoints, w.cell_size)
    calls = {"alloc": [], "free": []}

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n)
        calls["alloc"].append((p, n))
        return p

    def free(p):
        calls["free"].append(p)
        torch.cuda.caching_allocator_delete(p)

    a = vf.Frontend([stream], vf.params_for(w), allocator=(alloc, free))
    with vf.Frontend([stream], vf.params_for(w)) as b:
        assert len(calls["alloc"]) == 1 and calls["alloc"][0][0] % 256 == 0
        for t in range(4):
            a.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            b.push_stereo_frame(0, t + 1, list(seq.frames[t]))
            ra = a.get_tracks(0)
            assert len(ra) > 0 and ra.tobytes() == b.get_tracks(0).tobytes(), t
    a.close()
    assert calls["free"] == [calls["alloc"][0][0]]


def test_a_failing_allocator_fails_create():
    import paper_2609_30459_amd as vf
    w = synthgen.WORKLOADS["stereo752"]
    freed = []
    with pytest.raises(vf.VioError) as e:
        vf.Frontend([(2, w.width, w.height, 300, 32)], vf.params_for(w), allocator=(lambda n: 0, freed.append))
    assert e.value.code == vf._native.VIO_ENOMEM and freed == []
