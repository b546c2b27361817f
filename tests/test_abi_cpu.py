"""The C-ABI library loads, exports every declared entry point and validates
arguments before touching a device (no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("vio_frontend.h", "vio_mlp.h")]


def _declared():
    names = set()
    for path in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names |= set(re.findall(r"\b(vio_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def native():
    from paper_2609_30459_amd import _native
    return _native


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("vio_frontend_create", "vio_frontend_destroy", "vio_frontend_push_stereo_frame",
                 "vio_frontend_get_tracks"):
        assert must in names


def test_library_exports_every_declared_symbol(native):
    missing = [n for n in _declared() if not hasattr(native.lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header(native):
    assert ctypes.sizeof(native.vio_stream_desc) == 20
    assert native.TRACK_DTYPE.itemsize == 40
    assert native.KEYPOINT_DTYPE.itemsize == 32
    assert ctypes.sizeof(native.vio_kp_prediction) == 24
    assert ctypes.sizeof(native.vio_pinhole) == 16
    assert ctypes.sizeof(native.vio_kb4) == 32
    assert ctypes.sizeof(native.vio_camera_motion) == 56
    assert ctypes.sizeof(native.vio_kp_depth) == 16


def test_default_params_are_the_standard_configuration():
    import paper_2609_30459_amd as vf
    p = vf.default_params()
    assert (p.levels, p.gn_iters, p.cell_size, p.k_per_cell) == (4, 5, 50, 1)
    assert list(p.thresholds)[:p.n_thresholds] == [40, 20, 10, 5]
    assert abs(p.fb_threshold - 0.3) < 1e-7 and p.edge_margin == 8


def _create(native, streams, params):
    descs = (native.vio_stream_desc * max(1, len(streams)))()
    for d, s in zip(descs, streams):
        d.n_cameras, d.width, d.height, d.max_keypoints, d.cell_size = s
    h = ctypes.c_void_p()
    rc = native.lib.vio_frontend_create(descs, len(streams), ctypes.byref(params), ctypes.byref(h))
    if rc == 0:
        native.lib.vio_frontend_destroy(h)
    return rc


def test_create_rejects_bad_arguments_before_any_device_call(native):
    import paper_2609_30459_amd as vf
    ok = (2, 752, 480, 300, 32)
    p = vf.default_params()
    bad = vf.default_params()
    bad.struct_size = 12
    assert _create(native, [ok], bad) == native.VIO_EINVAL
    for field, value in (("levels", 0), ("levels", 7), ("gn_iters", 0), ("edge_margin", 3),
                         ("n_thresholds", 0), ("fb_threshold", 0.0), ("track_block_waves", 3),
                         ("track_waves_per_cu", 65), ("flags", 8), ("pyr_tile", 48), ("stereo_mode", 2),
                         ("track_kp_per_wave", 3), ("track_kp_per_wave", -1)):
        q = vf.default_params()
        setattr(q, field, value)
        assert _create(native, [ok], q) == native.VIO_EINVAL, field
    for k in (0, 9):
        q = vf.default_params()
        q.k_per_cell = k
        assert _create(native, [ok], q) == native.VIO_EINVAL, k
    q = vf.default_params()
    q.flags = native.VIO_FLAG_EAGER | native.VIO_FLAG_PLAIN
    assert _create(native, [ok], q) == native.VIO_EINVAL
    # two keypoints per wave cannot host the fused learned stage
    q = vf.default_params()
    q.track_kp_per_wave, q.init_mode, q.learned_fused = 2, 1, 1
    assert _create(native, [ok], q) == native.VIO_EINVAL
    q.learned_fused = 0  # its own launch: the arguments pass (the device call that follows fails here)
    assert _create(native, [ok], q) != native.VIO_EINVAL
    # a device allocator needs both callbacks
    cb = native.DEV_ALLOC(lambda n, ctx: None)
    q = vf.default_params()
    q.dev_alloc = ctypes.cast(cb, ctypes.c_void_p)
    assert _create(native, [ok], q) == native.VIO_EINVAL
    # the largest grid (8192 cells) takes the largest k
    q = vf.default_params()
    q.k_per_cell = 8
    assert _create(native, [(1, 1024, 512, 300, 8)], q) != native.VIO_EINVAL
    # the threshold walk goes down
    for thr in ((20, 40), (40, 40), (40, 20, 20, 5)):
        q = vf.default_params()
        q.n_thresholds = len(thr)
        for i, t in enumerate(thr):
            q.thresholds[i] = t
        assert _create(native, [ok], q) == native.VIO_EINVAL, thr
    for s in ((3, 752, 480, 300, 32), (2, 8, 480, 300, 32), (2, 5000, 480, 300, 32), (2, 4096, 4096, 300, 32),
              (1, 64, 64, 300, 2), (1, 4000, 4000, 300, 32)):
        assert _create(native, [s], p) == native.VIO_EINVAL, s
    # coarsest level must keep at least 2x2 pixels
    q = vf.default_params()
    q.levels = 6
    assert _create(native, [(1, 40, 40, 10, 8)], q) == native.VIO_EINVAL
    assert native.lib.vio_frontend_create(None, 1, ctypes.byref(p), None) == native.VIO_EINVAL


def test_null_handle_calls_are_safe(native):
    n = ctypes.c_int32()
    assert native.lib.vio_frontend_get_tracks(None, 0, None, 0, ctypes.byref(n)) == native.VIO_EINVAL
    assert native.lib.vio_frontend_push_stereo_frame(None, 0, 0, None, None, None, 0) == native.VIO_EINVAL
    native.lib.vio_frontend_destroy(None)
    assert native.lib.vio_frontend_last_error(None) == b"null handle"


def test_sanitized_run_loads_the_sanitized_variants():
    """Under tests/sanitize.py (VIO_SANITIZE=1): the sanitizer runtime and the
    three *_san.so libraries are the ones mapped into the process."""
    if os.environ.get("VIO_SANITIZE") != "1":
        pytest.skip("not a sanitized run")
    import oracle
    import synthgen
    from paper_2609_30459_amd import _native
    oracle._lib_()
    synthgen._load()
    maps = open("/proc/self/maps").read()
    assert "libclang_rt.asan" in maps
    for name in ("liboracle_san.so", "libsynthgen_san.so", "libvio_frontend_san.so"):
        assert name in maps, name
    assert _native.LIB_PATH.endswith("libvio_frontend_san.so")
