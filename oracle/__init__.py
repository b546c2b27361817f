"""CPU oracle of the stereo VIO frontend -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It wraps ``oracle.cpp``, a plain C++
statement of the frontend written from the paper (Sec. III-C to III-E) that
shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_SAN = os.environ.get("VIO_SANITIZE") == "1"
# VIO_SANITIZE=1: built with clang's AddressSanitizer and UndefinedBehaviorSanitizer instead
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SAN else "liboracle.so")
_lib = None

TRACKED, DETECTED, MATCHED, LOST_FB, LOST_OOB, LOST_DEGENERATE, LOST_CAP = range(7)

RECORD_DTYPE = np.dtype([
    ("id", "<i8"), ("x", "<f4"), ("y", "<f4"), ("theta", "<f4"), ("fb_err", "<f4"),
    ("resid_rms", "<f4"), ("age", "<i4"), ("camera", "<i2"), ("status", "<i2"), ("score", "<i4"),
])
assert RECORD_DTYPE.itemsize == 40


SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build() -> str:
    """Compile the oracle with g++ -O2 (no fast-math, no SIMD intrinsics); with VIO_SANITIZE=1, with
    ROCm's clang and the address and undefined-behaviour sanitizers (one runtime with the product
    library's sanitized host code)."""
    if _SAN:
        cmd = ["/opt/rocm/llvm/bin/clang++", "-O1", *SAN_FLAGS, "-std=c++17", "-shared", "-fPIC", "-o",
               _LIB + ".tmp", _SRC]
    else:
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("levels", ctypes.c_int32), ("gn_iters", ctypes.c_int32), ("cell_size", ctypes.c_int32),
        ("k_per_cell", ctypes.c_int32), ("n_thresholds", ctypes.c_int32),
        ("thresholds", ctypes.c_int32 * 4),
        ("edge_margin", ctypes.c_int32), ("max_keypoints", ctypes.c_int32),
        ("fb_threshold", ctypes.c_float), ("disparity0", ctypes.c_float),
        ("init_mode", ctypes.c_int32), ("learned_levels", ctypes.c_int32), ("learned_iters", ctypes.c_int32),
        ("learned_rho", ctypes.c_float), ("pred_levels", ctypes.c_int32), ("pred_iters", ctypes.c_int32),
        ("pred_rho", ctypes.c_float), ("topology", ctypes.c_int32),
        ("learned_fb_levels", ctypes.c_int32), ("learned_fb_iters", ctypes.c_int32),
        ("stereo_init", ctypes.c_int32), ("stereo_levels", ctypes.c_int32), ("stereo_iters", ctypes.c_int32),
    ]


def _lib_():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, i32, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        lib.orc_pyramid.argtypes = [vp, i32, i32, i32, vp]
        lib.orc_fast_scores.argtypes = [vp, i32, i32, vp]
        lib.orc_detect.argtypes = [vp, i32, i32, i32, i32, vp, i32, i32, i32, vp, vp]
        lib.orc_fe_set_mask.argtypes = [vp, i32, vp]
        lib.orc_track.argtypes = [vp, vp, i32, i32, i32, i32, f64, i32, vp, vp, vp, vp, vp, i32, vp, vp]
        lib.orc_klt_pass.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        lib.orc_template.argtypes = [vp, i32, i32, f64, f64, vp]
        lib.orc_pattern.argtypes = [vp, vp]
        lib.orc_se2_exp.argtypes = [f64, f64, f64, vp, vp]
        lib.orc_se2_exp.restype = None
        lib.orc_inverse3.argtypes = [vp, vp]
        lib.orc_inverse3.restype = f64
        lib.orc_fe_create.argtypes = [i32, vp, vp, i32, ctypes.POINTER(Params)]
        lib.orc_fe_create.restype = vp
        lib.orc_fe_destroy.argtypes = [vp]
        lib.orc_fe_destroy.restype = None
        lib.orc_fe_push.argtypes = [vp, vp, vp]
        lib.orc_fe_push_pred.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        lib.orc_fe_get.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_int)]
        lib.orc_fe_set_keypoints.argtypes = [vp, i32, i32, vp, vp, vp]
        lib.orc_fe_get_keypoints.argtypes = [vp, i32, i32, vp, vp, vp]
        lib.orc_fe_next_id.argtypes = [vp]
        lib.orc_fe_next_id.restype = ctypes.c_int64
        lib.orc_fe_set_mlp.argtypes = [vp, vp, i32]
        lib.orc_fe_set_motion.argtypes = [vp, i32, vp, vp, vp, f64, i32, vp, vp]
        lib.orc_motion_start.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
        lib.orc_fe_set_stereo.argtypes = [vp, i32, vp, vp, vp, vp, f64]
        lib.orc_camera_roundtrip.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        lib.orc_camera_project.argtypes = [vp, i32, vp, vp, vp]
        lib.orc_fe_last_fallback.argtypes = [vp]
        lib.orc_mlp_nparam.restype = i32
        lib.orc_bf16.argtypes = [ctypes.c_float]
        lib.orc_bf16.restype = ctypes.c_float
        lib.orc_features.argtypes = [i32, vp, vp, vp, vp, i32, i32, vp]
        lib.orc_mlp_forward.argtypes = [vp, vp, i32, i32, vp, vp, vp]
        lib.orc_mlp_loss_grad.argtypes = [vp, vp, vp, i32, i32, vp, vp]
        lib.orc_mlp_loss_grad.restype = f64
        lib.orc_adam.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float]
        lib.orc_adam.restype = None
        _lib = lib
    return _lib


def _u8(a):
    return np.ascontiguousarray(a, np.uint8)


def pyramid(img, levels):
    """List of pyramid levels (Sec. III-C eqs. 1-3)."""
    img = _u8(img)
    h, w = img.shape
    sizes = [(h >> l, w >> l) for l in range(levels)]
    out = np.zeros(sum(a * b for a, b in sizes), np.uint8)
    assert _lib_().orc_pyramid(img.ctypes.data, w, h, levels, out.ctypes.data) == 0
    res, off = [], 0
    for a, b in sizes:
        res.append(out[off:off + a * b].reshape(a, b))
        off += a * b
    return res


def fast_scores(img):
    """FAST-9 score map (Sec. III-D); INT32_MIN where undefined (3-px border)."""
    img = _u8(img)
    h, w = img.shape
    out = np.zeros((h, w), np.int32)
    assert _lib_().orc_fast_scores(img.ctypes.data, w, h, out.ctypes.data) == 0
    return out


def detect(img, cell, k=1, thresholds=(40, 20, 10, 5), margin=8, single_pass=False, mask=None):
    """Per-cell winners [n_cells, k, 3] = (x, y, score), -1 where none; mask:
    uint8 HxW, nonzero pixels hold no detection."""
    img = _u8(img)
    h, w = img.shape
    ncells = ((w + cell - 1) // cell) * ((h + cell - 1) // cell)
    thr = np.asarray(thresholds, np.int32)
    out = np.zeros((ncells, k, 3), np.int32)
    m = None if mask is None else _u8(mask)
    assert m is None or m.shape == img.shape
    assert _lib_().orc_detect(img.ctypes.data, w, h, cell, k, thr.ctypes.data, len(thr), margin,
                              int(single_pass), None if m is None else m.ctypes.data, out.ctypes.data) == 0
    return out


def track(src, dst, pts, init, levels, iters, fb_threshold=0.3, double=False, theta0=None):
    """Forward-backward tracking from the start `init` (and start rotations
    theta0, default 0); returns (xy_theta_fb_resid [n,5], status [n])."""
    src, dst = _u8(src), _u8(dst)
    h, w = src.shape
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 2)
    init = np.ascontiguousarray(init, np.float64).reshape(-1, 2)
    n = len(pts)
    px, py = np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1])
    ix, iy = np.ascontiguousarray(init[:, 0]), np.ascontiguousarray(init[:, 1])
    out = np.zeros((n, 5), np.float64)
    st = np.zeros(n, np.int32)
    th = None if theta0 is None else np.ascontiguousarray(np.broadcast_to(np.asarray(theta0, np.float64), (n,)))
    assert _lib_().orc_track(src.ctypes.data, dst.ctypes.data, w, h, levels, iters, fb_threshold, n,
                             px.ctypes.data, py.ctypes.data, ix.ctypes.data, iy.ctypes.data,
                             None if th is None else th.ctypes.data, int(double),
                             out.ctypes.data, st.ctypes.data) == 0
    return out, st


def _f64(a, n):
    a = np.ascontiguousarray(a, np.float64).reshape(-1)
    assert len(a) == n
    return a


def _cam(K):
    """A camera model in the oracle's C form: K = (fx, fy, cx, cy) is the
    pinhole model, K = (fx, fy, cx, cy, k1, k2, k3, k4) the Kannala-Brandt
    equidistant fisheye model (KB4)."""
    K = np.asarray(K, np.float64).reshape(-1)
    assert len(K) in (4, 8), "a camera model has 4 (pinhole) or 8 (KB4) values"
    out = np.zeros(9, np.float64)
    out[:4] = K[:4]
    if len(K) == 8:
        out[4] = 1.0
        out[5:] = K[4:]
    return out


def camera_roundtrip(K, pts):
    """Unprojects pixels pts [n, 2] through camera model K (see _cam) at
    inverse depth 1 and projects them again: (pixels [n, 2], points [n, 3], ok [n])."""
    K = _cam(K)
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 2)
    n = len(pts)
    x, y = np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1])
    out, rays, ok = np.zeros((n, 2)), np.zeros((n, 3)), np.zeros(n, np.int32)
    assert _lib_().orc_camera_roundtrip(K.ctypes.data, n, x.ctypes.data, y.ctypes.data, out.ctypes.data,
                                        rays.ctypes.data, ok.ctypes.data) == 0
    return out, rays, ok.astype(bool)


def camera_project(K, X):
    """Pixels of camera-frame points X [n, 3] through camera model K: (pixels [n, 2], ok [n])."""
    K = _cam(K)
    X = np.ascontiguousarray(X, np.float64).reshape(-1, 3)
    out, ok = np.zeros((len(X), 2)), np.zeros(len(X), np.int32)
    assert _lib_().orc_camera_project(K.ctypes.data, len(X), X.ctypes.data, out.ctypes.data, ok.ctypes.data) == 0
    return out, ok.astype(bool)


def motion_start(K, R, t, pts, rho, Kq=None):
    """Camera-model start of the warp (Sec. III-E) for keypoints pts [n, 2] at
    inverse depths rho [n], projected into a camera of intrinsics Kq (default
    K): (start [n, 3] = x, y, theta, ok [n])."""
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 2)
    n = len(pts)
    x, y = np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1])
    rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, np.float64), (n,)))
    out = np.zeros((n, 3), np.float64)
    ok = np.zeros(n, np.int32)
    K, R, t = _cam(K), _f64(R, 9), _f64(t, 3)
    Kq = None if Kq is None else _cam(Kq)
    assert _lib_().orc_motion_start(K.ctypes.data, R.ctypes.data, t.ctypes.data, n, x.ctypes.data, y.ctypes.data,
                                    rho.ctypes.data, out.ctypes.data, ok.ctypes.data,
                                    None if Kq is None else Kq.ctypes.data) == 0
    return out, ok.astype(bool)


def klt_pass(src, dst, pts, init, levels, iters, theta0=None):
    """One forward pass in FP64: [n, 6] = tx, ty, theta, resid, last_step, status."""
    src, dst = _u8(src), _u8(dst)
    h, w = src.shape
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 2)
    init = np.ascontiguousarray(init, np.float64).reshape(-1, 2)
    n = len(pts)
    th = np.zeros(n) if theta0 is None else np.ascontiguousarray(theta0, np.float64)
    cols = [np.ascontiguousarray(a) for a in (pts[:, 0], pts[:, 1], init[:, 0], init[:, 1], th)]
    out = np.zeros((n, 6), np.float64)
    assert _lib_().orc_klt_pass(src.ctypes.data, dst.ctypes.data, w, h, levels, iters, n,
                                *[c.ctypes.data for c in cols], out.ctypes.data) == 0
    return out


def template(img, px, py):
    img = _u8(img)
    h, w = img.shape
    out = np.zeros(20)
    _lib_().orc_template(img.ctypes.data, w, h, px, py, out.ctypes.data)
    return out[:9].reshape(3, 3), out[9:18].reshape(3, 3), bool(out[18]), bool(out[19])


def pattern():
    u = np.zeros(52, np.float32)
    v = np.zeros(52, np.float32)
    _lib_().orc_pattern(u.ctypes.data, v.ctypes.data)
    return u, v


def se2_exp(a, b, phi):
    tx, ty = ctypes.c_double(), ctypes.c_double()
    _lib_().orc_se2_exp(a, b, phi, ctypes.byref(tx), ctypes.byref(ty))
    return tx.value, ty.value


def inverse3(m):
    m = np.ascontiguousarray(m, np.float64)
    inv = np.zeros(9)
    det = _lib_().orc_inverse3(m.ctypes.data, inv.ctypes.data)
    return det, inv.reshape(3, 3)


def make_params(levels=4, gn_iters=5, cell_size=32, k_per_cell=1, thresholds=(40, 20, 10, 5),
                edge_margin=8, max_keypoints=300, fb_threshold=0.3, disparity0=32.5, init_mode=0,
                learned_levels=2, learned_iters=3, learned_rho=0.0, pred_levels=0, pred_iters=0,
                pred_rho=0.0, topology=0, learned_fb_levels=0, learned_fb_iters=0, stereo_init=0,
                stereo_levels=2, stereo_iters=3) -> Params:
    p = Params()
    p.struct_size = ctypes.sizeof(Params)
    p.levels, p.gn_iters, p.cell_size, p.k_per_cell = levels, gn_iters, cell_size, k_per_cell
    p.n_thresholds = len(thresholds)
    for i, t in enumerate(thresholds):
        p.thresholds[i] = t
    p.edge_margin, p.max_keypoints = edge_margin, max_keypoints
    p.fb_threshold, p.disparity0 = fb_threshold, disparity0
    p.init_mode, p.learned_levels, p.learned_iters, p.learned_rho = init_mode, learned_levels, learned_iters, \
        learned_rho
    p.pred_levels, p.pred_iters, p.pred_rho = pred_levels, pred_iters, pred_rho
    p.topology = topology
    p.learned_fb_levels, p.learned_fb_iters = learned_fb_levels, learned_fb_iters
    p.stereo_init, p.stereo_levels, p.stereo_iters = stereo_init, stereo_levels, stereo_iters
    return p


def params_for(workload, **overrides) -> Params:
    kw = dict(levels=workload.levels, gn_iters=workload.gn_iters, cell_size=workload.cell_size,
              k_per_cell=workload.k_per_cell, thresholds=workload.thresholds, edge_margin=workload.edge_margin,
              max_keypoints=workload.max_keypoints, fb_threshold=workload.fb_threshold,
              disparity0=workload.disparity0, topology=1 if workload.star else 0)
    kw.update(overrides)
    return make_params(**kw)


class Frontend:
    """The whole per-frame pipeline (Sec. III-B) on the CPU."""

    def __init__(self, widths, heights, stereo, params: Params):
        self.n_cams = len(widths)
        w = np.asarray(widths, np.int32)
        h = np.asarray(heights, np.int32)
        self._h = _lib_().orc_fe_create(self.n_cams, w.ctypes.data, h.ctypes.data, int(stereo),
                                        ctypes.byref(params))
        if not self._h:
            raise ValueError("oracle frontend rejected its parameters")
        self.params = params

    def close(self):
        if self._h:
            _lib_().orc_fe_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def push(self, images, predictions=None):
        """predictions: iterable of (id, camera, x, y) replacing those keypoints' initialisation."""
        imgs = [_u8(im) for im in images]
        ptrs = (ctypes.c_void_p * len(imgs))(*[im.ctypes.data for im in imgs])
        strides = np.asarray([im.shape[1] for im in imgs], np.int32)
        if predictions is None or not len(predictions):
            assert _lib_().orc_fe_push(self._h, ptrs, strides.ctypes.data) == 0
            return
        pid = np.ascontiguousarray([int(p[0]) for p in predictions], np.int64)
        pcam = np.ascontiguousarray([int(p[1]) for p in predictions], np.int32)
        pxy = np.ascontiguousarray([[float(p[2]), float(p[3])] for p in predictions], np.float32)
        assert _lib_().orc_fe_push_pred(self._h, ptrs, strides.ctypes.data, len(pid), pid.ctypes.data,
                                        pcam.ctypes.data, pxy.ctypes.data) == 0

    def set_motion(self, cam, K, R, t, rho, depths=None):
        """Camera model K (pinhole (fx, fy, cx, cy) or KB4 (fx, fy, cx, cy, k1..k4))
        and predicted motion (X_new = R X_prev + t) of camera `cam` for the next
        frame only; rho: inverse depth of keypoints without their own; depths:
        iterable of (id, inverse depth)."""
        K, R, t = _cam(K), _f64(R, 9), _f64(t, 3)
        depths = list(depths or [])
        ids = np.ascontiguousarray([int(d[0]) for d in depths], np.int64)
        rhos = np.ascontiguousarray([float(d[1]) for d in depths], np.float64)
        assert _lib_().orc_fe_set_motion(self._h, cam, K.ctypes.data, R.ctypes.data, t.ctypes.data, float(rho),
                                         len(ids), ids.ctypes.data, rhos.ctypes.data) == 0

    def set_mask(self, cam, mask):
        """Detection mask of a camera (uint8 HxW, nonzero = no detections), None to remove."""
        m = None if mask is None else _u8(mask)
        assert _lib_().orc_fe_set_mask(self._h, cam, None if m is None else m.ctypes.data) == 0

    def set_stereo(self, cam, Ks=None, Kt=None, R=None, t=None, rho=0.0):
        """Stereo extrinsics of target camera `cam` (X_target = R X + t, keypoints at
        inverse depth rho, intrinsics Ks of the detecting and Kt of the target
        camera); R None: the disparity prior again."""
        if R is None:
            assert _lib_().orc_fe_set_stereo(self._h, cam, None, None, None, None, 0.0) == 0
            return
        Ks, Kt, R, t = _cam(Ks), _cam(Kt), _f64(R, 9), _f64(t, 3)
        assert _lib_().orc_fe_set_stereo(self._h, cam, Ks.ctypes.data, Kt.ctypes.data, R.ctypes.data, t.ctypes.data,
                                         float(rho)) == 0

    def records(self):
        n = ctypes.c_int()
        _lib_().orc_fe_get(self._h, None, 0, ctypes.byref(n))
        out = np.zeros(n.value, RECORD_DTYPE)
        assert _lib_().orc_fe_get(self._h, out.ctypes.data, n.value, ctypes.byref(n)) == 0
        return out

    def set_keypoints(self, cam, ids, xy, pxy, age):
        ids = np.ascontiguousarray(ids, np.int64)
        n = len(ids)
        st = np.ascontiguousarray(np.concatenate([np.asarray(xy, np.float32).reshape(n, 2),
                                                  np.asarray(pxy, np.float32).reshape(n, 2)], 1))
        age = np.ascontiguousarray(age, np.int32)
        assert _lib_().orc_fe_set_keypoints(self._h, cam, n, ids.ctypes.data, st.ctypes.data,
                                            age.ctypes.data) == 0

    def keypoints(self, cam, capacity=1 << 16):
        ids = np.zeros(capacity, np.int64)
        st = np.zeros((capacity, 4), np.float32)
        age = np.zeros(capacity, np.int32)
        n = _lib_().orc_fe_get_keypoints(self._h, cam, capacity, ids.ctypes.data, st.ctypes.data,
                                         age.ctypes.data)
        assert n >= 0
        return ids[:n], st[:n, :2], st[:n, 2:], age[:n]

    @property
    def next_id(self):
        return _lib_().orc_fe_next_id(self._h)

    def set_mlp(self, params):
        params = np.ascontiguousarray(params, np.float32)
        assert _lib_().orc_fe_set_mlp(self._h, params.ctypes.data, len(params)) == 0

    @property
    def last_fallback(self):
        return _lib_().orc_fe_last_fallback(self._h)


# ---- learned initialisation ----------------------------------------------------
MLP_IN, MLP_HIDDEN, MLP_OUT = 32, 128, 3
MLP_NPARAM = 21123


def bf16(x):
    return np.float32(_lib_().orc_bf16(float(x)))


def features(ids, xy, pxy, age, prev_img):
    """[n, 32] features of live keypoints over the previous frame's level-0 image."""
    ids = np.ascontiguousarray(ids, np.int64)
    n = len(ids)
    st = np.ascontiguousarray(np.concatenate([np.asarray(xy, np.float32).reshape(n, 2),
                                              np.asarray(pxy, np.float32).reshape(n, 2)], 1))
    age = np.ascontiguousarray(age, np.int32)
    img = _u8(prev_img)
    out = np.zeros((n, MLP_IN), np.float32)
    _lib_().orc_features(n, ids.ctypes.data, st.ctypes.data, age.ctypes.data, img.ctypes.data, img.shape[1],
                         img.shape[0], out.ctypes.data)
    return out


def mlp_forward(params, X, exact=False):
    """(Y [n,3], H1 [n,128], H2 [n,128]); exact=True: double, no bf16 rounding."""
    params = np.ascontiguousarray(params, np.float32)
    X = np.ascontiguousarray(X, np.float32)
    n = len(X)
    Y, H1, H2 = np.zeros((n, 3)), np.zeros((n, MLP_HIDDEN)), np.zeros((n, MLP_HIDDEN))
    _lib_().orc_mlp_forward(params.ctypes.data, X.ctypes.data, n, int(exact), Y.ctypes.data, H1.ctypes.data,
                            H2.ctypes.data)
    return Y, H1, H2


def mlp_loss_grad(params, X, targets, exact=False):
    """(loss, gradient [NPARAM], dY [n,3]) of a batch."""
    params = np.ascontiguousarray(params, np.float32)
    X = np.ascontiguousarray(X, np.float32)
    T = np.ascontiguousarray(targets, np.float32)
    G = np.zeros(MLP_NPARAM)
    dY = np.zeros((len(X), 3))
    L = _lib_().orc_mlp_loss_grad(params.ctypes.data, X.ctypes.data, T.ctypes.data, len(X), int(exact),
                                  G.ctypes.data, dY.ctypes.data)
    return L, G, dY


def adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float32 arrays."""
    for a in (params, m, v):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, np.float32)
    _lib_().orc_adam(params.ctypes.data, g.ctypes.data, m.ctypes.data, v.ctypes.data, t, lr, b1, b2, eps)


def mlp_init(seed=0):
    """He-uniform weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    P = np.zeros(MLP_NPARAM, np.float32)
    o = 0
    for fan_out, fan_in in ((MLP_HIDDEN, MLP_IN), (MLP_HIDDEN, MLP_HIDDEN), (MLP_OUT, MLP_HIDDEN)):
        lim = np.sqrt(6.0 / fan_in)
        P[o:o + fan_out * fan_in] = rng.uniform(-lim, lim, fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    return P
