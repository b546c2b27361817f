"""ctypes binding of libvio_frontend.so (the C ABI in include/vio_frontend.h).

Argument marshalling only: every step of the frontend runs in the library's HIP
kernels. Importing this module raises when the library has not been built, so
nothing can silently fall back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VIO_SANITIZE=1: the variant whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer
LIB_PATH = os.path.join(_HERE, "libvio_frontend_san.so" if os.environ.get("VIO_SANITIZE") == "1"
                        else "libvio_frontend.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2609_30459_amd.build` "
        "(hipcc, gfx950) before using the frontend")

# The PyTorch wheel ships its own HIP runtime under the same soname
# (libamdhip64.so.7); whichever is loaded first serves the whole process. Load
# torch's first so that one runtime owns the GPU for both torch and this
# library (torch fails to start on a runtime other than its own), and torch
# streams and allocations are valid handles here.
try:
    import torch  # noqa: F401
except ImportError:  # the C ABI works without torch
    pass

lib = ctypes.CDLL(LIB_PATH)

VIO_OK, VIO_EINVAL, VIO_ENOMEM, VIO_EDEVICE, VIO_ETOOSMALL, VIO_ESTATE, VIO_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
ERR_NAMES = {0: "VIO_OK", -1: "VIO_EINVAL", -2: "VIO_ENOMEM", -3: "VIO_EDEVICE", -4: "VIO_ETOOSMALL",
             -5: "VIO_ESTATE", -6: "VIO_EUNSUPPORTED"}
(VIO_TRACKED, VIO_DETECTED, VIO_MATCHED, VIO_LOST_FB, VIO_LOST_OOB, VIO_LOST_DEGENERATE,
 VIO_LOST_CAP) = range(7)
VIO_INIT_CONST_VEL, VIO_INIT_LEARNED = 0, 1
VIO_MAX_LEVELS = 6
VIO_MAX_CAMERAS = 64


class vio_stream_desc(ctypes.Structure):
    _fields_ = [("n_cameras", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("max_keypoints", ctypes.c_int32), ("cell_size", ctypes.c_int32)]


class vio_frontend_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("levels", ctypes.c_int32), ("gn_iters", ctypes.c_int32),
        ("cell_size", ctypes.c_int32), ("k_per_cell", ctypes.c_int32), ("n_thresholds", ctypes.c_int32),
        ("thresholds", ctypes.c_int32 * 4), ("edge_margin", ctypes.c_int32), ("max_keypoints", ctypes.c_int32),
        ("fb_threshold", ctypes.c_float), ("disparity0", ctypes.c_float), ("init_mode", ctypes.c_int32),
        ("learned_levels", ctypes.c_int32), ("learned_iters", ctypes.c_int32), ("learned_rho", ctypes.c_float),
        ("flags", ctypes.c_uint32), ("track_waves_per_cu", ctypes.c_int32),
        ("track_block_waves", ctypes.c_int32), ("pyr_tile", ctypes.c_int32), ("stereo_mode", ctypes.c_int32),
        ("pred_levels", ctypes.c_int32), ("pred_iters", ctypes.c_int32), ("pred_rho", ctypes.c_float),
        ("topology", ctypes.c_int32),
        ("dev_alloc", ctypes.c_void_p), ("dev_free", ctypes.c_void_p), ("alloc_ctx", ctypes.c_void_p),
        ("learned_fb_levels", ctypes.c_int32), ("learned_fb_iters", ctypes.c_int32),
        ("stereo_init", ctypes.c_int32), ("stereo_levels", ctypes.c_int32), ("stereo_iters", ctypes.c_int32),
        ("track_parallel_fallback", ctypes.c_int32), ("learned_block_waves", ctypes.c_int32),
        ("learned_fused", ctypes.c_int32), ("pyramid_stream", ctypes.c_int32),
        ("track_kp_per_wave", ctypes.c_int32),
    ]

# the optional device allocator of vio_frontend_params
DEV_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DEV_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


VIO_FLAG_EAGER = 1
VIO_FLAG_PLAIN = 2
VIO_STEREO_SPECULATIVE = 0
VIO_STEREO_DEFERRED = 1
VIO_TOPOLOGY_PAIRS = 0
VIO_TOPOLOGY_STAR = 1
VIO_PYRAMID_SIGNAL, VIO_PYRAMID_EVENT, VIO_PYRAMID_SAME_STREAM = 0, 1, 2
VIO_STEREO_INIT_PRIOR = 0
VIO_STEREO_INIT_NEIGHBOUR = 1


class vio_kp_prediction(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("camera", ctypes.c_int32), ("x", ctypes.c_float), ("y", ctypes.c_float)]


class vio_pinhole(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class vio_kb4(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("k", ctypes.c_float * 4)]


class vio_camera_motion(ctypes.Structure):
    _fields_ = [("camera", ctypes.c_int32), ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("inv_depth", ctypes.c_float)]


class vio_kp_depth(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("camera", ctypes.c_int32), ("inv_depth", ctypes.c_float)]


class vio_stats(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_int64), ("last_gpu_ms", ctypes.c_double),
                ("last_stage_ms", ctypes.c_double * 3), ("last_learned_ms", ctypes.c_double * 2),
                ("last_tracked", ctypes.c_int32),
                ("last_lost", ctypes.c_int32), ("last_detected", ctypes.c_int32),
                ("last_matched", ctypes.c_int32), ("last_fallback", ctypes.c_int32)]


TRACK_DTYPE = np.dtype([
    ("id", "<i8"), ("x", "<f4"), ("y", "<f4"), ("theta", "<f4"), ("fb_err", "<f4"), ("resid_rms", "<f4"),
    ("age", "<i4"), ("camera", "<i2"), ("status", "<i2"), ("score", "<i4"),
])
KEYPOINT_DTYPE = np.dtype([("id", "<i8"), ("x", "<f4"), ("y", "<f4"), ("px", "<f4"), ("py", "<f4"),
                           ("age", "<i4"), ("reserved", "<i4")])
assert TRACK_DTYPE.itemsize == 40 and KEYPOINT_DTYPE.itemsize == 32

_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_P = ctypes.POINTER

lib.vio_frontend_default_params.argtypes = [_P(vio_frontend_params)]
lib.vio_frontend_default_params.restype = None
lib.vio_frontend_create.argtypes = [_P(vio_stream_desc), _i32, _P(vio_frontend_params), _P(_vp)]
lib.vio_frontend_destroy.argtypes = [_vp]
lib.vio_frontend_destroy.restype = None
lib.vio_frontend_push_stereo_frame.argtypes = [_vp, _i32, _i64, _vp, _vp, _vp, _i32]
lib.vio_frontend_push_stereo_frame_device.argtypes = [_vp, _i32, _i64, _vp, _vp, _vp]
lib.vio_frontend_get_tracks.argtypes = [_vp, _i32, _vp, _i32, _P(_i32)]
lib.vio_frontend_get_tracks_streams.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _P(_i32)]
lib.vio_frontend_set_keypoints.argtypes = [_vp, _i32, _i32, _vp, _i32]
lib.vio_frontend_get_keypoints.argtypes = [_vp, _i32, _i32, _vp, _i32, _P(_i32)]
lib.vio_frontend_get_pyramid.argtypes = [_vp, _i32, _i32, _i32, _vp, _sz]
lib.vio_frontend_get_cell_winners.argtypes = [_vp, _i32, _i32, _vp, _i32, _P(_i32)]
lib.vio_frontend_get_stats.argtypes = [_vp, _P(vio_stats)]
lib.vio_frontend_last_error.argtypes = [_vp]
lib.vio_frontend_last_error.restype = ctypes.c_char_p
lib.vio_frontend_set_mlp.argtypes = [_vp, _vp, _i32, ctypes.c_float]
lib.vio_frontend_stage_frame.argtypes = [_vp, _i32, _i64, _vp, _vp]
lib.vio_frontend_stage_frame_device.argtypes = [_vp, _i32, _i64, _vp, _vp]
lib.vio_frontend_step.argtypes = [_vp]
lib.vio_frontend_step_async.argtypes = [_vp]
lib.vio_frontend_wait.argtypes = [_vp]
lib.vio_frontend_in_flight.argtypes = [_vp]
lib.vio_frontend_stage_frames_device.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp]
lib.vio_frontend_get_features.argtypes = [_vp, _i32, _i32, _vp, _i32, _P(_i32)]
lib.vio_frontend_set_camera_model.argtypes = [_vp, _i32, _i32, _P(vio_pinhole)]
lib.vio_frontend_set_camera_kb4.argtypes = [_vp, _i32, _i32, _P(vio_kb4)]
lib.vio_frontend_set_detection_mask.argtypes = [_vp, _i32, _i32, _vp, _i32]
lib.vio_frontend_set_stereo_extrinsics.argtypes = [_vp, _i32, _i32, _vp, _vp, ctypes.c_float]
lib.vio_frontend_set_motion.argtypes = [_vp, _i32, _vp, _i32, _vp, _i32]
# learned-initialisation network (vio_mlp.h)
VIO_MLP_NPARAM = 21123
lib.vio_mlp_create.argtypes = [_i32, _P(_vp)]
lib.vio_mlp_destroy.argtypes = [_vp]
lib.vio_mlp_destroy.restype = None
lib.vio_mlp_set_params.argtypes = [_vp, _vp, _i32]
lib.vio_mlp_get_params.argtypes = [_vp, _vp, _i32]
lib.vio_mlp_forward.argtypes = [_vp, _vp, _i32, _vp, _vp]
lib.vio_mlp_gradient.argtypes = [_vp, _vp, _vp, _i32, _vp, _P(ctypes.c_float), _vp]
lib.vio_mlp_train_step.argtypes = [_vp, _vp, _vp, _i32, ctypes.c_float, _P(ctypes.c_float), _vp]
lib.vio_mlp_gradient_noalloc.argtypes = [_vp, _vp, _vp, _i32, _vp, _P(ctypes.c_float), _vp]
VIO_MLP_NOALLOC_MAX_ROWS = 4096
for _name in ("vio_frontend_create", "vio_frontend_push_stereo_frame", "vio_frontend_push_stereo_frame_device",
              "vio_frontend_get_tracks", "vio_frontend_set_keypoints", "vio_frontend_get_keypoints",
              "vio_frontend_get_pyramid", "vio_frontend_get_cell_winners", "vio_frontend_get_stats",
              "vio_frontend_set_mlp", "vio_frontend_get_features", "vio_frontend_stage_frame",
              "vio_frontend_stage_frame_device", "vio_frontend_step", "vio_frontend_stage_frames_device",
              "vio_mlp_create", "vio_mlp_set_params", "vio_mlp_get_params",
              "vio_mlp_forward", "vio_mlp_gradient", "vio_mlp_train_step", "vio_mlp_gradient_noalloc"):
    getattr(lib, _name).restype = ctypes.c_int


class VioError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        super().__init__(f"{where} -> {ERR_NAMES.get(code, code)} {detail}".strip())
