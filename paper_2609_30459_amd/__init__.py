"""MI355X (gfx950) stereo VIO frontend: Python binding of the C ABI.

The frontend of VkVIO (arXiv 2609.30459, Sec. III): image pyramid, grid FAST-9
detection with non-maximum suppression, inverse-compositional SE(2) patch
tracking with a forward-backward check, temporal tracking and stereo matching.
Every step runs in the library's HIP kernels; this module only marshals
arguments (numpy for host data, torch tensors for device memory and streams).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native as _n
from ._native import (KEYPOINT_DTYPE, TRACK_DTYPE, VIO_DETECTED, VIO_LOST_CAP, VIO_LOST_DEGENERATE,  # noqa: F401
                      VIO_LOST_FB, VIO_LOST_OOB, VIO_MATCHED, VIO_PYRAMID_EVENT, VIO_PYRAMID_SAME_STREAM,
                      VIO_PYRAMID_SIGNAL, VIO_TRACKED, VioError)

__all__ = ["Frontend", "Mlp", "default_params", "make_params", "TRACK_DTYPE", "KEYPOINT_DTYPE", "VioError"]

MLP_NPARAM = _n.VIO_MLP_NPARAM


def default_params() -> _n.vio_frontend_params:
    p = _n.vio_frontend_params()
    _n.lib.vio_frontend_default_params(ctypes.byref(p))
    return p


def make_params(levels=4, gn_iters=5, cell_size=50, k_per_cell=1, thresholds=(40, 20, 10, 5), edge_margin=8,
                max_keypoints=300, fb_threshold=0.3, disparity0=32.5, init_mode=0, learned_levels=2,
                learned_iters=3, learned_rho=0.0, eager=False, track_waves_per_cu=0,
                track_block_waves=0, pyr_tile=0, stereo_mode=0, pred_levels=0, pred_iters=0,
                pred_rho=0.0, topology=0, plain=False, learned_fb_levels=0, learned_fb_iters=0, stereo_init=0,
                stereo_levels=2, stereo_iters=3, track_parallel_fallback=0,
                learned_block_waves=0, learned_fused=0, pyramid_stream=0,
                track_kp_per_wave=0) -> _n.vio_frontend_params:
    p = default_params()
    p.levels, p.gn_iters, p.cell_size, p.k_per_cell = levels, gn_iters, cell_size, k_per_cell
    p.n_thresholds = len(thresholds)
    for i, t in enumerate(thresholds):
        p.thresholds[i] = t
    p.edge_margin, p.max_keypoints = edge_margin, max_keypoints
    p.fb_threshold, p.disparity0, p.init_mode = fb_threshold, disparity0, init_mode
    p.learned_levels, p.learned_iters, p.learned_rho = learned_levels, learned_iters, learned_rho
    p.flags = (_n.VIO_FLAG_EAGER if eager else 0) | (_n.VIO_FLAG_PLAIN if plain else 0)
    p.track_waves_per_cu = track_waves_per_cu
    p.track_block_waves = track_block_waves
    p.pyr_tile = pyr_tile
    p.stereo_mode = stereo_mode
    p.pred_levels, p.pred_iters, p.pred_rho = pred_levels, pred_iters, pred_rho
    p.topology = topology
    p.learned_fb_levels, p.learned_fb_iters = learned_fb_levels, learned_fb_iters
    p.stereo_init, p.stereo_levels, p.stereo_iters = stereo_init, stereo_levels, stereo_iters
    p.track_parallel_fallback = track_parallel_fallback
    p.learned_block_waves = learned_block_waves
    p.learned_fused = learned_fused
    p.pyramid_stream = pyramid_stream
    p.track_kp_per_wave = track_kp_per_wave
    return p


def params_for(workload, **overrides) -> _n.vio_frontend_params:
    kw = dict(levels=workload.levels, gn_iters=workload.gn_iters, cell_size=workload.cell_size,
              k_per_cell=workload.k_per_cell, thresholds=workload.thresholds, edge_margin=workload.edge_margin,
              max_keypoints=workload.max_keypoints, fb_threshold=workload.fb_threshold,
              disparity0=workload.disparity0, topology=1 if workload.star else 0)
    kw.update(overrides)
    return make_params(**kw)


def _prebuilt(images):
    """True for the (pointer array, pitch array) pair that Frontend.device_images returns."""
    return isinstance(images, tuple) and len(images) == 2 and isinstance(images[0], ctypes.Array)


class Frontend:
    """A frontend handle (vio_frontend_create .. vio_frontend_destroy).

    streams: list of (n_cameras, width, height[, max_keypoints[, cell_size]]).
    allocator: optional (alloc(nbytes) -> device pointer as int, free(pointer)),
    used for the handle's one device arena (e.g. torch's caching allocator).
    """

    def __init__(self, streams, params: _n.vio_frontend_params, allocator=None):
        descs = (_n.vio_stream_desc * len(streams))()
        for d, s in zip(descs, streams):
            s = tuple(s) + (0,) * (5 - len(s))
            d.n_cameras, d.width, d.height, d.max_keypoints, d.cell_size = s
        self.streams = [tuple(s) for s in streams]
        self._alloc_cb = None
        if allocator is not None:
            alloc, free = allocator
            params = _n.vio_frontend_params.from_buffer_copy(params)
            self._alloc_cb = (_n.DEV_ALLOC(lambda nbytes, ctx: int(alloc(int(nbytes))) or None),
                              _n.DEV_FREE(lambda ptr, ctx: free(int(ptr))))
            params.dev_alloc = ctypes.cast(self._alloc_cb[0], ctypes.c_void_p)
            params.dev_free = ctypes.cast(self._alloc_cb[1], ctypes.c_void_p)
        self.params = params
        self._rec_hint = {}  # per stream: record buffer size for get_tracks
        h = ctypes.c_void_p()
        rc = _n.lib.vio_frontend_create(descs, len(streams), ctypes.byref(params), ctypes.byref(h))
        if rc != 0:
            raise VioError(rc, "vio_frontend_create")
        self._h = h

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _n.lib.vio_frontend_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc, where):
        if rc != 0:
            raise VioError(rc, where, _n.lib.vio_frontend_last_error(self._h).decode(errors="replace"))

    # -- frames ------------------------------------------------------------
    def push_stereo_frame(self, stream, t_ns, images, predictions=None):
        """images: one uint8 HxW numpy array per camera of the stream."""
        imgs = [np.ascontiguousarray(im, np.uint8) for im in images]
        ptrs = (ctypes.c_void_p * len(imgs))(*[im.ctypes.data for im in imgs])
        strides = np.asarray([im.strides[0] for im in imgs], np.int32)
        pred_arr, n_pred = None, 0
        if predictions is not None and len(predictions):
            n_pred = len(predictions)
            pred_arr = (_n.vio_kp_prediction * n_pred)()
            for q, (pid, cam, x, y) in zip(pred_arr, predictions):
                q.id, q.camera, q.x, q.y = int(pid), int(cam), float(x), float(y)
        rc = _n.lib.vio_frontend_push_stereo_frame(self._h, stream, int(t_ns), ptrs, strides.ctypes.data,
                                                   pred_arr, n_pred)
        self._check(rc, "vio_frontend_push_stereo_frame")

    def set_detection_mask(self, stream, camera, mask):
        """Detection mask of a detecting camera (uint8 HxW, nonzero = no new keypoint), None to remove."""
        if mask is None:
            rc = _n.lib.vio_frontend_set_detection_mask(self._h, stream, camera, None, 0)
        else:
            m = np.ascontiguousarray(mask, np.uint8)
            _, w, h = self.streams[stream][:3] if 0 <= stream < len(self.streams) else (0, 0, 0)
            if w and m.shape != (h, w):
                raise ValueError(f"mask shape {m.shape}, stream images are {(h, w)}")
            rc = _n.lib.vio_frontend_set_detection_mask(self._h, stream, camera, m.ctypes.data, m.strides[0])
        self._check(rc, "vio_frontend_set_detection_mask")

    def set_stereo_extrinsics(self, stream, camera, R=None, t=None, inv_depth=1.0):
        """Stereo matches into `camera` start from the rig's extrinsics (X_camera = R X_detecting + t,
        keypoints at inverse depth inv_depth); R None: the disparity prior again."""
        if R is None:
            rc = _n.lib.vio_frontend_set_stereo_extrinsics(self._h, stream, camera, None, None, 1.0)
        else:
            r = np.ascontiguousarray(np.asarray(R, np.float32).reshape(9))
            tt = np.ascontiguousarray(np.asarray(t, np.float32).reshape(3))
            rc = _n.lib.vio_frontend_set_stereo_extrinsics(self._h, stream, camera, r.ctypes.data, tt.ctypes.data,
                                                           float(inv_depth))
        self._check(rc, "vio_frontend_set_stereo_extrinsics")

    def set_camera_model(self, stream, camera, K):
        """Camera model of a camera: pinhole K = (fx, fy, cx, cy), the KB4
        fisheye K = (fx, fy, cx, cy, k1, k2, k3, k4), or None to clear it."""
        if K is not None and len(K) == 8:
            k = _n.vio_kb4(*[float(v) for v in K[:4]], (ctypes.c_float * 4)(*[float(v) for v in K[4:]]))
            self._check(_n.lib.vio_frontend_set_camera_kb4(self._h, stream, camera, ctypes.byref(k)),
                        "vio_frontend_set_camera_kb4")
            return
        k = None
        if K is not None:
            if len(K) != 4:
                raise ValueError("a camera model has 4 (pinhole) or 8 (KB4) values")
            k = _n.vio_pinhole(*[float(v) for v in K])
        rc = _n.lib.vio_frontend_set_camera_model(self._h, stream, camera, ctypes.byref(k) if k is not None else None)
        self._check(rc, "vio_frontend_set_camera_model")

    @staticmethod
    def motion_array(motions):
        """ctypes array of vio_camera_motion from (camera, R [9 or 3x3], t [3],
        inv_depth) tuples; set_motion takes it as is (no per-call conversion)."""
        motions = list(motions)
        m = (_n.vio_camera_motion * max(1, len(motions)))()
        for q, (cam, R, t, rho) in zip(m, motions):
            q.camera, q.inv_depth = int(cam), float(rho)
            q.R[:] = [float(v) for v in np.asarray(R, np.float64).reshape(9)]
            q.t[:] = [float(v) for v in np.asarray(t, np.float64).reshape(3)]
        return m, len(motions)

    def set_motion(self, stream, motions, depths=None):
        """Camera-model start for the stream's next frame. motions: iterable of
        (camera, R [9 or 3x3], t [3], inv_depth), or the result of
        motion_array; depths: iterable of (id, camera, inv_depth)."""
        prebuilt = isinstance(motions, tuple) and len(motions) == 2 and isinstance(motions[1], int)
        m, n_m = motions if prebuilt else self.motion_array(motions)
        depths = list(depths or [])
        d = None
        if depths:
            d = (_n.vio_kp_depth * len(depths))()
            for q, (kid, cam, rho) in zip(d, depths):
                q.id, q.camera, q.inv_depth = int(kid), int(cam), float(rho)
        rc = _n.lib.vio_frontend_set_motion(self._h, stream, m, n_m, d, len(depths))
        self._check(rc, "vio_frontend_set_motion")

    def push_stereo_frame_device(self, stream, t_ns, images, hip_stream=None):
        """images: one device uint8 tensor (HxW, row-contiguous) per camera, or the
        result of device_images."""
        ptrs, pitches = images if _prebuilt(images) else self.device_images(images)
        st = None
        if hip_stream is not None:
            st = ctypes.c_void_p(int(getattr(hip_stream, "cuda_stream", hip_stream)))
        rc = _n.lib.vio_frontend_push_stereo_frame_device(self._h, stream, int(t_ns), ptrs, pitches.ctypes.data, st)
        self._check(rc, "vio_frontend_push_stereo_frame_device")

    def stage_frame(self, stream, t_ns, images):
        """Stages host images (one uint8 HxW array per camera) for the next step()."""
        imgs = [np.ascontiguousarray(im, np.uint8) for im in images]
        ptrs = (ctypes.c_void_p * len(imgs))(*[im.ctypes.data for im in imgs])
        strides = np.asarray([im.strides[0] for im in imgs], np.int32)
        self._check(_n.lib.vio_frontend_stage_frame(self._h, stream, int(t_ns), ptrs, strides.ctypes.data),
                    "vio_frontend_stage_frame")

    def stage_frame_device(self, stream, t_ns, images):
        """Stages device images (uint8 tensors, kept alive until step()) for the next step()."""
        ptrs = (ctypes.c_void_p * len(images))(*[int(t.data_ptr()) for t in images])
        pitches = np.asarray([int(t.stride(0)) * t.element_size() for t in images], np.int32)
        self._check(_n.lib.vio_frontend_stage_frame_device(self._h, stream, int(t_ns), ptrs, pitches.ctypes.data),
                    "vio_frontend_stage_frame_device")

    @staticmethod
    def device_images(images):
        """(pointer array, pitch array) of device image tensors, as stage_frames_device
        takes them; build it once per frame's images to skip the per-call conversion."""
        ptrs = (ctypes.c_void_p * len(images))(*[int(t.data_ptr()) for t in images])
        pitches = np.asarray([int(t.stride(0)) * t.element_size() for t in images], np.int32)
        return ptrs, pitches

    def stage_frames_device(self, streams, t_ns, images):
        """Stages device images of several streams in one call; images: all cameras, stream by
        stream, as tensors or as the result of device_images."""
        n = len(streams)
        st = np.ascontiguousarray(streams, np.int32)
        ts = np.ascontiguousarray(t_ns, np.int64)
        ptrs, pitches = images if _prebuilt(images) else self.device_images(images)
        self._check(_n.lib.vio_frontend_stage_frames_device(self._h, n, st.ctypes.data, ts.ctypes.data, ptrs,
                                                            pitches.ctypes.data), "vio_frontend_stage_frames_device")

    def step(self):
        """Runs every staged stream's frame in one submit (synchronous)."""
        self._check(_n.lib.vio_frontend_step(self._h), "vio_frontend_step")

    def step_async(self):
        """Submits every staged stream's frame without waiting (at most three frames in flight)."""
        self._check(_n.lib.vio_frontend_step_async(self._h), "vio_frontend_step_async")

    def wait(self):
        """Waits for the oldest frame in flight; its records are then readable."""
        self._check(_n.lib.vio_frontend_wait(self._h), "vio_frontend_wait")

    @property
    def in_flight(self) -> int:
        return _n.lib.vio_frontend_in_flight(self._h)

    def get_tracks(self, stream=0) -> np.ndarray:
        """The last frame's records of the stream (one C call while the buffer guess holds)."""
        n = ctypes.c_int32()
        cap = self._rec_hint.get(stream, 256)
        out = np.empty(cap, TRACK_DTYPE)
        rc = _n.lib.vio_frontend_get_tracks(self._h, stream, out.ctypes.data, cap, ctypes.byref(n))
        if rc == _n.VIO_ETOOSMALL:
            cap = n.value + n.value // 4
            out = np.empty(cap, TRACK_DTYPE)
            rc = _n.lib.vio_frontend_get_tracks(self._h, stream, out.ctypes.data, cap, ctypes.byref(n))
        self._check(rc, "vio_frontend_get_tracks")
        self._rec_hint[stream] = cap
        return out[:n.value]

    def get_tracks_many(self, streams) -> list:
        """The last frame's records of several streams with one C call: a list of
        arrays (views into one buffer), one per stream in the given order."""
        key = tuple(int(s) for s in streams)
        ids = np.asarray(key, np.int32)
        counts = np.zeros(len(key), np.int32)
        n = ctypes.c_int32()
        cap = self._rec_hint.get(key, 1024)
        out = np.empty(cap, TRACK_DTYPE)
        rc = _n.lib.vio_frontend_get_tracks_streams(self._h, len(key), ids.ctypes.data, out.ctypes.data, cap,
                                                    counts.ctypes.data, ctypes.byref(n))
        if rc == _n.VIO_ETOOSMALL:
            cap = n.value + n.value // 4
            out = np.empty(cap, TRACK_DTYPE)
            rc = _n.lib.vio_frontend_get_tracks_streams(self._h, len(key), ids.ctypes.data, out.ctypes.data, cap,
                                                        counts.ctypes.data, ctypes.byref(n))
        self._check(rc, "vio_frontend_get_tracks_streams")
        self._rec_hint[key] = cap
        views, at = [], 0
        for m in counts.tolist():
            views.append(out[at:at + m])
            at += m
        return views

    # -- keypoint state ----------------------------------------------------
    def set_keypoints(self, stream, camera, kps: np.ndarray):
        kps = np.ascontiguousarray(kps, KEYPOINT_DTYPE)
        rc = _n.lib.vio_frontend_set_keypoints(self._h, stream, camera, kps.ctypes.data if len(kps) else None,
                                               len(kps))
        self._check(rc, "vio_frontend_set_keypoints")

    def get_keypoints(self, stream, camera) -> np.ndarray:
        n = ctypes.c_int32()
        rc = _n.lib.vio_frontend_get_keypoints(self._h, stream, camera, None, 0, ctypes.byref(n))
        if rc not in (0, _n.VIO_ETOOSMALL):
            self._check(rc, "vio_frontend_get_keypoints")
        out = np.zeros(n.value, KEYPOINT_DTYPE)
        rc = _n.lib.vio_frontend_get_keypoints(self._h, stream, camera, out.ctypes.data, n.value, ctypes.byref(n))
        self._check(rc, "vio_frontend_get_keypoints")
        return out

    # -- diagnostics -------------------------------------------------------
    def get_pyramid(self, stream, camera, level) -> np.ndarray:
        _, w, h = self.streams[stream][:3]
        out = np.zeros((h >> level, w >> level), np.uint8)
        rc = _n.lib.vio_frontend_get_pyramid(self._h, stream, camera, level, out.ctypes.data, out.size)
        self._check(rc, "vio_frontend_get_pyramid")
        return out

    def get_cell_winners(self, stream, camera) -> np.ndarray:
        n = ctypes.c_int32()
        rc = _n.lib.vio_frontend_get_cell_winners(self._h, stream, camera, None, 0, ctypes.byref(n))
        if rc not in (0, _n.VIO_ETOOSMALL):
            self._check(rc, "vio_frontend_get_cell_winners")
        out = np.zeros((n.value, 3), np.int32)
        rc = _n.lib.vio_frontend_get_cell_winners(self._h, stream, camera, out.ctypes.data, out.size,
                                                  ctypes.byref(n))
        self._check(rc, "vio_frontend_get_cell_winners")
        return out

    def stats(self) -> dict:
        s = _n.vio_stats()
        self._check(_n.lib.vio_frontend_get_stats(self._h, ctypes.byref(s)), "vio_frontend_get_stats")
        return {"frames": s.frames, "last_gpu_ms": s.last_gpu_ms, "last_stage_ms": list(s.last_stage_ms),
                "last_learned_ms": list(s.last_learned_ms),
                "last_tracked": s.last_tracked, "last_lost": s.last_lost, "last_detected": s.last_detected,
                "last_matched": s.last_matched, "last_fallback": s.last_fallback}

    def set_mlp(self, params, rho=-1.0):
        """Installs learned-initialisation weights (VIO_MLP_NPARAM floats); rho >= 0 sets the fallback threshold."""
        p = np.ascontiguousarray(params, np.float32)
        self._check(_n.lib.vio_frontend_set_mlp(self._h, p.ctypes.data, len(p), float(rho)), "vio_frontend_set_mlp")


    def get_features(self, stream, camera) -> np.ndarray:
        """Network inputs of the camera's previous keypoints in the last frame (learned mode)."""
        n = ctypes.c_int32()
        rc = _n.lib.vio_frontend_get_features(self._h, stream, camera, None, 0, ctypes.byref(n))
        if rc not in (0, _n.VIO_ETOOSMALL):
            self._check(rc, "vio_frontend_get_features")
        out = np.zeros((n.value, 32), np.float32)
        rc = _n.lib.vio_frontend_get_features(self._h, stream, camera, out.ctypes.data, out.size, ctypes.byref(n))
        self._check(rc, "vio_frontend_get_features")
        return out


def _stream_ptr(hip_stream):
    if hip_stream is None:
        return None
    return ctypes.c_void_p(int(getattr(hip_stream, "cuda_stream", hip_stream)))


class Mlp:
    """The learned-initialisation network on the device (vio_mlp_create .. vio_mlp_destroy).

    Device data are torch tensors (float32, contiguous, on the GPU).
    """

    def __init__(self, max_batch=1024):
        h = ctypes.c_void_p()
        rc = _n.lib.vio_mlp_create(int(max_batch), ctypes.byref(h))
        if rc != 0:
            raise VioError(rc, "vio_mlp_create")
        self._h = h
        self.max_batch = max_batch

    def close(self):
        if getattr(self, "_h", None):
            _n.lib.vio_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32)
        rc = _n.lib.vio_mlp_set_params(self._h, p.ctypes.data, len(p))
        if rc != 0:
            raise VioError(rc, "vio_mlp_set_params")

    def get_params(self):
        p = np.zeros(MLP_NPARAM, np.float32)
        rc = _n.lib.vio_mlp_get_params(self._h, p.ctypes.data, len(p))
        if rc != 0:
            raise VioError(rc, "vio_mlp_get_params")
        return p

    def forward(self, x, y, hip_stream=None):
        rc = _n.lib.vio_mlp_forward(self._h, x.data_ptr(), x.shape[0], y.data_ptr(), _stream_ptr(hip_stream))
        if rc != 0:
            raise VioError(rc, "vio_mlp_forward")

    def gradient(self, x, targets, grad, hip_stream=None):
        loss = ctypes.c_float()
        rc = _n.lib.vio_mlp_gradient(self._h, x.data_ptr(), targets.data_ptr(), x.shape[0], grad.data_ptr(),
                                     ctypes.byref(loss), _stream_ptr(hip_stream))
        if rc != 0:
            raise VioError(rc, "vio_mlp_gradient")
        return loss.value

    def train_step(self, x, targets, lr=1e-3, want_loss=True, hip_stream=None):
        loss = ctypes.c_float()
        rc = _n.lib.vio_mlp_train_step(self._h, x.data_ptr(), targets.data_ptr(), x.shape[0], float(lr),
                                       ctypes.byref(loss) if want_loss else None, _stream_ptr(hip_stream))
        if rc != 0:
            raise VioError(rc, "vio_mlp_train_step")
        return loss.value if want_loss else None
