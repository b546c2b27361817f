"""Seeded synthetic stereo sequences and their ground-truth warps.

The paper measures on recorded visual-inertial datasets that are not available
here; these sequences stand in for them with the image sizes, camera counts,
motion bounds and texture statistics of the benchmark workloads (see
``workloads.py``). This package holds only scene rendering and motion: none of
the frontend's own arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .workloads import WORKLOADS, Workload, eval_seed, splitmix64  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synthgen.cpp")
_SAN = os.environ.get("VIO_SANITIZE") == "1"
# VIO_SANITIZE=1: built with clang's AddressSanitizer and UndefinedBehaviorSanitizer instead
_LIB = os.path.join(_HERE, "libsynthgen_san.so" if _SAN else "libsynthgen.so")
_lib = None


def build() -> str:
    """Compile the renderer with g++ (host code only); with VIO_SANITIZE=1, with ROCm's clang and the
    address and undefined-behaviour sanitizers."""
    if _SAN:
        cmd = ["/opt/rocm/llvm/bin/clang++", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-g", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", _LIB + ".tmp",
               _SRC]
    else:
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("n_frames", ctypes.c_int32),
        ("n_canvases", ctypes.c_int32),
        ("stereo", ctypes.c_int32),
        ("warp_second", ctypes.c_int32),
        ("density", ctypes.c_double),
        ("max_t", ctypes.c_double),
        ("max_rot_deg", ctypes.c_double),
        ("max_scale", ctypes.c_double),
        ("smooth", ctypes.c_double),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.sg_render.restype = ctypes.c_int
        lib.sg_render.argtypes = [ctypes.POINTER(_Params)] + [ctypes.c_void_p] * 4
        _lib = lib
    return _lib


class Sequence:
    """Rendered frames plus everything needed for ground truth.

    frames: uint8 [T, n_cams, H, W]; poses: float64 [T, 4] (s, phi, ox, oy);
    planes: float64 [n_canvases, 3] disparity planes; warp: (tx, ty, theta)
    of the second frame in two-frame warp mode.
    """

    def __init__(self, frames, poses, planes, warp, stereo, warp_second):
        self.frames = frames
        self.poses = poses
        self.planes = planes
        self.warp = warp
        self.stereo = stereo
        self.warp_second = warp_second

    @property
    def n_frames(self):
        return self.frames.shape[0]

    @property
    def n_cams(self):
        return self.frames.shape[1]

    @property
    def size(self):
        return self.frames.shape[3], self.frames.shape[2]

    # ---- ground truth (fp64) -------------------------------------------------
    def _centres(self):
        W, H = self.size
        return (W - 1) * 0.5, (H - 1) * 0.5, (3 * W - 1) * 0.5, (3 * H - 1) * 0.5

    def _to_canvas(self, t, x, y):
        s, phi, ox, oy = self.poses[t]
        cx, cy, Cx, Cy = self._centres()
        dx, dy = x - cx, y - cy
        c, sn = np.cos(phi), np.sin(phi)
        return Cx + s * (c * dx - sn * dy) + ox, Cy + s * (sn * dx + c * dy) + oy

    def _from_canvas(self, t, X, Y):
        s, phi, ox, oy = self.poses[t]
        cx, cy, Cx, Cy = self._centres()
        dx, dy = (X - Cx - ox) / s, (Y - Cy - oy) / s
        c, sn = np.cos(phi), np.sin(phi)
        return cx + c * dx + sn * dy, cy - sn * dx + c * dy

    @property
    def views(self):
        """Cameras per canvas: 1 mono, 2 a stereo pair, 4 a star rig."""
        return self.frames.shape[1] // self.planes.shape[0]

    def _plane(self, cam):
        v = cam % self.views
        return self.planes[cam // self.views][max(v, 1) - 1]

    def right_to_left(self, cam, x, y):
        """Reference-view position of the point seen at (x, y) by view `cam`."""
        a, b, c = self._plane(cam)
        return x + a * x + b * y + c, y

    def left_to_right(self, cam, x, y):
        """Position in view `cam` of the reference-view point (x, y)."""
        a, b, c = self._plane(cam)
        return (x - b * y - c) / (1.0 + a), y

    def gt_temporal(self, t, cam, x, y):
        """Position at frame t+1 of the scene point seen at (x, y) in frame t."""
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        if self.warp_second:
            tx, ty, th = self.warp
            cx, cy, _, _ = self._centres()
            c, s = np.cos(th), np.sin(th)
            return cx + c * (x - cx) - s * (y - cy) + tx, cy + s * (x - cx) + c * (y - cy) + ty
        right = self.views > 1 and cam % self.views != 0
        if right:
            x, y = self.right_to_left(cam, x, y)
        X, Y = self._to_canvas(t, x, y)
        x1, y1 = self._from_canvas(t + 1, X, Y)
        if right:
            x1, y1 = self.left_to_right(cam, x1, y1)
        return x1, y1

    def camera_motion(self, t, f, rho):
        """The image motion of a left (or mono) camera from frame t to t+1 as a
        pinhole camera moving over a fronto-parallel scene: intrinsics
        K = (f, f, cx, cy) at the image centre, scene at inverse depth rho, and
        the rigid motion (R, tr) with X_new = R X_prev + tr. The frame-to-frame
        map is a similarity about the centre, p' - c = sigma Rot(alpha) (p - c) + d,
        which is what a roll by alpha, a move along the axis to depth Z / sigma
        and a sideways move of d Z / (sigma f) produce (Z = 1 / rho). Returns
        (K [4], R [9] row-major, tr [3]), float64."""
        cx, cy, _, _ = self._centres()
        if self.warp_second:
            tx, ty, alpha = self.warp
            sigma, d = 1.0, np.array([tx, ty])
        else:
            s0, phi0, ox0, oy0 = self.poses[t]
            s1, phi1, ox1, oy1 = self.poses[t + 1]
            sigma, alpha = s0 / s1, phi0 - phi1
            c1, n1 = np.cos(phi1), np.sin(phi1)
            d = np.array([c1 * (ox0 - ox1) + n1 * (oy0 - oy1), -n1 * (ox0 - ox1) + c1 * (oy0 - oy1)]) / s1
        Z = 1.0 / rho
        ca, sa = np.cos(alpha), np.sin(alpha)
        R = np.array([ca, -sa, 0.0, sa, ca, 0.0, 0.0, 0.0, 1.0])
        tr = np.array([d[0] * Z / (sigma * f), d[1] * Z / (sigma * f), Z * (1.0 / sigma - 1.0)])
        return np.array([f, f, cx, cy]), R, tr

    def gt_stereo(self, cam_left, x, y, cam_target=None):
        """Position in camera cam_target (default: the next camera) of the point
        (x, y) of reference camera cam_left."""
        tgt = cam_left + 1 if cam_target is None else cam_target
        return self.left_to_right(tgt, np.asarray(x, np.float64), np.asarray(y, np.float64))


def render(seed: int, width: int, height: int, n_frames: int, n_canvases: int = 1,
           stereo: bool = False, warp_second: bool = False, density: float = 1.0,
           max_t: float = 3.0, max_rot_deg: float = 2.0, max_scale: float = 0.0,
           smooth: float = 0.8, views: int | None = None) -> Sequence:
    """views: cameras per canvas (1, 2, 4); default 2 with stereo, else 1."""
    lib = _load()
    views = views or (2 if stereo else 1)
    p = _Params(seed, width, height, n_frames, n_canvases, views - 1, int(warp_second),
                density, max_t, max_rot_deg, max_scale, smooth)
    n_cams = n_canvases * views
    frames = np.zeros((n_frames, n_cams, height, width), np.uint8)
    poses = np.zeros((n_frames, 4), np.float64)
    planes = np.zeros((n_canvases, max(1, views - 1), 3), np.float64)
    warp = np.zeros(3, np.float64)
    rc = lib.sg_render(ctypes.byref(p), frames.ctypes.data, poses.ctypes.data,
                       planes.ctypes.data, warp.ctypes.data)
    if rc != 0:
        raise ValueError("sg_render rejected its arguments")
    return Sequence(frames, poses, planes, warp, stereo, warp_second)


def sequence(workload: Workload, seq: int = 0, stream: int = 0, n_frames: int | None = None,
             seed: int | None = None) -> Sequence:
    """Render one seeded sequence of a named workload."""
    w = workload
    if seed is None:
        seed = eval_seed(w.cfg_index, seq, stream)
    return render(seed, w.width, w.height, n_frames or w.n_frames, w.n_canvases, w.stereo,
                  w.warp_second, w.density, w.max_t, w.max_rot_deg, w.max_scale, w.smooth,
                  views=4 if w.star else None)
