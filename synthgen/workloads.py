"""Named benchmark workloads: scene recipe plus frontend parameters.

Five workloads, from a two-frame mono check to a four-camera rig:

* ``mono320``    one 320x240 camera, two frames, the second a bilinear SE(2)
                 warp of the first; 3 levels, 16-px cells, <=200 keypoints.
* ``stereo752``  752x480 stereo, 200 frames, 4x texture density, smooth
                 SE(2)+scale motion, planar disparity 5..60 px; 4 levels,
                 32-px cells, <=300 keypoints per camera.
* ``stereo1280`` 1280x720 stereo, same motion; 48-px cells. The learned
                 initialisation is evaluated here.
* ``batch16``    sixteen independent streams of uneven size.
* ``rig4``       four 1920x1200 cameras (two stereo pairs), 5 levels, fast
                 motion, 1500 keypoints per camera.

The frontend thresholds follow the paper's standard configuration: FAST
thresholds 40, 20, 10, 5 with one keypoint per cell, 5 Gauss-Newton
iterations per level, forward-backward threshold 0.3 px.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One SplitMix64 output for state x (Steele, Lea & Flood; public domain)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def eval_seed(cfg: int, seq: int, stream: int) -> int:
    return splitmix64(0x56B10000 + 1000 * cfg + 16 * seq + stream)


def train_seed(seq: int, stream: int = 0) -> int:
    return splitmix64(0x7EA10000 + 16 * seq + stream)


@dataclass(frozen=True)
class Workload:
    name: str
    cfg_index: int
    width: int
    height: int
    n_canvases: int = 1
    stereo: bool = False
    star: bool = False      # four cameras per canvas: detection in the first, matched into the other three
    n_frames: int = 200
    warp_second: bool = False
    density: float = 4.0
    max_t: float = 3.0
    max_rot_deg: float = 2.0
    max_scale: float = 0.01
    smooth: float = 0.8
    # frontend parameters
    levels: int = 4
    gn_iters: int = 5
    cell_size: int = 32
    k_per_cell: int = 1
    max_keypoints: int = 300
    fb_threshold: float = 0.3
    thresholds: tuple = (40, 20, 10, 5)
    edge_margin: int = 8
    disparity0: float = 32.5
    extra: dict = field(default_factory=dict)

    @property
    def n_cams(self) -> int:
        return self.n_canvases * (4 if self.star else 2 if self.stereo else 1)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


WORKLOADS = {
    "mono320": Workload("mono320", 0, 320, 240, n_frames=2, warp_second=True, density=1.0,
                        max_scale=0.0, levels=3, cell_size=16, max_keypoints=200),
    "stereo752": Workload("stereo752", 1, 752, 480, stereo=True),
    "stereo1280": Workload("stereo1280", 2, 1280, 720, stereo=True, cell_size=48),
    "star752": Workload("star752", 5, 752, 480, stereo=True, star=True),
    "rig4": Workload("rig4", 4, 1920, 1200, n_canvases=2, stereo=True, n_frames=500,
                     max_t=25.0, max_rot_deg=8.0, levels=5, cell_size=32, max_keypoints=1500),
}

# Sixteen uneven streams: 4 mono 640x480, 6 stereo 752x480, 4 stereo 1280x720,
# 2 stereo 1920x1080; keypoint caps 150 / 300 / 600 / 1000 by resolution.
BATCH16 = (
    [Workload("b640", 3, 640, 480, n_frames=200, cell_size=40, max_keypoints=150)] * 4
    + [Workload("b752", 3, 752, 480, stereo=True, cell_size=32, max_keypoints=300)] * 6
    + [Workload("b1280", 3, 1280, 720, stereo=True, cell_size=32, max_keypoints=600)] * 4
    + [Workload("b1920", 3, 1920, 1080, stereo=True, cell_size=40, max_keypoints=1000)] * 2
)
