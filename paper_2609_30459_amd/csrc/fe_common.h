// Device-side data layout of the frontend, shared by the kernels and the host
// runtime of this library (not by anything outside it).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vio_frontend.h"

namespace vio {

constexpr int kMaxLevels = VIO_MAX_LEVELS;
constexpr int kMaxCams = VIO_MAX_CAMERAS;
constexpr int kPatch = 52;      // pattern points (Sec. III-E)
constexpr int kTile = 64;       // level-0 output tile edge of the pyramid/detector kernel
constexpr int kPyrThreads = 1024;
constexpr int kTrackWaves = 4;  // waves (keypoints) per tracking block
constexpr int kSelectThreads = 1024;

// Live keypoint, 32 bytes (same layout as vio_keypoint).
struct Kp {
  int64_t id;
  float x, y, px, py;
  int32_t age;
  int32_t reserved;
};
static_assert(sizeof(Kp) == 32, "Kp layout");
static_assert(sizeof(Kp) == sizeof(vio_keypoint), "Kp mirrors vio_keypoint");

// Result of one forward-backward track, 32 bytes.
struct TrackRes {
  float x, y, theta, fb, resid;
  int32_t status;
  int32_t pad[2];
};
static_assert(sizeof(TrackRes) == 32, "TrackRes layout");

// Static description of one camera (written once at create).
struct CamDesc {
  int w, h, levels;
  int cap;             // keypoint capacity of the state buffers
  int cell, ncx, ncy, ncells;
  int detect;          // 1: mono camera or left camera of a pair
  int partner;         // right camera of a left camera, left camera of a right one, else -1
  int stream;
  int local;           // camera index within its stream
  int tiles_x, tiles_y, tile_begin;  // pyramid/detector tiles of this camera
  int pitch[kMaxLevels];
  uint8_t* lvl[2][kMaxLevels];       // two pyramid slots (frame parity)
  Kp* state[2];                      // keypoint state, double-buffered by frame parity
  TrackRes* res;                     // temporal results [cap]
  uint32_t* keys[2];                 // per-cell packed winner keys, by frame parity [ncells]
  TrackRes* sres;                    // stereo match of every cell winner [ncells]
  vio_track* rec;                    // output records [rec_cap], in mapped pinned host memory
  int32_t* rec_count_out;            // record count of the last frame, mapped pinned host memory
  int rec_cap;
};

// Per-frame inputs, copied host -> device before every frame.
struct FrameCam {
  const uint8_t* src;  // level-0 image to read (own level 0 or the caller's)
  int src_pitch;
  int copy_l0;         // 1: write src into the own level-0 buffer
  int parity;          // current slot; the previous frame is parity ^ 1
  int has_prev;        // a previous frame exists (temporal tracking runs)
  int active;          // camera takes part in this frame
  int n_pred;          // caller predictions for this camera (ascending id)
  int pred_off;        // their offset in the prediction buffer
};

struct FrameTable {
  FrameCam cam[kMaxCams];
};

// Per-camera counters, indexed [parity][camera]; rec_count[camera].
struct Counters {
  int32_t n_live[2][kMaxCams];
  int32_t rec_count[kMaxCams];
  int64_t next_id[kMaxCams];  // per stream (indexed by stream)
};

struct Tuning {
  int levels, iters;
  float fb_threshold, disparity0;
  int k, tmin, margin;
};

// Work items of the tracking kernel: one segment per (camera, mode).
enum : int { kModeTemporal = 0, kModeStereo = 1 };
struct TrackSeg {
  int cam, mode, begin, count;
};

struct Prediction {
  int64_t id;
  float x, y;
};

// ---- launchers (defined in the kernel translation units) ----
hipError_t launch_pyr_detect_range(const CamDesc* d_cams, const FrameTable* d_frame, int cam_begin, int cam_end,
                                   int tile_base, int n_tiles, int levels, int tmin, int margin, hipStream_t s);
size_t pyr_detect_lds_bytes(int levels);
hipError_t launch_track(const CamDesc* d_cams, const FrameTable* d_frame, Counters* d_cnt,
                        const TrackSeg* d_segs, int n_segs, int n_items, const Prediction* d_pred,
                        Tuning tune, hipStream_t s);
hipError_t launch_select(const CamDesc* d_cams, const FrameTable* d_frame, Counters* d_cnt,
                         const int* d_stream_cams, int n_streams_launch, int cams_per_stream_max, Tuning tune,
                         hipStream_t s);

}  // namespace vio
