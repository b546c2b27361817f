// Device-side data layout of the frontend, shared by the kernels and the host
// runtime of this library (not by anything outside it).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vio_frontend.h"

namespace vio {

constexpr int kMaxLevels = VIO_MAX_LEVELS;
constexpr int kMaxCams = VIO_MAX_CAMERAS;
constexpr int kPatch = 52;      // pattern points (Sec. III-E)
constexpr int kTileDefault = 64;  // level-0 tile edge of the pyramid/detector kernel unless chosen
// Kernel timing: while set, the frontend's kernel launches on this thread
// attach these events to the dispatch itself (the kernel's own start and end
// timestamps, without the gaps between launches); null for plain launches and
// during graph capture.
struct KernelTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local KernelTiming tl_timing;

template <class F, class... A>
inline void launch_kernel(F kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, A... args) {
  if (tl_timing.start)
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, tl_timing.start, tl_timing.stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// Word 3 of a raw buffer resource on the gfx9 family (32-bit data format,
// byte-addressed range check).
constexpr int kBufferWord3 = 0x00020000;
constexpr int kTrackWaves = 4;  // most waves (keypoints) per tracking block
constexpr int kLearnWavesDefault = 4;  // keypoints (waves) per learned-stage workgroup
// Frames a handle may have in flight; a camera's pyramid slots hold those
// frames' pyramids and the previous frame's, its record slots one frame each.
constexpr int kInFlight = 3;
constexpr int kPyrSlots = kInFlight + 1;
constexpr int kRecSlots = kInFlight;
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
  int kcell, nslots;   // keypoints per cell k; winner key slots ncells * k (cell-major)
  int has_mask;        // detection mask in use (nonzero mask byte: no detection at that pixel)
  // target camera of stereo matches: start from the rig's extrinsics instead of
  // the disparity prior (X_target = R X_detecting + t, keypoints at inverse
  // depth ext_rho, intrinsics ext_Ks of the detecting and ext_Kt of this camera;
  // ext_kbs / ext_kbt: that camera is a KB4 fisheye with coefficients ext_ks / ext_kt)
  int has_ext;
  float ext_Ks[4], ext_Kt[4], ext_R[9], ext_t[3], ext_rho;
  int ext_kbs, ext_kbt;
  float ext_ks[4], ext_kt[4];
  int detect;          // 1: mono camera or left camera of a pair
  int n_targets;       // detecting camera: cameras c+1 .. c+n_targets receive its new keypoints' matches
                       // (1: a stereo pair's right camera, 3: a star rig's other cameras)
  int stream;
  int local;           // camera index within its stream
  int tiles_x, tiles_y, tile_begin;  // pyramid/detector tiles of this camera
  int pitch[kMaxLevels];
  uint8_t* lvl[kPyrSlots][kMaxLevels];  // pyramid slots (frame index mod kPyrSlots: the frames in flight
                                        // and the one before them)
  Kp* state[2];                      // keypoint state, double-buffered by frame parity
  TrackRes* res;                     // temporal results [cap]
  TrackRes* res_fb;                  // parallel fallbacks of short temporal attempts [cap] (or null)
  uint32_t* keys[kPyrSlots];         // packed winner keys, slot cell * k + rank, by pyramid slot [nslots]
  TrackRes* sres;                    // stereo matches [n_targets][nslots], by key slot or selection rank
  const uint8_t* mask;               // detection mask [h][w] (detecting cameras)
  // outputs in mapped pinned host memory, by record slot (frame index mod
  // kRecSlots: the host reads one frame's while the later ones run)
  vio_track* rec[kRecSlots];         // records [rec_cap]
  int32_t* rec_count_out[kRecSlots]; // record count
  int32_t* stats_out[kRecSlots];     // [kCamStats] counts (CamStat)
  int rec_cap;
  int row_off;                       // first row of this camera in the learned-init feature/guess buffers
  // target cameras with the neighbour stereo start: the keypoints that live in
  // both this camera and its detecting camera, in id order, as (x, y) in the
  // detecting camera and the offset to this camera, by frame parity [cap]
  float4* pairs[2];
};

// Per-camera counts of a frame, written by the selection kernel into mapped
// host memory (CamDesc::stats_out).
enum CamStat : int {
  kStatFallback = 0,  // learned tracks that fell back to the plain tracker
  kStatTracked,       // temporal records with VIO_TRACKED
  kStatLost,          // temporal records without VIO_TRACKED
  kStatDetected,      // VIO_DETECTED records
  kStatMatched,       // VIO_MATCHED records
  kCamStats
};

// Per-frame inputs, copied host -> device before every frame.
struct FrameCam {
  const uint8_t* src;  // level-0 image to read (own level 0 or the caller's)
  int src_pitch;
  int copy_l0;         // 1: write src into the own level-0 buffer
  int parity;          // keypoint state slot; the previous frame's is parity ^ 1
  int pyr, pyr_prev;   // pyramid and key slots (frame index mod kPyrSlots) of this and the previous frame
  int rec_slot;        // record slot (frame index mod kRecSlots)
  int has_prev;        // a previous frame exists (temporal tracking runs)
  int active;          // camera takes part in this frame
  int n_pred;          // caller predictions for this camera (ascending id)
  int pred_off;        // their offset in the prediction buffer
  // camera-model start of the temporal tracks (Sec. III-E), this frame only
  int has_motion;
  int n_depth;         // per-keypoint inverse depths (ascending id) at depth_off in Tuning::depths
  int depth_off;
  float K[4];          // fx, fy, cx, cy
  int kb4;             // 1: KB4 fisheye model with coefficients kk (else pinhole)
  float kk[4];
  float R[9], t[3];    // X_new = R X_prev + t
  float rho;           // inverse depth of keypoints without their own
};

struct FrameTable {
  // work-queue counters of the persistent tracker, one per tracking launch
  // of the frame (all items, or temporal then stereo items), zero at the
  // start of every frame
  int queue_head[4];
  FrameCam cam[kMaxCams];
};

// Per-camera counters, indexed [parity][camera]; rec_count[camera].
struct Counters {
  int32_t n_live[2][kMaxCams];
  int32_t rec_count[kMaxCams];
  int64_t next_id[kMaxCams];  // per stream (indexed by stream)
  // deferred stereo matching: a left camera's new detections of the frame
  // are state[P][sel_base .. sel_base + n_sel) (written by the first
  // selection phase, matched by the second tracking launch)
  int32_t sel_base[kMaxCams];
  int32_t n_sel[kMaxCams];
  int32_t n_pairs[2][kMaxCams];  // entries of CamDesc::pairs, [parity][target camera]
};

// Per-keypoint inverse depth of the camera-model start, 16 bytes.
struct KpDepth {
  int64_t id;
  float rho;
  int32_t pad;
};

struct Tuning {
  int levels, iters;
  float fb_threshold, disparity0;
  int tmin, margin;
  int learned;            // temporal tracks start from the learned guess
  int llevels, liters;    // tracker budget from the guess
  float rho;              // residual RMS above which a learned track falls back
  const float* guess;     // [rows][3] network outputs (learned mode)
  int deferred;           // stereo items match the selected detections (by rank), not every cell winner
  const KpDepth* depths;  // per-keypoint inverse depths of the camera-model start (FrameCam ranges)
  int plevels, piters;    // short budget of predicted tracks (plevels 0: none)
  float prho;             // residual RMS above which a predicted short track falls back
  int fblevels, fbiters;  // budget of a learned track's fallback from the constant-velocity start
  int stereo_nb;          // stereo matches start from the nearest paired keypoint's offset
  int slevels, siters;    // budget of such a match
  int par_fb;             // short temporal attempts' fallbacks run as items of their own (CamDesc::res_fb)
  // learned stage fused into the tracker: each learned temporal item computes
  // its own features (into feat) and network output before its short attempt
  int fused;
  float* feat;            // [rows][32] network inputs (learned mode)
  const uint16_t* W1b;    // the network's bf16 weights and FP32 parameters (fused learned stage)
  const uint16_t* W2b;
  const uint16_t* W3b;
  const float* mlpP;
};

// Learned-initialisation network on the device (see vio_mlp.h).
struct MlpDev {
  float* P;        // master parameters [VIO_MLP_NPARAM]
  float* m;        // Adam first moments
  float* v;        // Adam second moments
  uint16_t* W1b;   // bf16 [128][32]
  uint16_t* W2b;   // bf16 [128][128]
  uint16_t* W2tb;  // bf16 [128][128], transposed
  uint16_t* W3b;   // bf16 [3][128]
};

// Work items of the tracking kernel: one segment per (camera, mode).
// kModeFallback: the fallback attempt of temporal item j, run beside it
// (parallel fallbacks), into CamDesc::res_fb[j].
enum : int { kModeTemporal = 0, kModeStereo = 1, kModeFallback = 2 };
struct TrackSeg {
  int cam, mode, begin, count;
};

struct Prediction {
  int64_t id;
  float x, y;
};

// ---- launchers (defined in the kernel translation units) ----
// Pyramid + detector over tiles [tile_base, tile_base + n_tiles) (at least
// one) of cameras [cam_begin, cam_end); tile: the level-0 tile edge the
// cameras' tile grids use (32 or 64). h_frame: the frame's table, mapped
// pinned host memory, which the kernel reads and whose first copy_bytes (a
// multiple of 4) its first workgroup copies to d_frame for the frame's later
// kernels.
hipError_t launch_pyr_detect_range(const CamDesc* d_cams, const FrameTable* h_frame, FrameTable* d_frame,
                                   int copy_bytes, int cam_begin, int cam_end, int tile_base, int n_tiles, int levels,
                                   int tile, int tmin, int margin, hipStream_t s);
size_t pyr_detect_lds_bytes(int levels, int tile);
// Tracking work items [item_base, item_base + n_items) over the segments
// d_segs[0..n_segs) (segment begins are global item indices). waves_per_cu = 0
// launches one wave per item; > 0 launches a persistent grid of that many
// waves per compute unit that pops items from FrameTable::queue_head[shape.queue].
// Launch shape of the tracker: waves_per_cu = 0 gives one wave per work item
// (kp_per_wave = 1) or per two (kp_per_wave = 2, one per 32-lane half), > 0 a
// persistent grid of waves_per_cu * n_cus waves; block_waves waves (1, 2 or
// kTrackWaves) per workgroup.
struct TrackShape {
  int waves_per_cu, block_waves, n_cus;
  int queue;  // the frame's work-queue counter the persistent grid pops (one per tracking launch)
  int kp_per_wave;
};
hipError_t launch_track(const CamDesc* d_cams, FrameTable* d_frame, Counters* d_cnt, const TrackSeg* d_segs,
                        int n_segs, int item_base, int n_items, const Prediction* d_pred, Tuning tune,
                        TrackShape shape, hipStream_t s);
// Features (into d_feat) and network outputs (into d_guess) of the previous
// keypoints of cameras [cam_begin, cam_end); h_cams: host copy of the
// descriptors (caps).
hipError_t launch_learn(const CamDesc* d_cams, const FrameTable* d_frame, const Counters* d_cnt, const CamDesc* h_cams,
                        int cam_begin, int cam_end, const MlpDev& M, float* d_feat, float* d_guess, int waves,
                        hipStream_t s);
hipError_t mlp_forward_launch(const MlpDev& M, const float* X, int K, float* Y, hipStream_t s);
hipError_t mlp_pack_launch(const MlpDev& M, hipStream_t s);
// Selection phases: kSelectAll (speculative stereo: everything in one
// launch), kSelectLeft (deferred: survivors of every camera, selection and
// records of the left cameras; the right cameras' matches follow),
// kSelectRight (deferred: acceptance of the matches into the right cameras).
enum { kSelectAll = 0, kSelectLeft = 1, kSelectRight = 2 };
hipError_t launch_select(const CamDesc* d_cams, const FrameTable* d_frame, Counters* d_cnt,
                         const int* d_stream_cams, int n_streams_launch, int phase, Tuning tune, hipStream_t s);

}  // namespace vio
