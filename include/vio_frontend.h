/*
 * vio_frontend.h -- C ABI of the MI355X (gfx950) stereo VIO frontend.
 *
 * The frontend is the data-parallel half of a visual-inertial odometry
 * pipeline as stated in VkVIO (arXiv 2609.30459), Sec. III-B: per frame it
 *   1. builds an image pyramid per camera (Sec. III-C, eqs. 1-3),
 *   2. tracks every camera's previous keypoints KP_{t-1} into the new frame with
 *      inverse-compositional SE(2) patch alignment and a forward-backward check
 *      (Sec. III-E, eqs. 4-5),
 *   3. detects FAST-9 corners on a grid of cells with 3x3 non-maximum
 *      suppression, masking cells that still hold a track (Sec. III-D),
 *   4. matches the new detections of each stereo pair's left camera into its
 *      right camera with the same tracker (Sec. III-B, "cross-camera matching"),
 * and hands back the tracked/matched positions (TR_t) and the new detections
 * (DET_t) after one synchronous submit and wait (Sec. III-B, Fig. 2).
 *
 * Conventions
 *  - Every call returns VIO_OK (0) or a negative vio_result. No C++ exception
 *    crosses this boundary. On any error other than VIO_EDEVICE the handle is
 *    unchanged. VIO_EDEVICE (a HIP runtime error) poisons the handle: every
 *    later call except destroy/last_error returns VIO_EDEVICE.
 *  - A handle is single-threaded; separate handles are independent.
 *  - The library owns the handle and all device memory, allocated once in
 *    vio_frontend_create (Sec. III-B: resources are allocated at
 *    initialisation and reused every frame). Pointers passed in are borrowed
 *    for the duration of the call only.
 *  - Pixel coordinates are level-0 pixels, origin at the centre of the top-left
 *    pixel, x to the right, y down.
 */
#ifndef VIO_FRONTEND_H
#define VIO_FRONTEND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VIO_MAX_LEVELS 6
#define VIO_MAX_CAMERAS 64

typedef enum vio_result {
  VIO_OK = 0,
  VIO_EINVAL = -1,       /* null pointer, bad size, unknown stream or camera */
  VIO_ENOMEM = -2,       /* device or pinned host allocation failed */
  VIO_EDEVICE = -3,      /* HIP runtime error; the handle is poisoned */
  VIO_ETOOSMALL = -4,    /* output capacity too small; *n_out holds the count needed */
  VIO_ESTATE = -5,       /* call out of order (e.g. get before any push, timestamps not increasing) */
  VIO_EUNSUPPORTED = -6  /* valid request this build does not implement */
} vio_result;

/* Per-record status. */
typedef enum vio_status {
  VIO_TRACKED = 0,         /* temporal track kept (passed the forward-backward check) */
  VIO_DETECTED = 1,        /* new keypoint detected in this frame (left / mono camera) */
  VIO_MATCHED = 2,         /* new keypoint matched into the right camera of its pair */
  VIO_LOST_FB = 3,         /* forward-backward distance above the threshold */
  VIO_LOST_OOB = 4,        /* the patch left the image */
  VIO_LOST_DEGENERATE = 5, /* template Hessian near singular or patch mean not positive */
  VIO_LOST_CAP = 6         /* stereo match dropped: the right camera is full */
} vio_status;

typedef enum vio_init_mode {
  VIO_INIT_CONST_VEL = 0, /* p + (p - p_prev); the caller's predictions override it */
  VIO_INIT_LEARNED = 1    /* learned displacement guess refined by the tracker */
} vio_init_mode;

/* One input stream: a mono camera, a stereo pair (cameras 0,1), or four
 * cameras: two stereo pairs (0,1) and (2,3), or a star rig (0 -> 1, 2, 3) with
 * vio_frontend_params.topology = VIO_TOPOLOGY_STAR. All cameras of a stream
 * share the image size. */
typedef struct vio_stream_desc {
  int32_t n_cameras;     /* 1, 2 or 4 */
  int32_t width, height; /* level-0 size in pixels, 16..4096 each, width*height < 2^24 */
  int32_t max_keypoints; /* per camera; 0 = take vio_frontend_params.max_keypoints */
  int32_t cell_size;     /* detection cell edge in px; 0 = take vio_frontend_params.cell_size */
} vio_stream_desc;

/* Frontend parameters (versioned by struct_size). Defaults: see
 * vio_frontend_default_params. */
typedef struct vio_frontend_params {
  uint32_t struct_size;   /* sizeof(vio_frontend_params) */
  int32_t levels;         /* pyramid levels L including level 0, 1..VIO_MAX_LEVELS (Sec. III-C) */
  int32_t gn_iters;       /* Gauss-Newton iterations per level N, 1..32 (Sec. III-E) */
  int32_t cell_size;      /* default cell edge C in px (Sec. III-D) */
  int32_t k_per_cell;     /* keypoints per cell k, 1..8 (Sec. III-D) */
  int32_t n_thresholds;   /* 1..4 */
  int32_t thresholds[4];  /* FAST threshold walk, strictly decreasing, e.g. 40, 20, 10, 5 (Sec. III-D) */
  int32_t edge_margin;    /* detections keep this distance to the border, >= 4 px */
  int32_t max_keypoints;  /* default per-camera keypoint cap */
  float fb_threshold;     /* forward-backward distance limit in px (Sec. III-E) */
  float disparity0;       /* stereo initialisation: right = left - (disparity0, 0) */
  int32_t init_mode;      /* vio_init_mode */
  int32_t learned_levels; /* tracker budget when the learned guess is used */
  int32_t learned_iters;
  float learned_rho;      /* residual RMS above which a learned track falls back to the plain tracker */
  uint32_t flags;         /* VIO_FLAG_* */
  int32_t track_waves_per_cu; /* 0: one wave per tracking work item; > 0: a persistent tracking grid
                                 of this many waves per compute unit over a shared work queue */
  int32_t track_block_waves;  /* waves per tracking workgroup: 1, 2 or 4 (0 = 4) */
  int32_t pyr_tile;           /* level-0 tile edge of the pyramid/detector kernel: 32 (256-thread workgroups)
                                 or 64 (1024 threads); 0 = 64 */
  int32_t stereo_mode;        /* VIO_STEREO_SPECULATIVE: the tracking launch also matches every cell
                                 winner left to right, selection keeps the selected ones' matches (fewest
                                 dependent launches); VIO_STEREO_DEFERRED: only the selected detections are
                                 matched, in a second tracking launch after selection (least work). The
                                 records are the same either way. */
  int32_t pred_levels;        /* tracker budget of a predicted temporal track (caller prediction or camera-model
                                 start): 0 = the full budget; 1..levels = this many levels and pred_iters
                                 iterations first, the full budget from the same start when the track is not
                                 kept or its residual RMS exceeds pred_rho (counted as a fallback) */
  int32_t pred_iters;
  float pred_rho;
  int32_t topology;           /* four-camera streams: VIO_TOPOLOGY_PAIRS (pairs (0,1) and (2,3), each left
                                 camera detects) or VIO_TOPOLOGY_STAR (camera 0 detects, its new keypoints
                                 are matched into cameras 1, 2 and 3, each with its own keypoint cap) */
  /* Optional device allocator for the handle's one device arena (every device
   * buffer of the handle lives in it; allocated once in vio_frontend_create,
   * released in vio_frontend_destroy, Sec. III-B). dev_alloc(bytes, ctx)
   * returns device memory of the handle's device aligned to 256 bytes, or NULL
   * (create then fails with VIO_ENOMEM); dev_free(ptr, ctx) releases it. Set
   * both or neither (NULL: hipMalloc / hipFree). */
  void* (*dev_alloc)(size_t bytes, void* ctx);
  void (*dev_free)(void* ptr, void* ctx);
  void* alloc_ctx;
  /* Learned initialisation: budget of the fallback from the constant-velocity
   * start when the short track from the network's guess is not kept:
   * learned_fb_levels levels (1..levels) with learned_fb_iters iterations
   * (1..32); learned_fb_levels = 0 takes the full budget levels x gn_iters. */
  int32_t learned_fb_levels;
  int32_t learned_fb_iters;
  /* Start of a new keypoint's stereo matches into a camera without the rig's
   * extrinsics: VIO_STEREO_INIT_PRIOR, the disparity prior p - (disparity0, 0)
   * with the full budget; or VIO_STEREO_INIT_NEIGHBOUR (a project addition, in
   * the spirit of the learned initialisation): of the keypoints that, after
   * the previous frame, lived in both the detecting and the target camera, the
   * nearest to p by (squared distance between p and its detecting-camera
   * position, id) lends its offset (x_target - x_detecting, y_target -
   * y_detecting): the match starts at p plus that offset with stereo_levels
   * levels (1..levels) and stereo_iters iterations (1..32); without such a
   * keypoint, the disparity prior with the full budget. */
  int32_t stereo_init;
  int32_t stereo_levels;
  int32_t stereo_iters;
  /* Launch choice that never changes the records: 1 = a track that first runs a
   * short budget (learned guess or predicted start) has its fallback computed at
   * the same time by a second wave, and the selection takes it when the short
   * track is not kept (one frame's tracker chain is then the longer of the two,
   * not their sum, for up to twice the tracker work); 0 = the fallback runs after
   * the short attempt in the same wave. */
  int32_t track_parallel_fallback;
  /* Launch choice that never changes the records: keypoints (one wave each) per
   * workgroup of the learned stage, 4, 8 or 16 (0 = 4); fewer spread a camera's
   * keypoints over more compute units. */
  int32_t learned_block_waves;
  /* Launch choice that never changes the records: 1 = the learned stage runs
   * inside the tracker launch (each learned temporal track computes its own
   * features and network output before its short attempt, beside the stereo
   * and fallback work) instead of as a launch of its own before it; 0 = its
   * own launch. */
  int32_t learned_fused;
  /* Launch choice that never changes the records: where a frame's pyramid and
   * detection run. VIO_PYRAMID_SIGNAL (0): on a stream of their own, so that
   * the later frames' pyramids run beside this frame's tracking; the launch
   * stream waits for a count the pyramid stream writes (stream value
   * operations: the least host time per frame). VIO_PYRAMID_EVENT (1): the
   * same with an event record and wait. VIO_PYRAMID_SAME_STREAM (2): on the
   * launch stream, in order (no cross-stream dependency). */
  int32_t pyramid_stream;
  /* Launch choice that never changes the records: keypoints per tracking
   * wavefront. 1 (or 0): one wave64 per keypoint, a lane per pattern point
   * (the shortest chain per keypoint: few keypoints, one frame at a time);
   * 2: two keypoints per wave, one per 32-lane half, two pattern points per
   * lane (fewer instructions per keypoint: many keypoints, batched streams).
   * 2 needs learned_fused = 0 when init_mode is VIO_INIT_LEARNED. */
  int32_t track_kp_per_wave;
} vio_frontend_params;

#define VIO_PYRAMID_SIGNAL 0
#define VIO_PYRAMID_EVENT 1
#define VIO_PYRAMID_SAME_STREAM 2

#define VIO_STEREO_INIT_PRIOR 0
#define VIO_STEREO_INIT_NEIGHBOUR 1
#define VIO_STEREO_SPECULATIVE 0
#define VIO_STEREO_DEFERRED 1
#define VIO_TOPOLOGY_PAIRS 0
#define VIO_TOPOLOGY_STAR 1

/* vio_frontend_params.flags */
#define VIO_FLAG_EAGER 1u /* launch the per-frame kernels one by one, each with dispatch timestamps, instead
                             of replaying a captured hipGraph */
#define VIO_FLAG_PLAIN 2u /* launch the per-frame kernels one by one without timestamps (fewer host calls
                             than a graph launch for small frames); excludes VIO_FLAG_EAGER */

/* Output record: one per previous keypoint of each camera (tracked or lost) and
 * one per new detection / stereo match, sorted by (camera, id). */
typedef struct vio_track {
  int64_t id;       /* keypoint identifier, shared by a left keypoint and its right match */
  float x, y;       /* level-0 position in this frame (forward result for tracks) */
  float theta;      /* estimated in-plane patch rotation, radians */
  float fb_err;     /* forward-backward distance, px (0 for detections) */
  float resid_rms;  /* RMS of the photometric residual at the last level-0 iteration */
  int32_t age;      /* frames this keypoint has been tracked */
  int16_t camera;   /* camera index within the stream */
  int16_t status;   /* vio_status */
  int32_t score;    /* FAST score for VIO_DETECTED, -1 otherwise */
} vio_track;        /* 40 bytes */

/* A live keypoint (the state KP_{t-1} the paper uploads from the host). */
typedef struct vio_keypoint {
  int64_t id;
  float x, y;   /* position in the last frame */
  float px, py; /* position one frame earlier (equal to x, y for a new keypoint) */
  int32_t age;
  int32_t reserved;
} vio_keypoint;  /* 32 bytes */

/* A caller-side prediction of a keypoint's position in the new frame (Sec.
 * III-E: the backend projects the pattern through its predicted pose). It
 * replaces the constant-velocity initialisation of that keypoint. */
typedef struct vio_kp_prediction {
  int64_t id;
  int32_t camera;
  float x, y;
} vio_kp_prediction;

/* Pinhole camera model: focal lengths and principal point in pixels. */
typedef struct vio_pinhole {
  float fx, fy, cx, cy;
} vio_pinhole;  /* 16 bytes */

/* Kannala-Brandt equidistant fisheye model with four coefficients (KB4, the
 * calibration model of wide-angle datasets; Sec. III-E only names "the camera
 * model"): a ray at angle theta to the optical axis, azimuth phi, lands at
 * pixel (fx r cos phi + cx, fy r sin phi + cy) with r = theta (1 + k[0]
 * theta^2 + k[1] theta^4 + k[2] theta^6 + k[3] theta^8). A keypoint's inverse
 * depth under this model is the inverse of its distance along the ray (the
 * pinhole model's is that of its depth along the optical axis). */
typedef struct vio_kb4 {
  float fx, fy, cx, cy;
  float k[4];
} vio_kb4;  /* 32 bytes */

/* Predicted rigid motion of one camera from its previous frame to the next
 * one: a point X of the previous camera frame is R X + t in the new one (R
 * row-major, t in the units of 1 / inv_depth). */
typedef struct vio_camera_motion {
  int32_t camera;    /* camera index within the stream */
  float R[9];
  float t[3];
  float inv_depth;   /* inverse depth of the camera's keypoints without their own entry, > 0 */
} vio_camera_motion;  /* 56 bytes */

/* Inverse depth of one keypoint (its landmark, as the backend estimates it). */
typedef struct vio_kp_depth {
  int64_t id;
  int32_t camera;
  float inv_depth;   /* > 0 */
} vio_kp_depth;  /* 16 bytes */

typedef struct vio_stats {
  int64_t frames;        /* frames processed by the handle */
  double last_gpu_ms;    /* device time of the last completed frame, from the start of its pyramid to its
                            selection (with frames in flight it overlaps the neighbouring frames'); -1 with
                            VIO_FLAG_PLAIN (no timestamps) */
  double last_stage_ms[3]; /* durations of the last frame's pyramid+detector, tracker and selection
                              kernels from their own dispatch timestamps (HIP events attached to the
                              launch); -1 unless launched one by one (VIO_FLAG_EAGER) */
  double last_learned_ms[2]; /* the same for the learned stage's own launch (features and network) in
                                [0], -1 when it is fused into the tracker; [1] is -1 (unused) */
  int32_t last_tracked;  /* VIO_TRACKED records of the last frame, all cameras */
  int32_t last_lost;     /* lost temporal records of the last frame */
  int32_t last_detected; /* VIO_DETECTED records */
  int32_t last_matched;  /* VIO_MATCHED records */
  int32_t last_fallback; /* tracks whose short attempt (learned or predicted start) fell back to the
                            full budget */
} vio_stats;

typedef struct vio_frontend vio_frontend;

/* Fills *p with the paper's standard configuration: L = 4, N = 5, cells of 50
 * px, k = 1, thresholds 40/20/10/5, margin 8, 300 keypoints, FB threshold 0.3
 * px, disparity prior 32.5 px, constant-velocity init. */
void vio_frontend_default_params(vio_frontend_params* p);

/* Creates a frontend for n_streams streams (1..VIO_MAX_CAMERAS cameras in all).
 * Allocates every device buffer and the pinned host staging here; nothing is
 * allocated per frame. On success *out receives the handle (caller frees it
 * with vio_frontend_destroy). Errors: VIO_EINVAL, VIO_ENOMEM, VIO_EDEVICE,
 * VIO_EUNSUPPORTED (a pyramid depth whose tile does not fit in LDS). */
int vio_frontend_create(const vio_stream_desc* streams, int32_t n_streams, const vio_frontend_params* params,
                        vio_frontend** out);

/* Releases the handle and all its memory. NULL is a no-op. */
void vio_frontend_destroy(vio_frontend* h);

/* Processes one frame of `stream`: images[c] points to camera c's width x height
 * uint8 image with row stride strides[c] bytes (host memory, read before the
 * call returns). pred (n_pred entries, may be NULL when n_pred == 0) overrides
 * the initialisation of the listed keypoints. t_ns must increase strictly per
 * stream. Synchronous: returns once the frame's records are ready for
 * vio_frontend_get_tracks. */
int vio_frontend_push_stereo_frame(vio_frontend* h, int32_t stream, int64_t t_ns, const uint8_t* const* images,
                                   const int32_t* strides, const vio_kp_prediction* pred, int32_t n_pred);

/* As above with device-resident images: d_images[c] is a device pointer with
 * row pitch pitches[c] bytes, read on `hip_stream` (a hipStream_t, NULL = the
 * handle's own stream) during this call only. The frame runs on that stream. */
int vio_frontend_push_stereo_frame_device(vio_frontend* h, int32_t stream, int64_t t_ns,
                                          const void* const* d_images, const int32_t* pitches, void* hip_stream);

/* Batched stepping: stage one frame for any number of streams, then run every
 * staged stream in one submit (one pyramid/detector launch over all their
 * cameras, one tracking launch over all their keypoints, one selection
 * launch), replayed as one captured graph. The staging calls copy nothing:
 * d_images must stay valid until vio_frontend_step returns; host images are
 * copied into pinned staging at stage time. A stream staged twice keeps the
 * last frame. vio_frontend_step is synchronous; afterwards each staged
 * stream's records are read with vio_frontend_get_tracks. */
int vio_frontend_stage_frame(vio_frontend* h, int32_t stream, int64_t t_ns, const uint8_t* const* images,
                             const int32_t* strides);
int vio_frontend_stage_frame_device(vio_frontend* h, int32_t stream, int64_t t_ns, const void* const* d_images,
                                    const int32_t* pitches);
int vio_frontend_step(vio_frontend* h);

/* Pipelined stepping: vio_frontend_step_async submits the staged streams'
 * frames like vio_frontend_step but returns without waiting; while it runs
 * the host may stage the next frames and submit them too (at most three
 * frames in flight: staging, pushing or submitting a fourth returns
 * VIO_ESTATE). vio_frontend_wait waits for the oldest frame in flight
 * (VIO_ESTATE when none); afterwards vio_frontend_get_tracks returns its
 * records, while the later frames may still run (records rotate over three
 * buffers by frame: a completed frame's records stay valid until the next
 * submission).
 * Every other call (pushes, keypoint and diagnostic calls) first waits for
 * all frames in flight. Device images staged for a frame must stay valid
 * until that frame is waited for. vio_frontend_in_flight returns the number
 * of frames in flight (0 for NULL). */
int vio_frontend_step_async(vio_frontend* h);
int vio_frontend_wait(vio_frontend* h);
int vio_frontend_in_flight(const vio_frontend* h);

/* Stages device images for n streams at once: stream streams[i] at t_ns[i]
 * takes the next n_cameras entries of d_images / pitches (in stream order). */
int vio_frontend_stage_frames_device(vio_frontend* h, int32_t n, const int32_t* streams, const int64_t* t_ns,
                                     const void* const* d_images, const int32_t* pitches);

/* Detection mask of a detecting camera (mono or left; the mask buffer the
 * host uploads with the frames, Fig. 2): mask points to width x height bytes
 * with row pitch `pitch` >= width (host memory, copied during the call); a
 * nonzero byte means no new keypoint at that pixel. A masked corner is dropped
 * after non-maximum suppression, so it still suppresses its neighbours, and
 * the cell's next strongest corners compete for its k places (Sec. III-D).
 * Stays in effect for every following frame; mask == NULL removes it. Tracked
 * keypoints are not affected. Errors: VIO_EINVAL (stream or camera out of
 * range, a camera that does not detect, pitch < width), VIO_EDEVICE. */
int vio_frontend_set_detection_mask(vio_frontend* h, int32_t stream, int32_t camera, const uint8_t* mask,
                                    int32_t pitch);

/* Sets (K != NULL) or clears (K == NULL) the pinhole model of one camera of a
 * stream; fx, fy > 0. Needed before vio_frontend_set_motion names the camera.
 * Errors: VIO_EINVAL. */
int vio_frontend_set_camera_model(vio_frontend* h, int32_t stream, int32_t camera, const vio_pinhole* K);

/* Sets a camera's model to the KB4 fisheye model K (replacing a pinhole model
 * or an earlier KB4 one; vio_frontend_set_camera_model switches it back). Every
 * use of the camera model (the temporal start of vio_frontend_set_motion and
 * the stereo extrinsics start) then back-projects a pixel by inverting the
 * radius polynomial with Newton's method (the ray is undefined where it has no
 * root below pi at which the radius rises with slope >= 0.05, i.e. at and near
 * the polynomial's fold: such a keypoint keeps the start it would have
 * without the model) and projects through the same model. The
 * start rotation is the angle of the image of the pixel step (1, 0), as for
 * the pinhole model. Stereo extrinsics copy both cameras' models when they are
 * set: set the models first. VIO_EINVAL for a null K, non-finite values,
 * fx <= 0 or fy <= 0, or a stream or camera out of range. */
int vio_frontend_set_camera_kb4(vio_frontend* h, int32_t stream, int32_t camera, const vio_kb4* K);

/* Stereo extrinsics of a camera that receives matches (a pair's right camera
 * or a star rig's cameras 1-3): its matches of the detecting camera's new
 * keypoints start at the projection of the keypoint, back-projected through
 * the detecting camera's model (pinhole or KB4) at inverse depth inv_depth, moved by
 * X_this = R X_detecting + t (R row-major) and projected through this camera's
 * model, instead of the disparity prior p - (disparity0, 0) (Sec. III-E starts
 * every warp from the camera model). Both cameras' models must be set first
 * (they are copied now). Stays in effect for every following frame; R == NULL
 * returns to the disparity prior. A point not in front of this camera keeps
 * the prior. Errors: VIO_EINVAL (camera out of range or detecting, models
 * missing, a non-finite value, inv_depth <= 0), VIO_EDEVICE. */
int vio_frontend_set_stereo_extrinsics(vio_frontend* h, int32_t stream, int32_t camera, const float* R,
                                       const float* t, float inv_depth);

/* Camera-model initialisation (Sec. III-E: the forward warp starts from the
 * pattern projected into the new image through the camera model, with the
 * predicted pose and the keypoint's inverse depth), for the stream's next frame
 * only (the next push or stage of the stream consumes it; a second call before
 * that replaces the first). For every camera named in m[0..n_m), each temporal
 * track without a caller prediction (vio_kp_prediction, which takes
 * precedence) starts at the projection of its keypoint p: back-projected at the
 * keypoint's inverse depth rho (its depths[] entry, else the camera's
 * inv_depth) to X = ((p - c) / f, 1) / rho, moved to R X + t and projected
 * through the same pinhole model, with the start rotation of the image x axis
 * under that mapping. A keypoint whose point would not lie in front of the new
 * camera keeps its usual start. Learned mode skips the network for such
 * tracks. Host arrays are read during the call. Errors (nothing is kept):
 * VIO_EINVAL for a camera out of range or without a model, a repeated camera,
 * a non-finite value, inv_depth <= 0, a repeated (camera, id) depth, more
 * depths for a camera than its keypoint cap. */
int vio_frontend_set_motion(vio_frontend* h, int32_t stream, const vio_camera_motion* m, int32_t n_m,
                            const vio_kp_depth* depths, int32_t n_depths);

/* Copies the last frame's records of `stream` into out[0..capacity). *n_out
 * receives the record count; VIO_ETOOSMALL (nothing written) when capacity is
 * smaller. VIO_ESTATE before the stream's first push. */
int vio_frontend_get_tracks(vio_frontend* h, int32_t stream, vio_track* out, int32_t capacity, int32_t* n_out);

/* The last frame's records of n streams in one call: those of streams[i]
 * follow those of streams[0..i), each stream's as vio_frontend_get_tracks
 * orders them; counts[i] receives stream i's record count and *n_out the
 * total. VIO_ETOOSMALL (nothing written to out, counts and *n_out set) when
 * capacity is smaller; VIO_EINVAL / VIO_ESTATE as vio_frontend_get_tracks. */
int vio_frontend_get_tracks_streams(vio_frontend* h, int32_t n, const int32_t* streams, vio_track* out,
                                    int32_t capacity, int32_t* counts, int32_t* n_out);

/* Replaces camera `camera`'s live keypoints of `stream` with kps[0..n) (ids
 * strictly ascending, n <= the camera's keypoint cap): the host upload of
 * KP_{t-1} (Sec. III-B, Fig. 2). New identifiers continue above the largest id
 * seen. */
int vio_frontend_set_keypoints(vio_frontend* h, int32_t stream, int32_t camera, const vio_keypoint* kps,
                               int32_t n);

/* Copies camera `camera`'s live keypoints (after the last frame) into out. */
int vio_frontend_get_keypoints(vio_frontend* h, int32_t stream, int32_t camera, vio_keypoint* out,
                               int32_t capacity, int32_t* n_out);

/* Diagnostics: copies pyramid level `level` of the last frame of a camera into
 * out (width>>level columns, height>>level rows, packed). */
int vio_frontend_get_pyramid(vio_frontend* h, int32_t stream, int32_t camera, int32_t level, uint8_t* out,
                             size_t capacity);

/* Diagnostics: per-cell detector winners of the last frame of a detecting
 * camera (mono or left), before masking and the cap, k per cell in rank order
 * (score desc, y asc, x asc): out[3*(cell*k + rank) + {0,1,2}] = x, y, score,
 * or -1, -1, -1 for an empty rank. *n_out = cells * k. */
int vio_frontend_get_cell_winners(vio_frontend* h, int32_t stream, int32_t camera, int32_t* out,
                                  int32_t capacity, int32_t* n_out);

int vio_frontend_get_stats(vio_frontend* h, vio_stats* out);

/* Human-readable description of the handle's last error ("" when none). The
 * string lives as long as the handle. */
const char* vio_frontend_last_error(const vio_frontend* h);

#ifdef __cplusplus
}
#endif

#endif /* VIO_FRONTEND_H */
