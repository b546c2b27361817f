// Host runtime behind the C ABI in vio_frontend.h.
//
// Device memory is one arena allocated at create (Sec. III-B: every resource
// is allocated once and reused). Per frame the runtime fills a small frame
// table in pinned memory and launches the frame's kernels on two streams: the
// pyramid stream runs the pyramid+detector kernel (which copies the table to
// the device and, for a host push, reads the staged images); the launch
// stream runs the learned stage, then, once the pyramid stream's signal says
// the pyramid is done, the tracker and the selection. The selection writes
// the records into mapped pinned host memory, so nothing is copied back; the
// host fences on an event after the selection.
//
// Per camera the arena holds: pyramid levels and per-cell winner keys by
// pyramid slot, keypoint state by frame parity, temporal and stereo results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fe_common.h"
#include "vio_mlp.h"

using namespace vio;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxCellsAbi = 8192;  // matches the selection kernel's LDS tables
constexpr int kMaxPerCell = 8;
static_assert(kMaxCellsAbi * kMaxPerCell <= 65536, "the selection kernel keeps key slot indices in 16 bits");

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Captured submit of a launch set: the whole frame as one graph.
// Captured launches of one submission slot: the learned stage (features and
// network) and the tracking part (tracker and selection) of a frame. The
// frame-table copy and the pyramid/detector run as plain launches on the
// pyramid stream (a captured copy-and-kernel graph launched slower).
struct Graphs {
  hipGraphExec_t learn = nullptr, trk = nullptr;
  bool captured = false;
  bool any() const { return captured; }
  void destroy() {
    for (hipGraphExec_t* g : {&learn, &trk}) {
      if (*g) (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
    captured = false;
  }
};

struct StreamInfo {
  int first_cam, n_cams, w, h, cap, cell;
  int64_t frames = 0;
  int64_t last_t = 0;
  int tile_begin = 0, n_tiles = 0;
  int seg_begin = 0, n_segs = 0, item_begin = 0, n_items = 0;
  int st_segs = 0, st_items = 0;  // the stream's stereo segments/items come first
  int64_t done = 0;        // frames whose records are ready (frames - done are in flight)
  bool staged = false;     // a frame is staged for the next vio_frontend_step
  int64_t staged_t = 0;
  size_t rec_off = 0, rec_n = 0;  // record range (in vio_track units) of the stream's cameras
  Graphs graph[kInFlight];         // captured per-frame submit by submission slot, replayed every frame
  // camera-model start for the next frame (vio_frontend_set_motion)
  std::vector<vio_camera_motion> motion;  // at most one per camera
  std::vector<vio_kp_depth> depths;       // sorted by (camera, id)
};

}  // namespace

thread_local KernelTiming vio::tl_timing;

// A set of cameras/streams launched together: one stream (push) or all (step).
struct LaunchSet {
  int cam_begin, cam_end, tile_begin, n_tiles, seg_begin, n_segs, item_begin, n_items, stream_begin, n_streams;
  bool all;               // every stream: the batched item order (segs_all)
  int st_segs, st_items;  // the leading stereo segments/items of the range
};

enum {
  kKernPyr,
  kKernFeatures,
  kKernMlp,
  kKernTrack,
  kKernSelect,
  kKernTrackStereo,
  kKernSelectRight,
  kKernGrid,
  kKernels
};

struct vio_frontend {
  vio_frontend_params P{};
  int n_cus = 256;
  int tile = kTileDefault;  // pyramid/detector tile edge
  Graphs graph_all[kInFlight];  // captured batched step by submission slot
  std::vector<StreamInfo> streams;
  std::vector<CamDesc> cams;
  std::vector<TrackSeg> segs;      // per stream: the stream's items are contiguous
  std::vector<TrackSeg> segs_all;  // the same items in the batched step's order
  std::vector<int> stream_cams;
  int total_tiles = 0;
  size_t rec_total = 0;
  // device
  void* arena = nullptr;
  CamDesc* d_cams = nullptr;
  FrameTable* d_frames[kInFlight] = {};  // by submission slot
  FrameTable* d_frame = nullptr;                 // the slot being launched
  Counters* d_cnt = nullptr;
  TrackSeg* d_segs = nullptr;
  TrackSeg* d_segs_all = nullptr;
  int* d_stream_cams = nullptr;
  Prediction* d_pred = nullptr;
  int pred_cap = 0;
  KpDepth* d_depth = nullptr;  // per camera at CamDesc::row_off, up to its cap
  std::vector<vio_pinhole> K;  // per camera; fx == 0: no model
  std::vector<vio_kb4> kb;     // per camera: the KB4 coefficients when kb4[c]
  std::vector<int> kb4;
  std::vector<size_t> rec_host_off;  // per camera, in records
  // learned initialisation
  bool learned = false, mlp_ready = false;
  MlpDev mlp{};
  float* d_feat = nullptr;   // [rows][32]
  float* d_guess = nullptr;  // [rows][3]
  int32_t* h_camstats = nullptr;  // [record slot][cameras][kCamStats], written by the selection kernel
  // pinned host
  // Submissions rotate over kInFlight slots: the frame table, the host image
  // staging and the prediction / depth lists being filled belong to slot
  // sub % kInFlight, so the next frame can be staged while earlier ones run.
  // Records, their counts and the per-camera counts rotate over kRecSlots
  // buffers by each camera's frame index instead.
  FrameTable* h_frames[kInFlight] = {};
  FrameTable* h_frame = nullptr;  // h_frames[sub % kInFlight]
  FrameTable* hm_frames[kInFlight] = {};  // device mappings of h_frames
  FrameTable* hm_frame = nullptr;                 // the slot being launched
  int64_t sub = 0;                // submissions so far
  struct Pending {
    LaunchSet ls;
    bool graphed;
    int slot;
  };
  Pending pend[kInFlight];
  int n_pend = 0, pend_head = 0;  // submitted, not yet completed (oldest first)
  int32_t* h_rec_count = nullptr; // [record slot][cameras]
  vio_track* h_rec = nullptr;     // [record slot][rec_total]
  uint8_t* h_stage = nullptr;     // [slot][stage_bytes]
  size_t stage_bytes = 0;
  Prediction* h_pred = nullptr;  // [slot][pred_cap]
  KpDepth* h_depth = nullptr;    // [slot][pred_cap]
  hipStream_t stream = nullptr;   // the launch stream: learned stage, tracking, selection
  hipStream_t pstream = nullptr;  // frame-table copies and pyramids/detections
  hipEvent_t ev_pyr[kInFlight] = {}, ev_in = nullptr;  // per slot: pyramid done; a caller stream's images ready
  // the pyramid stream's completion count in signal memory (stream value
  // operations; null: events ev_pyr instead)
  uint32_t* pyr_sig = nullptr;
  uint32_t pyr_epoch = 0;  // the last value the pyramid stream was asked to write
  hipEvent_t ev[kInFlight][2] = {};  // per submission slot: frame start and end on the launch stream
  // eager launches: start/stop events attached to each kernel's dispatch
  // (pyramid+detector, features, network, tracker, selection)
  hipEvent_t kev[kKernels][2] = {};
  bool kran[kKernels] = {};  // kernels launched (and timed) in the last eager frame
  int device = 0;
  bool poisoned = false;
  bool fault_device = false;
  bool eager = false;        // graph capture off (flag) or unavailable
  bool plain = false;        // plain launches: no graphs, no per-kernel timing
  std::string err;
  vio_stats stats{};
};

namespace {

// Signals of the pyramid streams: 8-byte signal-memory allocations, one per
// live handle, taken from a per-device pool that is never freed (a handle
// returns its signal with its last value, and the next handle on the device
// continues from there). The launch stream waits for the value the pyramid
// stream writes after the frame's pyramid: for the host about ten
// microseconds per frame less than an event record and a wait on it.
struct PyrSignal {
  uint32_t* ptr;
  uint32_t last;
};
std::mutex g_sig_mu;
std::map<int, std::vector<PyrSignal>> g_sig_free;  // by device
std::map<int, bool> g_sig_unsupported;

bool signal_acquire(int device, uint32_t** ptr, uint32_t* last) {
  std::lock_guard<std::mutex> lk(g_sig_mu);
  std::vector<PyrSignal>& fr = g_sig_free[device];
  if (!fr.empty()) {
    *ptr = fr.back().ptr;
    *last = fr.back().last;
    fr.pop_back();
    return true;
  }
  if (g_sig_unsupported[device]) return false;
  int can = 0;
  void* p = nullptr;
  if (hipDeviceGetAttribute(&can, hipDeviceAttributeCanUseStreamWaitValue, device) != hipSuccess || !can ||
      hipExtMallocWithFlags(&p, 8, hipMallocSignalMemory) != hipSuccess || hipMemset(p, 0, 8) != hipSuccess) {
    // events instead (an allocation that could not be cleared is left alone)
    g_sig_unsupported[device] = true;
    (void)hipGetLastError();
    return false;
  }
  *ptr = static_cast<uint32_t*>(p);
  *last = 0;
  return true;
}

void signal_release(int device, uint32_t* ptr, uint32_t last) {
  std::lock_guard<std::mutex> lk(g_sig_mu);
  g_sig_free[device].push_back(PyrSignal{ptr, last});
}

int fail(vio_frontend* h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(vio_frontend* h, int code, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->err = buf;
    if (code == VIO_EDEVICE) h->poisoned = true;
  }
  return code;
}

#define HIP_CHECK(h, expr)                                                                          \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return fail((h), VIO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

int check_params(const vio_frontend_params* p, std::string& why) {
  if (p->struct_size != sizeof(vio_frontend_params)) return why = "struct_size mismatch", VIO_EINVAL;
  if (p->levels < 1 || p->levels > VIO_MAX_LEVELS) return why = "levels out of 1..6", VIO_EINVAL;
  if (p->gn_iters < 1 || p->gn_iters > 32) return why = "gn_iters out of 1..32", VIO_EINVAL;
  if (p->n_thresholds < 1 || p->n_thresholds > 4) return why = "n_thresholds out of 1..4", VIO_EINVAL;
  for (int i = 0; i < p->n_thresholds; ++i)
    if (p->thresholds[i] < 0 || p->thresholds[i] > 254) return why = "threshold out of 0..254", VIO_EINVAL;
  for (int i = 1; i < p->n_thresholds; ++i)
    if (p->thresholds[i] >= p->thresholds[i - 1]) return why = "thresholds must decrease", VIO_EINVAL;
  if (p->edge_margin < 4) return why = "edge_margin below 4", VIO_EINVAL;
  if (p->track_waves_per_cu < 0 || p->track_waves_per_cu > 64) return why = "track_waves_per_cu out of 0..64", VIO_EINVAL;
  if (p->track_block_waves != 0 && p->track_block_waves != 1 && p->track_block_waves != 2 &&
      p->track_block_waves != kTrackWaves)
    return why = "track_block_waves must be 0, 1, 2 or 4", VIO_EINVAL;
  if (p->flags & ~(VIO_FLAG_EAGER | VIO_FLAG_PLAIN)) return why = "unknown flag bits", VIO_EINVAL;
  if ((p->flags & VIO_FLAG_EAGER) && (p->flags & VIO_FLAG_PLAIN))
    return why = "VIO_FLAG_EAGER and VIO_FLAG_PLAIN exclude each other", VIO_EINVAL;
  if (p->pyr_tile != 0 && p->pyr_tile != 32 && p->pyr_tile != 64) return why = "pyr_tile must be 0, 32 or 64", VIO_EINVAL;
  if (p->stereo_mode != VIO_STEREO_SPECULATIVE && p->stereo_mode != VIO_STEREO_DEFERRED)
    return why = "stereo_mode must be VIO_STEREO_SPECULATIVE or VIO_STEREO_DEFERRED", VIO_EINVAL;
  if (!(p->fb_threshold > 0.f)) return why = "fb_threshold must be positive", VIO_EINVAL;
  if (p->k_per_cell < 1 || p->k_per_cell > kMaxPerCell) return why = "k_per_cell out of 1..8", VIO_EINVAL;
  if (p->init_mode != VIO_INIT_CONST_VEL && p->init_mode != VIO_INIT_LEARNED) return why = "init_mode", VIO_EINVAL;
  if (p->init_mode == VIO_INIT_LEARNED) {
    if (p->learned_levels < 1 || p->learned_levels > 3 || p->learned_levels > p->levels)
      return why = "learned_levels out of 1..min(3, levels)", VIO_EINVAL;
    if (p->learned_iters < 1 || p->learned_iters > 32) return why = "learned_iters out of 1..32", VIO_EINVAL;
  }
  if (p->pred_levels < 0 || p->pred_levels > p->levels) return why = "pred_levels out of 0..levels", VIO_EINVAL;
  if ((p->dev_alloc == nullptr) != (p->dev_free == nullptr)) return why = "set both dev_alloc and dev_free or neither", VIO_EINVAL;
  if (p->topology != VIO_TOPOLOGY_PAIRS && p->topology != VIO_TOPOLOGY_STAR)
    return why = "topology must be VIO_TOPOLOGY_PAIRS or VIO_TOPOLOGY_STAR", VIO_EINVAL;
  if (p->pred_levels > 0 && (p->pred_iters < 1 || p->pred_iters > 32))
    return why = "pred_iters out of 1..32", VIO_EINVAL;
  if (std::isnan(p->pred_rho)) return why = "pred_rho is NaN", VIO_EINVAL;
  if (p->learned_fb_levels < 0 || p->learned_fb_levels > p->levels)
    return why = "learned_fb_levels out of 0..levels", VIO_EINVAL;
  if (p->learned_fb_levels > 0 && (p->learned_fb_iters < 1 || p->learned_fb_iters > 32))
    return why = "learned_fb_iters out of 1..32", VIO_EINVAL;
  if (p->stereo_init != VIO_STEREO_INIT_PRIOR && p->stereo_init != VIO_STEREO_INIT_NEIGHBOUR)
    return why = "stereo_init must be VIO_STEREO_INIT_PRIOR or VIO_STEREO_INIT_NEIGHBOUR", VIO_EINVAL;
  if (p->stereo_init == VIO_STEREO_INIT_NEIGHBOUR &&
      (p->stereo_levels < 1 || p->stereo_levels > p->levels || p->stereo_iters < 1 || p->stereo_iters > 32))
    return why = "stereo_levels out of 1..levels or stereo_iters out of 1..32", VIO_EINVAL;
  if (p->track_parallel_fallback != 0 && p->track_parallel_fallback != 1)
    return why = "track_parallel_fallback must be 0 or 1", VIO_EINVAL;
  if (p->learned_block_waves != 0 && p->learned_block_waves != 4 && p->learned_block_waves != 8 &&
      p->learned_block_waves != 16)
    return why = "learned_block_waves must be 0, 4, 8 or 16", VIO_EINVAL;
  if (p->track_kp_per_wave < 0 || p->track_kp_per_wave > 2)
    return why = "track_kp_per_wave must be 0, 1 or 2", VIO_EINVAL;
  if (p->track_kp_per_wave == 2 && p->init_mode == VIO_INIT_LEARNED && p->learned_fused)
    return why = "track_kp_per_wave 2 needs learned_fused 0 (the fused learned stage runs one keypoint per wave)",
           VIO_EINVAL;
  if (p->learned_fused != 0 && p->learned_fused != 1) return why = "learned_fused must be 0 or 1", VIO_EINVAL;
  if (p->pyramid_stream < VIO_PYRAMID_SIGNAL || p->pyramid_stream > VIO_PYRAMID_SAME_STREAM)
    return why = "pyramid_stream must be VIO_PYRAMID_SIGNAL, _EVENT or _SAME_STREAM", VIO_EINVAL;
  return VIO_OK;
}

}  // namespace

extern "C" {

void vio_frontend_default_params(vio_frontend_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->struct_size = sizeof *p;
  p->levels = 4;
  p->gn_iters = 5;
  p->cell_size = 50;
  p->k_per_cell = 1;
  p->n_thresholds = 4;
  p->thresholds[0] = 40;
  p->thresholds[1] = 20;
  p->thresholds[2] = 10;
  p->thresholds[3] = 5;
  p->edge_margin = 8;
  p->max_keypoints = 300;
  p->fb_threshold = 0.3f;
  p->disparity0 = 32.5f;
  p->init_mode = VIO_INIT_CONST_VEL;
  p->learned_levels = 2;
  p->learned_iters = 3;
  p->learned_rho = 0.f;
  p->stereo_init = VIO_STEREO_INIT_PRIOR;
  p->stereo_levels = 2;
  p->stereo_iters = 3;
}

void vio_frontend_destroy(vio_frontend* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->pstream) (void)hipStreamSynchronize(h->pstream);
  for (auto& si : h->streams)
    for (Graphs& g : si.graph) g.destroy();
  for (Graphs& g : h->graph_all) g.destroy();
  if (h->arena) {
    if (h->P.dev_free) h->P.dev_free(h->arena, h->P.alloc_ctx);
    else (void)hipFree(h->arena);
  }
  for (FrameTable* f : h->h_frames)
    if (f) (void)hipHostFree(f);
  if (h->h_rec_count) (void)hipHostFree(h->h_rec_count);
  if (h->h_camstats) (void)hipHostFree(h->h_camstats);
  if (h->h_rec) (void)hipHostFree(h->h_rec);
  if (h->h_stage) (void)hipHostFree(h->h_stage);
  if (h->h_pred) (void)hipHostFree(h->h_pred);
  if (h->h_depth) (void)hipHostFree(h->h_depth);
  for (auto& pr : h->ev)
    for (hipEvent_t& e : pr)
      if (e) (void)hipEventDestroy(e);
  for (int slot = 0; slot < kInFlight; ++slot) {
    if (h->ev_pyr[slot]) (void)hipEventDestroy(h->ev_pyr[slot]);
  }
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  // the streams were synchronized above: the signal holds its last value
  if (h->pyr_sig) signal_release(h->device, h->pyr_sig, h->pyr_epoch);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  if (h->pstream && h->pstream != h->stream) (void)hipStreamDestroy(h->pstream);
  delete h;
}

static int create_impl(vio_frontend* h, const vio_stream_desc* sd, int32_t n_streams) {
  const vio_frontend_params& P = h->P;
  // ---- layout (host only) ---------------------------------------------------
  int n_cams = 0;
  for (int s = 0; s < n_streams; ++s) n_cams += sd[s].n_cameras;
  h->cams.resize(n_cams);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = round_up(off + bytes, kAlign);
    return o;
  };
  struct CamOffs {
    size_t lvl[kPyrSlots][kMaxLevels], state[2], res, res_fb, keys[kPyrSlots], sres, rec, mask, pairs[2];
  };
  // parallel fallbacks exist where a temporal track may first run a short budget
  const bool par_fb = P.track_parallel_fallback && (P.init_mode == VIO_INIT_LEARNED || P.pred_levels > 0);
  std::vector<CamOffs> co(n_cams);
  int cam = 0, tiles = 0, rows_total = 0, items = 0;
  size_t rec_total = 0, stage = 0;
  for (int s = 0; s < n_streams; ++s) {
    StreamInfo si;
    si.first_cam = cam;
    si.n_cams = sd[s].n_cameras;
    si.w = sd[s].width;
    si.h = sd[s].height;
    si.cap = sd[s].max_keypoints > 0 ? sd[s].max_keypoints : P.max_keypoints;
    si.cell = sd[s].cell_size > 0 ? sd[s].cell_size : P.cell_size;
    si.tile_begin = tiles;
    si.rec_off = rec_total;
    si.seg_begin = (int)h->segs.size();
    si.item_begin = items;
    for (int k = 0; k < si.n_cams; ++k, ++cam) {
      CamDesc& c = h->cams[cam];
      std::memset(&c, 0, sizeof c);
      c.w = si.w;
      c.h = si.h;
      c.levels = P.levels;
      c.cap = si.cap;
      c.cell = si.cell;
      c.ncx = (si.w + si.cell - 1) / si.cell;
      c.ncy = (si.h + si.cell - 1) / si.cell;
      c.ncells = c.ncx * c.ncy;
      c.kcell = P.k_per_cell;
      c.nslots = c.ncells * c.kcell;
      // groups: mono, stereo pairs (0,1), (2,3), or a star rig 0 -> 1, 2, 3
      const bool star = si.n_cams == 4 && P.topology == VIO_TOPOLOGY_STAR;
      const int group = si.n_cams == 1 ? 1 : (star ? 4 : 2);
      c.detect = k % group == 0 ? 1 : 0;
      c.n_targets = c.detect ? group - 1 : 0;
      c.stream = s;
      c.local = k;
      c.tiles_x = (si.w + h->tile - 1) / h->tile;
      c.tiles_y = (si.h + h->tile - 1) / h->tile;
      c.tile_begin = tiles;
      tiles += c.tiles_x * c.tiles_y;
      for (int l = 0; l < P.levels; ++l) {
        c.pitch[l] = (int)round_up((size_t)(si.w >> l), 64);
        // one guard row: the tracker's template window reads up to one row and
        // one column past a level (with weight 0)
        for (int ps = 0; ps < kPyrSlots; ++ps)
          co[cam].lvl[ps][l] = take((size_t)c.pitch[l] * (size_t)((si.h >> l) + 1));
      }
      for (int par = 0; par < 2; ++par) co[cam].state[par] = take(sizeof(Kp) * si.cap);
      co[cam].res = take(sizeof(TrackRes) * si.cap);
      if (par_fb) co[cam].res_fb = take(sizeof(TrackRes) * si.cap);
      if (c.detect) {
        for (int ps = 0; ps < kPyrSlots; ++ps) co[cam].keys[ps] = take(sizeof(uint32_t) * c.nslots);
        co[cam].sres = take(sizeof(TrackRes) * c.nslots * std::max(1, c.n_targets));
        co[cam].mask = take((size_t)si.w * si.h);
      } else if (P.stereo_init == VIO_STEREO_INIT_NEIGHBOUR && group > 1) {
        for (int par = 0; par < 2; ++par) co[cam].pairs[par] = take(sizeof(float4) * si.cap);
      }
      c.rec_cap = 2 * si.cap;
      c.row_off = rows_total;
      rows_total += si.cap;
      co[cam].rec = rec_total;
      rec_total += c.rec_cap;
      stage += (size_t)si.w * si.h;
    }
    // tracking work items: stereo matches of the left cameras' cell winners
    // (one per key slot) first (they run the full budget), then the temporal
    // tracks of every camera
    for (int k = 0; k < si.n_cams; ++k) {
      const int cc = si.first_cam + k;
      const CamDesc& cd = h->cams[cc];
      if (cd.n_targets > 0) {
        const int n = cd.nslots * cd.n_targets;
        h->segs.push_back({cc, kModeStereo, items, n});
        items += n;
        si.st_segs += 1;
        si.st_items += n;
      }
    }
    for (int k = 0; k < si.n_cams * (par_fb ? 2 : 1); ++k) {
      // temporal tracks of every camera, then (parallel fallbacks) their fallbacks
      h->segs.push_back({si.first_cam + k % si.n_cams, k < si.n_cams ? kModeTemporal : kModeFallback, items, si.cap});
      items += si.cap;
    }
    si.n_segs = (int)h->segs.size() - si.seg_begin;
    si.n_items = items - si.item_begin;
    si.n_tiles = tiles - si.tile_begin;
    si.rec_n = rec_total - si.rec_off;
    h->streams.push_back(si);
    h->stream_cams.push_back(si.first_cam);
    h->stream_cams.push_back(si.n_cams);
  }
  // the batched step's order: every stream's stereo items, then every temporal item
  {
    int at = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (const TrackSeg& g : h->segs)
        if ((g.mode == kModeStereo) == (pass == 0)) {
          h->segs_all.push_back({g.cam, g.mode, at, g.count});
          at += g.count;
        }
  }
  h->total_tiles = tiles;
  h->rec_total = rec_total;
  h->pred_cap = 0;
  for (auto& c : h->cams) h->pred_cap += c.cap;
  const size_t o_cams = take(sizeof(CamDesc) * n_cams);
  const size_t o_frame = take(kInFlight * sizeof(FrameTable));
  const size_t o_cnt = take(sizeof(Counters));
  const size_t o_segs = take(sizeof(TrackSeg) * h->segs.size());
  const size_t o_segs_all = take(sizeof(TrackSeg) * h->segs_all.size());
  const size_t o_sc = take(sizeof(int) * h->stream_cams.size());
  const size_t o_pred = take(sizeof(Prediction) * std::max(1, h->pred_cap));
  const size_t o_depth = take(sizeof(KpDepth) * std::max(1, h->pred_cap));
  size_t o_feat = 0, o_guess = 0, o_P = 0, o_W1 = 0, o_W2 = 0, o_W2t = 0, o_W3 = 0;
  if (h->learned) {
    const int rows = (rows_total + 15) / 16 * 16;
    o_feat = take(sizeof(float) * 32 * rows);
    o_guess = take(sizeof(float) * 3 * rows);
    o_P = take(sizeof(float) * VIO_MLP_NPARAM);
    o_W1 = take(2 * 128 * 32);
    o_W2 = take(2 * 128 * 128);
    o_W2t = take(2 * 128 * 128);
    o_W3 = take(2 * 3 * 128);
  }
  const size_t arena_bytes = off;

  // ---- device ---------------------------------------------------------------
  if (const char* fi = std::getenv("VIO_FAULT_INJECT")) {
    if (!std::strcmp(fi, "alloc")) return fail(h, VIO_ENOMEM, "injected allocation failure");
    if (!std::strcmp(fi, "device")) h->fault_device = true;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(h, VIO_EDEVICE, "no HIP device");
  HIP_CHECK(h, hipGetDevice(&h->device));
  HIP_CHECK(h, hipDeviceGetAttribute(&h->n_cus, hipDeviceAttributeMultiprocessorCount, h->device));
  int lds_max = 0;
  HIP_CHECK(h, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
  const size_t lds_need = pyr_detect_lds_bytes(P.levels, h->tile);
  if (lds_need == 0 || lds_need > (size_t)lds_max)
    return fail(h, VIO_EUNSUPPORTED, "%d levels with %d-pixel tiles need %zu bytes of LDS per workgroup, the device "
                "offers %d", P.levels, h->tile, lds_need, lds_max);
  if (P.dev_alloc) {
    h->arena = P.dev_alloc(arena_bytes, P.alloc_ctx);
    if (!h->arena) return fail(h, VIO_ENOMEM, "caller's allocator: device arena of %zu bytes", arena_bytes);
    if (reinterpret_cast<uintptr_t>(h->arena) % kAlign != 0) {
      P.dev_free(h->arena, P.alloc_ctx);
      h->arena = nullptr;
      return fail(h, VIO_EINVAL, "caller's allocator returned memory not aligned to %zu bytes", kAlign);
    }
  } else if (hipMalloc(&h->arena, arena_bytes) != hipSuccess) {
    h->arena = nullptr;
    return fail(h, VIO_ENOMEM, "device arena of %zu bytes", arena_bytes);
  }
  HIP_CHECK(h, hipMemset(h->arena, 0, arena_bytes));
  uint8_t* base = static_cast<uint8_t*>(h->arena);
  for (int c = 0; c < n_cams; ++c) {
    CamDesc& d = h->cams[c];
    for (int l = 0; l < P.levels; ++l)
      for (int ps = 0; ps < kPyrSlots; ++ps) d.lvl[ps][l] = base + co[c].lvl[ps][l];
    for (int par = 0; par < 2; ++par) d.state[par] = reinterpret_cast<Kp*>(base + co[c].state[par]);
    d.res = reinterpret_cast<TrackRes*>(base + co[c].res);
    d.res_fb = par_fb ? reinterpret_cast<TrackRes*>(base + co[c].res_fb) : nullptr;
    if (d.detect) {
      for (int ps = 0; ps < kPyrSlots; ++ps) d.keys[ps] = reinterpret_cast<uint32_t*>(base + co[c].keys[ps]);
      d.sres = reinterpret_cast<TrackRes*>(base + co[c].sres);
      d.mask = reinterpret_cast<const uint8_t*>(base + co[c].mask);
    } else if (co[c].pairs[0]) {
      for (int par = 0; par < 2; ++par) d.pairs[par] = reinterpret_cast<float4*>(base + co[c].pairs[par]);
    }
  }
  h->d_cams = reinterpret_cast<CamDesc*>(base + o_cams);
  for (int slot = 0; slot < kInFlight; ++slot)
    h->d_frames[slot] = reinterpret_cast<FrameTable*>(base + o_frame) + slot;
  h->d_frame = h->d_frames[0];
  h->d_cnt = reinterpret_cast<Counters*>(base + o_cnt);
  h->d_segs = reinterpret_cast<TrackSeg*>(base + o_segs);
  h->d_segs_all = reinterpret_cast<TrackSeg*>(base + o_segs_all);
  h->d_stream_cams = reinterpret_cast<int*>(base + o_sc);
  h->d_pred = reinterpret_cast<Prediction*>(base + o_pred);
  h->d_depth = reinterpret_cast<KpDepth*>(base + o_depth);
  h->K.assign(n_cams, vio_pinhole{0.f, 0.f, 0.f, 0.f});
  h->kb.assign(n_cams, vio_kb4{});
  h->kb4.assign(n_cams, 0);
  if (h->learned) {
    h->d_feat = reinterpret_cast<float*>(base + o_feat);
    h->d_guess = reinterpret_cast<float*>(base + o_guess);
    h->mlp.P = reinterpret_cast<float*>(base + o_P);
    h->mlp.W1b = reinterpret_cast<uint16_t*>(base + o_W1);
    h->mlp.W2b = reinterpret_cast<uint16_t*>(base + o_W2);
    h->mlp.W2tb = reinterpret_cast<uint16_t*>(base + o_W2t);
    h->mlp.W3b = reinterpret_cast<uint16_t*>(base + o_W3);
  }
  HIP_CHECK(h, hipMemcpy(h->d_segs, h->segs.data(), sizeof(TrackSeg) * h->segs.size(), hipMemcpyHostToDevice));
  HIP_CHECK(h, hipMemcpy(h->d_segs_all, h->segs_all.data(), sizeof(TrackSeg) * h->segs_all.size(),
                         hipMemcpyHostToDevice));
  HIP_CHECK(h, hipMemcpy(h->d_stream_cams, h->stream_cams.data(), sizeof(int) * h->stream_cams.size(),
                         hipMemcpyHostToDevice));
  // pinned host buffers; records and their counts are written by the
  // selection kernel through the device mapping of h_rec / h_rec_count
  h->stage_bytes = stage;
  bool host_ok = true;
  for (FrameTable*& f : h->h_frames) host_ok = host_ok && hipHostMalloc((void**)&f, sizeof(FrameTable)) == hipSuccess;
  if (!host_ok ||
      hipHostMalloc((void**)&h->h_rec_count, sizeof(int32_t) * kRecSlots * n_cams) != hipSuccess ||
      hipHostMalloc((void**)&h->h_camstats, sizeof(int32_t) * kCamStats * kRecSlots * n_cams) != hipSuccess ||
      hipHostMalloc((void**)&h->h_rec, sizeof(vio_track) * kRecSlots * rec_total) != hipSuccess ||
      hipHostMalloc((void**)&h->h_stage, kInFlight * stage) != hipSuccess ||
      hipHostMalloc((void**)&h->h_pred, sizeof(Prediction) * kInFlight * std::max(1, h->pred_cap)) != hipSuccess ||
      hipHostMalloc((void**)&h->h_depth, sizeof(KpDepth) * kInFlight * std::max(1, h->pred_cap)) != hipSuccess)
    return fail(h, VIO_ENOMEM, "pinned host buffers");
  for (FrameTable* f : h->h_frames) std::memset(f, 0, sizeof(FrameTable));
  h->h_frame = h->h_frames[0];
  for (int slot = 0; slot < kInFlight; ++slot)
    HIP_CHECK(h, hipHostGetDevicePointer((void**)&h->hm_frames[slot], h->h_frames[slot], 0));
  h->hm_frame = h->hm_frames[0];
  std::memset(h->h_rec_count, 0, sizeof(int32_t) * kRecSlots * n_cams);
  std::memset(h->h_camstats, 0, sizeof(int32_t) * kCamStats * kRecSlots * n_cams);
  vio_track* rec_dev = nullptr;
  int32_t *cnt_dev = nullptr, *stats_dev = nullptr;
  HIP_CHECK(h, hipHostGetDevicePointer((void**)&rec_dev, h->h_rec, 0));
  HIP_CHECK(h, hipHostGetDevicePointer((void**)&cnt_dev, h->h_rec_count, 0));
  HIP_CHECK(h, hipHostGetDevicePointer((void**)&stats_dev, h->h_camstats, 0));
  for (int c = 0; c < n_cams; ++c) {
    for (int rs = 0; rs < kRecSlots; ++rs) {
      h->cams[c].rec[rs] = rec_dev + rs * rec_total + co[c].rec;
      h->cams[c].rec_count_out[rs] = cnt_dev + rs * n_cams + c;
      h->cams[c].stats_out[rs] = stats_dev + (size_t)kCamStats * (rs * n_cams + c);
    }
    h->rec_host_off.push_back(co[c].rec);
  }
  HIP_CHECK(h, hipMemcpy(h->d_cams, h->cams.data(), sizeof(CamDesc) * n_cams, hipMemcpyHostToDevice));
  HIP_CHECK(h, hipStreamCreate(&h->stream));
  // VIO_PYRAMID_SAME_STREAM: the pyramid runs on the launch stream, in order
  if (h->P.pyramid_stream == VIO_PYRAMID_SAME_STREAM) h->pstream = h->stream;
  else HIP_CHECK(h, hipStreamCreate(&h->pstream));
  for (int slot = 0; slot < kInFlight; ++slot) {
    HIP_CHECK(h, hipEventCreateWithFlags(&h->ev_pyr[slot], hipEventDisableTiming));
  }
  HIP_CHECK(h, hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
  if (h->P.pyramid_stream != VIO_PYRAMID_SIGNAL || !signal_acquire(h->device, &h->pyr_sig, &h->pyr_epoch))
    h->pyr_sig = nullptr;
  for (auto& pr : h->ev)
    for (hipEvent_t& e : pr) HIP_CHECK(h, hipEventCreate(&e));
  for (auto& pr : h->kev)
    for (hipEvent_t& e : pr) HIP_CHECK(h, hipEventCreate(&e));
  return VIO_OK;
}

int vio_frontend_create(const vio_stream_desc* streams, int32_t n_streams, const vio_frontend_params* params,
                        vio_frontend** out) {
  if (!streams || !params || !out || n_streams < 1) return VIO_EINVAL;
  *out = nullptr;
  std::string why;
  const int pc = check_params(params, why);
  if (pc != VIO_OK) return pc;
  int n_cams = 0;
  for (int s = 0; s < n_streams; ++s) {
    const vio_stream_desc& d = streams[s];
    if (d.n_cameras != 1 && d.n_cameras != 2 && d.n_cameras != 4) return VIO_EINVAL;
    if (d.width < 16 || d.height < 16 || d.width > 4096 || d.height > 4096) return VIO_EINVAL;
    if ((int64_t)d.width * d.height >= (1 << 24)) return VIO_EINVAL;
    if ((d.width >> (params->levels - 1)) < 2 || (d.height >> (params->levels - 1)) < 2) return VIO_EINVAL;
    const int cap = d.max_keypoints > 0 ? d.max_keypoints : params->max_keypoints;
    const int cell = d.cell_size > 0 ? d.cell_size : params->cell_size;
    if (cap < 1 || cap > kMaxCellsAbi || cell < 4) return VIO_EINVAL;
    if ((int64_t)((d.width + cell - 1) / cell) * ((d.height + cell - 1) / cell) > kMaxCellsAbi) return VIO_EINVAL;
    n_cams += d.n_cameras;
  }
  if (n_cams > kMaxCams) return VIO_EINVAL;
  auto* h = new (std::nothrow) vio_frontend();
  if (!h) return VIO_ENOMEM;
  h->P = *params;
  h->eager = (params->flags & VIO_FLAG_EAGER) != 0;
  h->plain = (params->flags & VIO_FLAG_PLAIN) != 0;
  h->learned = params->init_mode == VIO_INIT_LEARNED;
  h->tile = params->pyr_tile ? params->pyr_tile : kTileDefault;
  const int rc = create_impl(h, streams, n_streams);
  if (rc != VIO_OK) {
    vio_frontend_destroy(h);
    return rc;
  }
  *out = h;
  return VIO_OK;
}

const char* vio_frontend_last_error(const vio_frontend* h) { return h ? h->err.c_str() : "null handle"; }

static Tuning tuning(const vio_frontend* h) {
  Tuning t;
  t.levels = h->P.levels;
  t.iters = h->P.gn_iters;
  t.fb_threshold = h->P.fb_threshold;
  t.disparity0 = h->P.disparity0;
  t.tmin = h->P.thresholds[h->P.n_thresholds - 1];
  t.margin = h->P.edge_margin;
  t.learned = h->learned ? 1 : 0;
  t.llevels = h->P.learned_levels;
  t.liters = h->P.learned_iters;
  t.rho = h->P.learned_rho;
  t.guess = h->d_guess;
  t.deferred = h->P.stereo_mode == VIO_STEREO_DEFERRED;
  t.depths = h->d_depth;
  t.plevels = h->P.pred_levels;
  t.piters = h->P.pred_iters;
  t.prho = h->P.pred_rho;
  t.fblevels = h->P.learned_fb_levels > 0 ? h->P.learned_fb_levels : h->P.levels;
  t.fbiters = h->P.learned_fb_levels > 0 ? h->P.learned_fb_iters : h->P.gn_iters;
  t.stereo_nb = h->P.stereo_init == VIO_STEREO_INIT_NEIGHBOUR ? 1 : 0;
  t.slevels = h->P.stereo_levels;
  t.siters = h->P.stereo_iters;
  t.par_fb = h->cams.empty() || h->cams[0].res_fb == nullptr ? 0 : 1;
  t.fused = h->learned && h->P.learned_fused ? 1 : 0;
  t.feat = h->d_feat;
  t.W1b = h->mlp.W1b;
  t.W2b = h->mlp.W2b;
  t.W3b = h->mlp.W3b;
  t.mlpP = h->mlp.P;
  return t;
}

static LaunchSet stream_set(const vio_frontend* h, int s) {
  const StreamInfo& si = h->streams[s];
  return {si.first_cam, si.first_cam + si.n_cams, si.tile_begin, si.n_tiles, si.seg_begin, si.n_segs,
          si.item_begin, si.n_items, s, 1, false, si.st_segs, si.st_items};
}

static LaunchSet all_set(const vio_frontend* h) {
  const StreamInfo& last = h->streams.back();
  int st_segs = 0, st_items = 0;
  for (const StreamInfo& si : h->streams) st_segs += si.st_segs, st_items += si.st_items;
  return {0, (int)h->cams.size(), 0, h->total_tiles, 0, (int)h->segs_all.size(), 0, last.item_begin + last.n_items, 0,
          (int)h->streams.size(), true, st_segs, st_items};
}

// Tracking launch over segments [seg_begin, seg_begin + n_segs) of the set's
// table and items [item_begin, item_begin + n_items).
// `queue`: the frame's work-queue counter this launch's persistent grid pops
// (each tracking launch of a frame has its own).
static hipError_t track_range(vio_frontend* h, const LaunchSet& ls, int seg_begin, int n_segs, int item_begin,
                              int n_items, const Tuning& tune, int queue, hipStream_t st) {
  return launch_track(h->d_cams, h->d_frame, h->d_cnt, (ls.all ? h->d_segs_all : h->d_segs) + seg_begin, n_segs,
                      item_begin, n_items, h->d_pred, tune,
                      TrackShape{h->P.track_waves_per_cu,
                                 h->P.track_block_waves ? h->P.track_block_waves : kTrackWaves, h->n_cus, queue,
                                 h->P.track_kp_per_wave ? h->P.track_kp_per_wave : 1},
                      st);
}

// Enqueues one step of a frame of the launch set on `st`: 0 = frame table
// copy, 1 = pyramid+detector, 2 = tracker, 3 = selection (deferred stereo:
// selection, stereo tracker, selection), 4 = learned mode's features and
// network. Nothing enqueued changes between frames (per-frame inputs live in
// the frame table), so the sequence can be captured once.
// `timed` attaches each kernel's start/stop events to its dispatch.
static hipError_t enqueue_stage(vio_frontend* h, const LaunchSet& ls, hipStream_t st, int stage, bool timed) {
  const Tuning tune = tuning(h);
  auto timing = [&](int k) {
    tl_timing = timed ? KernelTiming{h->kev[k][0], h->kev[k][1]} : KernelTiming{};
    if (timed) h->kran[k] = true;
  };
  struct Reset {
    ~Reset() { tl_timing = KernelTiming{}; }
  } reset;
  hipError_t e;
  if (stage == 1) {
    // the pyramid kernel reads the frame's table from its pinned host slot and
    // copies it to the device table the later kernels read
    timing(kKernPyr);
    return launch_pyr_detect_range(h->d_cams, h->hm_frame, h->d_frame,
                                   (int)(offsetof(FrameTable, cam) + sizeof(FrameCam) * h->cams.size()), ls.cam_begin,
                                   ls.cam_end, ls.tile_begin, ls.n_tiles, tune.levels, h->tile, tune.tmin, tune.margin,
                                   st);
  }
  if (stage == 4) {
    // the features of the previous keypoints and the network's guesses in one
    // launch; the tracker reads the guesses
    timing(kKernFeatures);
    // (it runs beside the pyramid kernel, which copies the frame's table to
    // the device: it reads the pinned host table)
    return launch_learn(h->d_cams, h->hm_frame, h->d_cnt, h->cams.data(), ls.cam_begin, ls.cam_end, h->mlp,
                        h->d_feat, h->d_guess, h->P.learned_block_waves ? h->P.learned_block_waves : kLearnWavesDefault,
                        st);
  }
  if (stage == 2) {
    // speculative: every item; deferred: the temporal items only (they follow the stereo ones)
    timing(kKernTrack);
    const int s0 = tune.deferred ? ls.st_segs : 0, i0 = tune.deferred ? ls.st_items : 0;
    return track_range(h, ls, ls.seg_begin + s0, ls.n_segs - s0, ls.item_begin + i0, ls.n_items - i0, tune, 0, st);
  }
  timing(kKernSelect);
  const int* sc = h->d_stream_cams + 2 * ls.stream_begin;
  if (!tune.deferred) return launch_select(h->d_cams, h->d_frame, h->d_cnt, sc, ls.n_streams, kSelectAll, tune, st);
  // deferred stereo: select, match the selected detections, accept the matches
  if ((e = launch_select(h->d_cams, h->d_frame, h->d_cnt, sc, ls.n_streams, kSelectLeft, tune, st))) return e;
  if (ls.st_items > 0) {
    timing(kKernTrackStereo);
    if ((e = track_range(h, ls, ls.seg_begin, ls.st_segs, ls.item_begin, ls.st_items, tune, 1, st))) return e;
  }
  timing(kKernSelectRight);
  return launch_select(h->d_cams, h->d_frame, h->d_cnt, sc, ls.n_streams, kSelectRight, tune, st);
}

// A frame runs on two streams. The pyramid stream builds the pyramid and
// detections (its kernel copies the slot's frame table to the device) and
// then raises its signal; the launch stream runs the learned stage (its
// inputs are the previous frame's keypoints and level 0, so it runs beside
// the pyramid) and, once the signal reaches the frame's count, the tracker
// and the selection. The pyramid slots rotate over kPyrSlots frames, so the
// pyramids of the later frames in flight can run beside this frame's
// tracking.
static hipError_t enqueue_pyr_part(vio_frontend* h, const LaunchSet& ls, int slot, bool timed, hipStream_t st) {
  hipError_t e;
  if ((e = enqueue_stage(h, ls, h->pstream, 1, timed))) return e;
  if (h->pstream == st) return hipSuccess;  // the launch stream itself: stream order suffices
  if (h->pyr_sig) return hipStreamWriteValue32(h->pstream, h->pyr_sig, ++h->pyr_epoch, 0);
  return hipEventRecord(h->ev_pyr[slot], h->pstream);
}

// The launch stream waits for the pyramid part of the frame just enqueued.
static hipError_t wait_pyr_part(vio_frontend* h, hipStream_t st, int slot) {
  if (h->pstream == st) return hipSuccess;
  if (h->pyr_sig) return hipStreamWaitValue32(st, h->pyr_sig, h->pyr_epoch, hipStreamWaitValueGte, 0xFFFFFFFFu);
  return hipStreamWaitEvent(st, h->ev_pyr[slot], 0);
}

static hipError_t enqueue_track_part(vio_frontend* h, const LaunchSet& ls, hipStream_t st, bool timed) {
  hipError_t e;
  if ((e = enqueue_stage(h, ls, st, 2, timed))) return e;
  return enqueue_stage(h, ls, st, 3, timed);
}

// Captures a slot's learned stage and tracking part on first use; a capture
// failure switches the handle to eager launches for good.
static void ensure_graph(vio_frontend* h, const LaunchSet& ls, Graphs* gr) {
  if (h->eager || h->plain || gr->any()) return;
  // part 1: learned stage, 2: tracking part
  auto capture = [&](hipGraphExec_t* out, int part) {
    hipStream_t cs = h->stream;
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      const hipError_t e = part == 1 ? enqueue_stage(h, ls, cs, 4, false) : enqueue_track_part(h, ls, cs, false);
      ok = hipStreamEndCapture(cs, &g) == hipSuccess && e == hipSuccess && g;
    }
    if (ok) ok = hipGraphInstantiate(out, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    return ok;
  };
  bool ok = capture(&gr->trk, 2);
  if (ok && h->learned && !h->P.learned_fused) ok = capture(&gr->learn, 1);
  gr->captured = ok;
  if (!ok) {
    gr->destroy();
    h->eager = true;
    (void)hipGetLastError();
  }
}

static int complete_all(vio_frontend* h);

// Submits one frame of a launch set whose inputs are in the current slot's
// frame table (h_frame) without waiting: the slot's captured graph, or eager
// launches with per-kernel timing. The next slot becomes the staging slot.
// At most two submissions are outstanding; eager ones are completed before
// the next submission (their kernel timing events are shared).
static int submit_set(vio_frontend* h, const LaunchSet& ls, Graphs* gr, hipStream_t st) {
  if (h->n_pend == kInFlight) return fail(h, VIO_ESTATE, "%d frames in flight: call vio_frontend_wait first", kInFlight);
  if (h->pyr_sig && h->pyr_epoch >= 0x80000000u) {
    // long before the 32-bit count could wrap: drain, then restart it at zero
    const int rc = complete_all(h);
    if (rc != VIO_OK) return rc;
    HIP_CHECK(h, hipStreamSynchronize(h->pstream));
    HIP_CHECK(h, hipMemset(h->pyr_sig, 0, 8));
    h->pyr_epoch = 0;
  }
  const int slot = (int)(h->sub % kInFlight);
  h->d_frame = h->d_frames[slot];
  h->hm_frame = h->hm_frames[slot];
  ensure_graph(h, ls, &gr[slot]);
  const bool graphed = gr[slot].any();
  // eager launches time each kernel with shared events: one frame at a time
  const bool timed = !graphed && !h->plain;
  if (timed && h->n_pend > 0) {
    const int rc = complete_all(h);
    if (rc != VIO_OK) return rc;
  }
  if (timed)
    for (bool& r : h->kran) r = false;
  if (st != h->stream) {
    // a caller's stream: the pyramid reads images produced there
    HIP_CHECK(h, hipEventRecord(h->ev_in, st));
    HIP_CHECK(h, hipStreamWaitEvent(h->pstream, h->ev_in, 0));
  }
  // the frame's start timestamp (last_gpu_ms), not taken with plain launches
  if (!h->plain) HIP_CHECK(h, hipEventRecord(h->ev[slot][0], h->pstream));
  HIP_CHECK(h, enqueue_pyr_part(h, ls, slot, timed, st));
  if (h->learned && !h->P.learned_fused) {
    // the learned stage's inputs are the previous frame's (ordered before it
    // on this stream) and the pinned frame table: it starts at once
    if (graphed) HIP_CHECK(h, hipGraphLaunch(gr[slot].learn, st));
    else HIP_CHECK(h, enqueue_stage(h, ls, st, 4, timed));
  }
  HIP_CHECK(h, wait_pyr_part(h, st, slot));
  if (graphed) HIP_CHECK(h, hipGraphLaunch(gr[slot].trk, st));
  else HIP_CHECK(h, enqueue_track_part(h, ls, st, timed));
  HIP_CHECK(h, hipEventRecord(h->ev[slot][1], st));
  for (int s = ls.stream_begin; s < ls.stream_begin + ls.n_streams; ++s)
    if (h->h_frame->cam[h->streams[s].first_cam].active) h->streams[s].frames += 1;
  h->pend[(h->pend_head + h->n_pend) % kInFlight] = vio_frontend::Pending{ls, graphed, slot};
  h->n_pend += 1;
  h->sub += 1;
  // a stream staged for a later step but not in this submission keeps its
  // staged inputs in the next slot's table
  FrameTable* next = h->h_frames[h->sub % kInFlight];
  for (int s = 0; s < (int)h->streams.size(); ++s) {
    const StreamInfo& si = h->streams[s];
    if (!si.staged || (s >= ls.stream_begin && s < ls.stream_begin + ls.n_streams)) continue;
    for (int k = 0; k < si.n_cams; ++k) next->cam[si.first_cam + k] = h->h_frame->cam[si.first_cam + k];
  }
  h->h_frame = next;
  return VIO_OK;
}

// Waits for the oldest outstanding submission and takes its statistics: the
// frame's device time, eager launches' kernel times, and the selection
// kernel's per-camera counts (no pass over the records).
static int complete_oldest(vio_frontend* h) {
  if (h->n_pend == 0) return fail(h, VIO_ESTATE, "no frame in flight");
  const vio_frontend::Pending p = h->pend[h->pend_head];
  h->pend_head = (h->pend_head + 1) % kInFlight;
  h->n_pend -= 1;
  HIP_CHECK(h, hipEventSynchronize(h->ev[p.slot][1]));
  const FrameTable* ft = h->h_frames[p.slot];
  float ms = -1.f;
  if (!h->plain) HIP_CHECK(h, hipEventElapsedTime(&ms, h->ev[p.slot][0], h->ev[p.slot][1]));
  float km[kKernels];
  for (int k = 0; k < kKernels; ++k) {
    km[k] = -1.f;
    if (!p.graphed && h->kran[k]) HIP_CHECK(h, hipEventElapsedTime(&km[k], h->kev[k][0], h->kev[k][1]));
  }
  // deferred stereo matching: the tracker and selection run twice per frame
  h->stats.last_stage_ms[0] = km[kKernPyr];
  h->stats.last_stage_ms[1] = km[kKernTrack] + (km[kKernTrackStereo] > 0.f ? km[kKernTrackStereo] : 0.f);
  h->stats.last_stage_ms[2] = km[kKernSelect] + (km[kKernSelectRight] > 0.f ? km[kKernSelectRight] : 0.f);
  h->stats.last_learned_ms[0] = km[kKernFeatures];
  h->stats.last_learned_ms[1] = km[kKernMlp];
  h->stats.last_gpu_ms = ms;
  h->stats.frames += 1;
  const int n_cams = (int)h->cams.size();
  int tr = 0, lost = 0, det = 0, mat = 0, fb = 0;
  for (int c = p.ls.cam_begin; c < p.ls.cam_end; ++c) {
    if (!ft->cam[c].active) continue;
    const int32_t* st = h->h_camstats + (size_t)kCamStats * (ft->cam[c].rec_slot * n_cams + c);
    tr += st[kStatTracked];
    lost += st[kStatLost];
    det += st[kStatDetected];
    mat += st[kStatMatched];
    fb += st[kStatFallback];
  }
  h->stats.last_fallback = fb;
  h->stats.last_tracked = tr;
  h->stats.last_lost = lost;
  h->stats.last_detected = det;
  h->stats.last_matched = mat;
  for (int s = p.ls.stream_begin; s < p.ls.stream_begin + p.ls.n_streams; ++s)
    if (ft->cam[h->streams[s].first_cam].active) h->streams[s].done += 1;
  return VIO_OK;
}

static int complete_all(vio_frontend* h) {
  while (h->n_pend > 0) {
    const int rc = complete_oldest(h);
    if (rc != VIO_OK) return rc;
  }
  return VIO_OK;
}

// Runs one frame of a launch set and waits for it (and for anything submitted
// before it).
static int run_set(vio_frontend* h, const LaunchSet& ls, Graphs* gr, hipStream_t st) {
  int rc = complete_all(h);
  if (rc == VIO_OK) rc = submit_set(h, ls, gr, st);
  if (rc == VIO_OK) rc = complete_all(h);
  return rc;
}

// Runs one frame of stream s whose level-0 sources are already in h_frame.
static int run_frame(vio_frontend* h, int s, hipStream_t st) {
  return run_set(h, stream_set(h, s), h->streams[s].graph, st);
}

static int check_push(vio_frontend* h, int32_t s, int64_t t_ns) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (h->learned && !h->mlp_ready) return fail(h, VIO_ESTATE, "learned init: call vio_frontend_set_mlp first");
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (si.frames > 0 && t_ns <= si.last_t) return fail(h, VIO_ESTATE, "timestamps must increase");
  if (h->n_pend == kInFlight) return fail(h, VIO_ESTATE, "%d frames in flight: call vio_frontend_wait first", kInFlight);
  if (h->fault_device) return fail(h, VIO_EDEVICE, "injected device failure");
  return VIO_OK;
}

static void fill_stream(vio_frontend* h, int s) {
  const StreamInfo& si = h->streams[s];
  const int par = (int)(si.frames & 1);
  for (int k = 0; k < si.n_cams; ++k) {
    FrameCam& f = h->h_frame->cam[si.first_cam + k];
    f.parity = par;
    f.pyr = (int)(si.frames % kPyrSlots);
    f.pyr_prev = (int)((si.frames + kPyrSlots - 1) % kPyrSlots);
    f.rec_slot = (int)(si.frames % kRecSlots);
    f.has_prev = si.frames > 0;
    f.active = 1;
    f.n_pred = 0;
    f.pred_off = 0;
    f.has_motion = 0;
    f.n_depth = 0;
    f.depth_off = 0;
  }
}

// Moves the stream's pending camera motion (vio_frontend_set_motion) into
// its cameras' frame-table entries and queues the per-keypoint inverse depths'
// upload on `st` (each camera's list at its row offset); the pending motion is
// consumed by this frame.
static int stage_motion(vio_frontend* h, int s, hipStream_t st) {
  StreamInfo& si = h->streams[s];
  if (si.motion.empty()) return VIO_OK;
  for (const vio_camera_motion& m : si.motion) {
    const int c = si.first_cam + m.camera;
    FrameCam& f = h->h_frame->cam[c];
    const CamDesc& cd = h->cams[c];
    const vio_pinhole& K = h->K[c];
    f.has_motion = 1;
    f.K[0] = K.fx;
    f.K[1] = K.fy;
    f.K[2] = K.cx;
    f.K[3] = K.cy;
    f.kb4 = h->kb4[c];
    for (int i = 0; i < 4; ++i) f.kk[i] = h->kb[c].k[i];
    for (int i = 0; i < 9; ++i) f.R[i] = m.R[i];
    for (int i = 0; i < 3; ++i) f.t[i] = m.t[i];
    f.rho = m.inv_depth;
    f.depth_off = cd.row_off;
    KpDepth* hd = h->h_depth + (h->sub % kInFlight) * std::max(1, h->pred_cap);  // the staging slot's lists
    int n = 0;
    for (const vio_kp_depth& d : si.depths)
      if (d.camera == m.camera) hd[cd.row_off + n++] = KpDepth{d.id, d.inv_depth, 0};
    f.n_depth = n;
    if (n > 0)
      HIP_CHECK(h, hipMemcpyAsync(h->d_depth + cd.row_off, hd + cd.row_off, sizeof(KpDepth) * n,
                                  hipMemcpyHostToDevice, st));
  }
  si.motion.clear();
  si.depths.clear();
  return VIO_OK;
}

static void fill_frame(vio_frontend* h, int s) {
  for (int c = 0; c < (int)h->cams.size(); ++c) h->h_frame->cam[c].active = 0;
  fill_stream(h, s);
}

static size_t stage_offset(const vio_frontend* h, int s) {
  size_t so = 0;
  for (int k = 0; k < h->streams[s].first_cam; ++k) so += (size_t)h->cams[k].w * h->cams[k].h;
  return so;
}

// Copies host images of stream s into pinned staging and queues their upload
// into the current pyramid slot's level 0.
static int upload_host_images(vio_frontend* h, int s, const uint8_t* const* images, const int32_t* strides) {
  const StreamInfo& si = h->streams[s];
  const int ps = (int)(si.frames % kPyrSlots);
  size_t so = stage_offset(h, s);
  for (int k = 0; k < si.n_cams; ++k) {
    const int c = si.first_cam + k;
    const CamDesc& cd = h->cams[c];
    uint8_t* stg = h->h_stage + (h->sub % kInFlight) * h->stage_bytes + so;
    for (int y = 0; y < si.h; ++y) std::memcpy(stg + (size_t)y * si.w, images[k] + (size_t)y * strides[k], si.w);
    HIP_CHECK(h, hipMemcpy2DAsync(cd.lvl[ps][0], cd.pitch[0], stg, si.w, si.w, si.h, hipMemcpyHostToDevice,
                                  h->pstream));
    FrameCam& f = h->h_frame->cam[c];
    f.src = cd.lvl[ps][0];
    f.src_pitch = cd.pitch[0];
    f.copy_l0 = 0;
    so += (size_t)si.w * si.h;
  }
  return VIO_OK;
}

static int upload_predictions(vio_frontend* h, int s, const vio_kp_prediction* pred, int32_t n_pred, hipStream_t st) {
  const StreamInfo& si = h->streams[s];
  if (n_pred == 0) return VIO_OK;
  if (!pred || n_pred < 0) return fail(h, VIO_EINVAL, "bad prediction list");
  std::vector<vio_kp_prediction> v(pred, pred + n_pred);
  for (const auto& q : v)
    if (q.camera < 0 || q.camera >= si.n_cams) return fail(h, VIO_EINVAL, "prediction camera out of range");
  std::stable_sort(v.begin(), v.end(), [](const vio_kp_prediction& a, const vio_kp_prediction& b) {
    return a.camera != b.camera ? a.camera < b.camera : a.id < b.id;
  });
  for (size_t i = 1; i < v.size(); ++i)
    if (v[i].camera == v[i - 1].camera && v[i].id == v[i - 1].id) return fail(h, VIO_EINVAL, "duplicate prediction");
  if (n_pred > h->pred_cap) return fail(h, VIO_EINVAL, "more predictions than keypoint capacity");
  Prediction* hp = h->h_pred + (h->sub % kInFlight) * std::max(1, h->pred_cap);  // the staging slot's list
  int at = 0;
  for (int k = 0; k < si.n_cams; ++k) {
    FrameCam& f = h->h_frame->cam[si.first_cam + k];
    f.pred_off = at;
    for (const auto& q : v)
      if (q.camera == k) hp[at++] = Prediction{q.id, q.x, q.y};
    f.n_pred = at - f.pred_off;
  }
  HIP_CHECK(h, hipMemcpyAsync(h->d_pred, hp, sizeof(Prediction) * at, hipMemcpyHostToDevice, st));
  return VIO_OK;
}

int vio_frontend_push_stereo_frame(vio_frontend* h, int32_t s, int64_t t_ns, const uint8_t* const* images,
                                   const int32_t* strides, const vio_kp_prediction* pred, int32_t n_pred) {
  int rc = check_push(h, s, t_ns);
  if (rc != VIO_OK) return rc;
  StreamInfo& si = h->streams[s];
  if (!images || !strides) return fail(h, VIO_EINVAL, "null images or strides");
  for (int k = 0; k < si.n_cams; ++k)
    if (!images[k] || strides[k] < si.w) return fail(h, VIO_EINVAL, "camera %d: null image or stride < width", k);
  fill_frame(h, s);
  rc = upload_predictions(h, s, pred, n_pred, h->stream);
  if (rc != VIO_OK) return rc;
  rc = stage_motion(h, s, h->stream);
  if (rc != VIO_OK) return rc;
  rc = upload_host_images(h, s, images, strides);
  if (rc != VIO_OK) return rc;
  rc = run_frame(h, s, h->stream);
  if (rc != VIO_OK) return rc;
  si.last_t = t_ns;
  return VIO_OK;
}

int vio_frontend_push_stereo_frame_device(vio_frontend* h, int32_t s, int64_t t_ns, const void* const* d_images,
                                          const int32_t* pitches, void* hip_stream) {
  int rc = check_push(h, s, t_ns);
  if (rc != VIO_OK) return rc;
  StreamInfo& si = h->streams[s];
  if (!d_images || !pitches) return fail(h, VIO_EINVAL, "null images or pitches");
  for (int k = 0; k < si.n_cams; ++k)
    if (!d_images[k] || pitches[k] < si.w) return fail(h, VIO_EINVAL, "camera %d: null image or pitch < width", k);
  fill_frame(h, s);
  for (int k = 0; k < si.n_cams; ++k) {
    FrameCam& f = h->h_frame->cam[si.first_cam + k];
    f.src = static_cast<const uint8_t*>(d_images[k]);
    f.src_pitch = pitches[k];
    f.copy_l0 = 1;
  }
  hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : h->stream;
  rc = stage_motion(h, s, st);
  if (rc != VIO_OK) return rc;
  rc = run_frame(h, s, st);
  if (rc != VIO_OK) return rc;
  si.last_t = t_ns;
  return VIO_OK;
}

int vio_frontend_stage_frame(vio_frontend* h, int32_t s, int64_t t_ns, const uint8_t* const* images,
                             const int32_t* strides) {
  int rc = check_push(h, s, t_ns);
  if (rc != VIO_OK) return rc;
  StreamInfo& si = h->streams[s];
  if (!images || !strides) return fail(h, VIO_EINVAL, "null images or strides");
  for (int k = 0; k < si.n_cams; ++k)
    if (!images[k] || strides[k] < si.w) return fail(h, VIO_EINVAL, "camera %d: null image or stride < width", k);
  fill_stream(h, s);
  rc = upload_host_images(h, s, images, strides);
  if (rc != VIO_OK) return rc;
  rc = stage_motion(h, s, h->stream);
  if (rc != VIO_OK) return rc;
  si.staged = true;
  si.staged_t = t_ns;
  return VIO_OK;
}

int vio_frontend_stage_frame_device(vio_frontend* h, int32_t s, int64_t t_ns, const void* const* d_images,
                                    const int32_t* pitches) {
  int rc = check_push(h, s, t_ns);
  if (rc != VIO_OK) return rc;
  StreamInfo& si = h->streams[s];
  if (!d_images || !pitches) return fail(h, VIO_EINVAL, "null images or pitches");
  for (int k = 0; k < si.n_cams; ++k)
    if (!d_images[k] || pitches[k] < si.w) return fail(h, VIO_EINVAL, "camera %d: null image or pitch < width", k);
  fill_stream(h, s);
  for (int k = 0; k < si.n_cams; ++k) {
    FrameCam& f = h->h_frame->cam[si.first_cam + k];
    f.src = static_cast<const uint8_t*>(d_images[k]);
    f.src_pitch = pitches[k];
    f.copy_l0 = 1;
  }
  rc = stage_motion(h, s, h->stream);
  if (rc != VIO_OK) return rc;
  si.staged = true;
  si.staged_t = t_ns;
  return VIO_OK;
}

int vio_frontend_stage_frames_device(vio_frontend* h, int32_t n, const int32_t* streams, const int64_t* t_ns,
                                     const void* const* d_images, const int32_t* pitches) {
  if (!h || n < 0 || (n > 0 && (!streams || !t_ns || !d_images || !pitches))) return VIO_EINVAL;
  int at = 0;
  for (int i = 0; i < n; ++i) {
    if (streams[i] < 0 || streams[i] >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream out of range");
    const int rc = vio_frontend_stage_frame_device(h, streams[i], t_ns[i], d_images + at, pitches + at);
    if (rc != VIO_OK) return rc;
    at += h->streams[streams[i]].n_cams;
  }
  return VIO_OK;
}

// Submits every staged stream's frame as one batched launch set.
static int submit_staged(vio_frontend* h) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (h->learned && !h->mlp_ready) return fail(h, VIO_ESTATE, "learned init: call vio_frontend_set_mlp first");
  bool any = false;
  for (auto& si : h->streams) {
    any |= si.staged;
    for (int k = 0; k < si.n_cams; ++k) h->h_frame->cam[si.first_cam + k].active = si.staged ? 1 : 0;
  }
  if (!any) return fail(h, VIO_ESTATE, "no frame staged");
  const int rc = submit_set(h, all_set(h), h->graph_all, h->stream);
  if (rc != VIO_OK) return rc;
  for (auto& si : h->streams)
    if (si.staged) {
      si.last_t = si.staged_t;
      si.staged = false;
    }
  return VIO_OK;
}

int vio_frontend_step(vio_frontend* h) {
  int rc = submit_staged(h);
  if (rc == VIO_OK) rc = complete_all(h);
  return rc;
}

int vio_frontend_step_async(vio_frontend* h) { return submit_staged(h); }

int vio_frontend_wait(vio_frontend* h) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  return complete_oldest(h);
}

int vio_frontend_in_flight(const vio_frontend* h) { return h ? h->n_pend : 0; }

int vio_frontend_set_camera_model(vio_frontend* h, int32_t s, int32_t camera, const vio_pinhole* K) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams) return fail(h, VIO_EINVAL, "camera %d out of range", camera);
  if (K && !(std::isfinite(K->fx) && std::isfinite(K->fy) && std::isfinite(K->cx) && std::isfinite(K->cy) &&
             K->fx > 0.f && K->fy > 0.f))
    return fail(h, VIO_EINVAL, "camera model needs finite values and fx, fy > 0");
  h->K[si.first_cam + camera] = K ? *K : vio_pinhole{0.f, 0.f, 0.f, 0.f};
  h->kb4[si.first_cam + camera] = 0;
  return VIO_OK;
}

int vio_frontend_set_camera_kb4(vio_frontend* h, int32_t s, int32_t camera, const vio_kb4* K) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams) return fail(h, VIO_EINVAL, "camera %d out of range", camera);
  if (!K) return fail(h, VIO_EINVAL, "null camera model");
  bool finite = std::isfinite(K->fx) && std::isfinite(K->fy) && std::isfinite(K->cx) && std::isfinite(K->cy);
  for (float v : K->k) finite &= std::isfinite(v);
  if (!finite || !(K->fx > 0.f) || !(K->fy > 0.f))
    return fail(h, VIO_EINVAL, "camera model needs finite values and fx, fy > 0");
  const int c = si.first_cam + camera;
  h->K[c] = vio_pinhole{K->fx, K->fy, K->cx, K->cy};
  h->kb[c] = *K;
  h->kb4[c] = 1;
  return VIO_OK;
}

int vio_frontend_set_detection_mask(vio_frontend* h, int32_t s, int32_t camera, const uint8_t* mask,
                                    int32_t pitch) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (const int rc = complete_all(h)) return rc;  // frames in flight finish first
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams) return fail(h, VIO_EINVAL, "camera %d out of range", camera);
  const int c = si.first_cam + camera;
  CamDesc& cd = h->cams[c];
  if (!cd.detect) return fail(h, VIO_EINVAL, "camera %d does not detect", camera);
  if (mask && pitch < cd.w) return fail(h, VIO_EINVAL, "mask pitch below the width");
  HIP_CHECK(h, hipStreamSynchronize(h->stream));
  if (mask)
    HIP_CHECK(h, hipMemcpy2D(const_cast<uint8_t*>(cd.mask), cd.w, mask, pitch, cd.w, cd.h, hipMemcpyHostToDevice));
  cd.has_mask = mask ? 1 : 0;
  HIP_CHECK(h, hipMemcpy(h->d_cams + c, &cd, sizeof(CamDesc), hipMemcpyHostToDevice));
  return VIO_OK;
}

int vio_frontend_set_stereo_extrinsics(vio_frontend* h, int32_t s, int32_t camera, const float* R, const float* t,
                                       float inv_depth) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams) return fail(h, VIO_EINVAL, "camera %d out of range", camera);
  const int c = si.first_cam + camera;
  CamDesc& cd = h->cams[c];
  if (cd.detect) return fail(h, VIO_EINVAL, "camera %d detects; extrinsics belong to a camera receiving matches", camera);
  int src = c - 1;  // the detecting camera whose matches this camera receives
  while (!h->cams[src].detect) --src;
  if (R) {
    if (!t) return fail(h, VIO_EINVAL, "null translation");
    if (!(h->K[c].fx > 0.f) || !(h->K[src].fx > 0.f))
      return fail(h, VIO_EINVAL, "set the camera models of both cameras first");
    bool finite = std::isfinite(inv_depth);
    for (int i = 0; i < 9; ++i) finite &= std::isfinite(R[i]);
    for (int i = 0; i < 3; ++i) finite &= std::isfinite(t[i]);
    if (!finite || !(inv_depth > 0.f)) return fail(h, VIO_EINVAL, "extrinsics need finite values and inv_depth > 0");
  }
  if (const int rc = complete_all(h)) return rc;  // frames in flight finish first
  cd.has_ext = R ? 1 : 0;
  if (R) {
    const vio_pinhole& Ks = h->K[src];
    const vio_pinhole& Kt = h->K[c];
    const float ks[4] = {Ks.fx, Ks.fy, Ks.cx, Ks.cy}, kt[4] = {Kt.fx, Kt.fy, Kt.cx, Kt.cy};
    for (int i = 0; i < 4; ++i) {
      cd.ext_Ks[i] = ks[i];
      cd.ext_Kt[i] = kt[i];
      cd.ext_ks[i] = h->kb[src].k[i];
      cd.ext_kt[i] = h->kb[c].k[i];
    }
    cd.ext_kbs = h->kb4[src];
    cd.ext_kbt = h->kb4[c];
    for (int i = 0; i < 9; ++i) cd.ext_R[i] = R[i];
    for (int i = 0; i < 3; ++i) cd.ext_t[i] = t[i];
    cd.ext_rho = inv_depth;
  }
  HIP_CHECK(h, hipStreamSynchronize(h->stream));
  HIP_CHECK(h, hipMemcpy(h->d_cams + c, &cd, sizeof(CamDesc), hipMemcpyHostToDevice));
  return VIO_OK;
}

int vio_frontend_set_motion(vio_frontend* h, int32_t s, const vio_camera_motion* m, int32_t n_m,
                            const vio_kp_depth* depths, int32_t n_depths) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  StreamInfo& si = h->streams[s];
  if (n_m < 0 || n_depths < 0 || (n_m > 0 && !m) || (n_depths > 0 && !depths))
    return fail(h, VIO_EINVAL, "bad motion or depth list");
  std::vector<vio_camera_motion> mv(m, m + n_m);
  std::vector<int> seen(si.n_cams, 0);
  for (const vio_camera_motion& q : mv) {
    if (q.camera < 0 || q.camera >= si.n_cams) return fail(h, VIO_EINVAL, "motion camera %d out of range", q.camera);
    if (seen[q.camera]++) return fail(h, VIO_EINVAL, "camera %d given two motions", q.camera);
    if (!(h->K[si.first_cam + q.camera].fx > 0.f))
      return fail(h, VIO_EINVAL, "camera %d has no camera model", q.camera);
    bool finite = std::isfinite(q.inv_depth);
    for (float v : q.R) finite &= std::isfinite(v);
    for (float v : q.t) finite &= std::isfinite(v);
    if (!finite || !(q.inv_depth > 0.f)) return fail(h, VIO_EINVAL, "motion needs finite values and inv_depth > 0");
  }
  std::vector<vio_kp_depth> dv(depths, depths + n_depths);
  std::vector<int> per_cam(si.n_cams, 0);
  for (const vio_kp_depth& d : dv) {
    if (d.camera < 0 || d.camera >= si.n_cams || !seen[d.camera])
      return fail(h, VIO_EINVAL, "depth for camera %d, which has no motion", d.camera);
    if (!std::isfinite(d.inv_depth) || !(d.inv_depth > 0.f)) return fail(h, VIO_EINVAL, "inv_depth must be > 0");
    if (++per_cam[d.camera] > si.cap) return fail(h, VIO_EINVAL, "more depths than keypoint capacity");
  }
  std::stable_sort(dv.begin(), dv.end(), [](const vio_kp_depth& a, const vio_kp_depth& b) {
    return a.camera != b.camera ? a.camera < b.camera : a.id < b.id;
  });
  for (size_t i = 1; i < dv.size(); ++i)
    if (dv[i].camera == dv[i - 1].camera && dv[i].id == dv[i - 1].id) return fail(h, VIO_EINVAL, "repeated depth");
  si.motion = std::move(mv);
  si.depths = std::move(dv);
  return VIO_OK;
}

// The record count and records of camera c's last completed frame (records
// rotate over kRecSlots buffers by frame index).
static int rec_count(const vio_frontend* h, const StreamInfo& si, int c) {
  const int rs = (int)((si.done - 1) % kRecSlots);
  return h->h_rec_count[rs * (int)h->cams.size() + c];
}

static const vio_track* rec_ptr(const vio_frontend* h, const StreamInfo& si, int c) {
  const int rs = (int)((si.done - 1) % kRecSlots);
  return h->h_rec + (size_t)rs * h->rec_total + h->rec_host_off[c];
}

int vio_frontend_get_tracks(vio_frontend* h, int32_t s, vio_track* out, int32_t capacity, int32_t* n_out) {
  if (!h || !n_out) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (si.done == 0) return fail(h, VIO_ESTATE, "no frame completed yet");
  int n = 0;
  for (int k = 0; k < si.n_cams; ++k) n += rec_count(h, si, si.first_cam + k);
  *n_out = n;
  if (capacity < n) return VIO_ETOOSMALL;
  if (n > 0 && !out) return VIO_EINVAL;
  int at = 0;
  for (int k = 0; k < si.n_cams; ++k) {
    const int m = rec_count(h, si, si.first_cam + k);
    std::memcpy(out + at, rec_ptr(h, si, si.first_cam + k), sizeof(vio_track) * m);
    at += m;
  }
  return VIO_OK;
}

int vio_frontend_get_tracks_streams(vio_frontend* h, int32_t n, const int32_t* streams, vio_track* out,
                                    int32_t capacity, int32_t* counts, int32_t* n_out) {
  if (!h || !n_out || n < 0 || (n > 0 && (!streams || !counts))) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  int total = 0;
  for (int i = 0; i < n; ++i) {
    const int s = streams[i];
    if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
    const StreamInfo& si = h->streams[s];
    if (si.done == 0) return fail(h, VIO_ESTATE, "stream %d: no frame completed yet", s);
    int m = 0;
    for (int k = 0; k < si.n_cams; ++k) m += rec_count(h, si, si.first_cam + k);
    counts[i] = m;
    total += m;
  }
  *n_out = total;
  if (capacity < total) return VIO_ETOOSMALL;
  if (total > 0 && !out) return VIO_EINVAL;
  int at = 0;
  for (int i = 0; i < n; ++i) {
    const StreamInfo& si = h->streams[streams[i]];
    for (int k = 0; k < si.n_cams; ++k) {
      const int m = rec_count(h, si, si.first_cam + k);
      std::memcpy(out + at, rec_ptr(h, si, si.first_cam + k), sizeof(vio_track) * m);
      at += m;
    }
  }
  return VIO_OK;
}

static int state_slot(const StreamInfo& si) { return (int)((si.frames & 1) ^ 1); }

// The neighbour stereo start's pair tables of stream s's target cameras, from
// the states the next frame reads (slot): the selection kernel keeps them
// after every frame; a host upload of keypoints rebuilds them here, in the
// same order (the target camera's keypoints in id order that also live in
// its detecting camera).
static int rebuild_pairs(vio_frontend* h, int s, int slot) {
  if (h->P.stereo_init != VIO_STEREO_INIT_NEIGHBOUR) return VIO_OK;
  const StreamInfo& si = h->streams[s];
  for (int k = 0; k < si.n_cams; ++k) {
    const int lc = si.first_cam + k;
    const CamDesc& L = h->cams[lc];
    if (!L.detect || L.n_targets == 0) continue;
    int32_t nl = 0;
    HIP_CHECK(h, hipMemcpy(&nl, &h->d_cnt->n_live[slot][lc], sizeof nl, hipMemcpyDeviceToHost));
    std::vector<Kp> ls((size_t)nl);
    if (nl > 0) HIP_CHECK(h, hipMemcpy(ls.data(), L.state[slot], sizeof(Kp) * nl, hipMemcpyDeviceToHost));
    for (int t = 0; t < L.n_targets; ++t) {
      const int rc = lc + 1 + t;
      const CamDesc& R = h->cams[rc];
      int32_t nr = 0;
      HIP_CHECK(h, hipMemcpy(&nr, &h->d_cnt->n_live[slot][rc], sizeof nr, hipMemcpyDeviceToHost));
      std::vector<Kp> rs((size_t)nr);
      if (nr > 0) HIP_CHECK(h, hipMemcpy(rs.data(), R.state[slot], sizeof(Kp) * nr, hipMemcpyDeviceToHost));
      std::vector<float4> pr;
      for (const Kp& q : rs) {
        const auto it = std::lower_bound(ls.begin(), ls.end(), q.id, [](const Kp& a, int64_t id) { return a.id < id; });
        if (it != ls.end() && it->id == q.id) pr.push_back(make_float4(it->x, it->y, q.x - it->x, q.y - it->y));
      }
      const int32_t np = (int32_t)pr.size();
      if (np > 0) HIP_CHECK(h, hipMemcpy(R.pairs[slot], pr.data(), sizeof(float4) * np, hipMemcpyHostToDevice));
      HIP_CHECK(h, hipMemcpy(&h->d_cnt->n_pairs[slot][rc], &np, sizeof np, hipMemcpyHostToDevice));
    }
  }
  return VIO_OK;
}

int vio_frontend_set_keypoints(vio_frontend* h, int32_t s, int32_t camera, const vio_keypoint* kps, int32_t n) {
  if (!h) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (const int rc = complete_all(h)) return rc;  // frames in flight finish first
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams) return fail(h, VIO_EINVAL, "camera out of range");
  if (n < 0 || n > si.cap || (n > 0 && !kps)) return fail(h, VIO_EINVAL, "bad keypoint count");
  int64_t max_id = -1;
  for (int i = 0; i < n; ++i) {
    if (i > 0 && kps[i].id <= kps[i - 1].id) return fail(h, VIO_EINVAL, "ids must ascend");
    if (kps[i].id < 0) return fail(h, VIO_EINVAL, "negative id");
    max_id = kps[i].id;
  }
  const int c = si.first_cam + camera;
  const int slot = state_slot(si);
  if (n > 0) HIP_CHECK(h, hipMemcpy(h->cams[c].state[slot], kps, sizeof(Kp) * n, hipMemcpyHostToDevice));
  HIP_CHECK(h, hipMemcpy(&h->d_cnt->n_live[slot][c], &n, sizeof(int32_t), hipMemcpyHostToDevice));
  int64_t next = 0;
  HIP_CHECK(h, hipMemcpy(&next, &h->d_cnt->next_id[s], sizeof next, hipMemcpyDeviceToHost));
  next = std::max(next, max_id + 1);
  HIP_CHECK(h, hipMemcpy(&h->d_cnt->next_id[s], &next, sizeof next, hipMemcpyHostToDevice));
  return rebuild_pairs(h, s, slot);
}

int vio_frontend_get_keypoints(vio_frontend* h, int32_t s, int32_t camera, vio_keypoint* out, int32_t capacity,
                               int32_t* n_out) {
  if (!h || !n_out) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (const int rc = complete_all(h)) return rc;  // frames in flight finish first
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams) return fail(h, VIO_EINVAL, "camera out of range");
  const int c = si.first_cam + camera;
  const int slot = state_slot(si);
  int32_t n = 0;
  HIP_CHECK(h, hipMemcpy(&n, &h->d_cnt->n_live[slot][c], sizeof n, hipMemcpyDeviceToHost));
  *n_out = n;
  if (capacity < n) return VIO_ETOOSMALL;
  if (n > 0) HIP_CHECK(h, hipMemcpy(out, h->cams[c].state[slot], sizeof(Kp) * n, hipMemcpyDeviceToHost));
  return VIO_OK;
}

int vio_frontend_get_pyramid(vio_frontend* h, int32_t s, int32_t camera, int32_t level, uint8_t* out,
                             size_t capacity) {
  if (!h || !out) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (const int rc = complete_all(h)) return rc;  // frames in flight finish first
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams || level < 0 || level >= h->P.levels) return fail(h, VIO_EINVAL, "bad camera/level");
  if (si.frames == 0) return fail(h, VIO_ESTATE, "no frame pushed yet");
  const CamDesc& c = h->cams[si.first_cam + camera];
  const int w = c.w >> level, hh = c.h >> level;
  if (capacity < (size_t)w * hh) return VIO_ETOOSMALL;
  const int ps = (int)((si.frames - 1) % kPyrSlots);
  HIP_CHECK(h, hipMemcpy2D(out, w, c.lvl[ps][level], c.pitch[level], w, hh, hipMemcpyDeviceToHost));
  return VIO_OK;
}

int vio_frontend_get_cell_winners(vio_frontend* h, int32_t s, int32_t camera, int32_t* out, int32_t capacity,
                                  int32_t* n_out) {
  if (!h || !n_out) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (const int rc = complete_all(h)) return rc;  // frames in flight finish first
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams) return fail(h, VIO_EINVAL, "camera out of range");
  const CamDesc& c = h->cams[si.first_cam + camera];
  if (!c.detect) return fail(h, VIO_EINVAL, "camera %d does not detect", camera);
  if (si.frames == 0) return fail(h, VIO_ESTATE, "no frame pushed yet");
  *n_out = c.nslots;
  if (capacity < 3 * c.nslots) return VIO_ETOOSMALL;
  if (!out) return VIO_EINVAL;
  std::vector<uint32_t> keys(c.nslots);
  const int ps = (int)((si.frames - 1) % kPyrSlots);
  HIP_CHECK(h, hipMemcpy(keys.data(), c.keys[ps], sizeof(uint32_t) * c.nslots, hipMemcpyDeviceToHost));
  for (int i = 0; i < c.nslots; ++i) {
    if (!keys[i]) {
      out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = -1;
      continue;
    }
    const int idx = 0xFFFFFF - (int)(keys[i] & 0xFFFFFFu);
    out[3 * i] = idx % c.w;
    out[3 * i + 1] = idx / c.w;
    out[3 * i + 2] = (int)(keys[i] >> 24);
  }
  return VIO_OK;
}

int vio_frontend_set_mlp(vio_frontend* h, const float* params, int32_t n, float rho) {
  if (!h || !params || n != VIO_MLP_NPARAM) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (const int rc = complete_all(h)) return rc;  // frames in flight finish first
  if (!h->learned) return fail(h, VIO_ESTATE, "the frontend was not created with VIO_INIT_LEARNED");
  HIP_CHECK(h, hipStreamSynchronize(h->stream));
  HIP_CHECK(h, hipMemcpy(h->mlp.P, params, sizeof(float) * VIO_MLP_NPARAM, hipMemcpyHostToDevice));
  HIP_CHECK(h, mlp_pack_launch(h->mlp, h->stream));
  HIP_CHECK(h, hipStreamSynchronize(h->stream));
  if (rho >= 0.f) h->P.learned_rho = rho;
  // the captured graphs hold the old threshold as a kernel argument
  for (auto& si : h->streams)
    for (Graphs& g : si.graph) g.destroy();
  for (Graphs& g : h->graph_all) g.destroy();
  h->mlp_ready = true;
  return VIO_OK;
}

int vio_frontend_get_features(vio_frontend* h, int32_t s, int32_t camera, float* out, int32_t capacity,
                              int32_t* n_out) {
  if (!h || !n_out) return VIO_EINVAL;
  if (h->poisoned) return VIO_EDEVICE;
  if (const int rc = complete_all(h)) return rc;  // frames in flight finish first
  if (!h->learned) return fail(h, VIO_ESTATE, "features exist in learned mode only");
  if (s < 0 || s >= (int)h->streams.size()) return fail(h, VIO_EINVAL, "stream %d out of range", s);
  const StreamInfo& si = h->streams[s];
  if (camera < 0 || camera >= si.n_cams) return fail(h, VIO_EINVAL, "camera out of range");
  if (si.frames < 2) return fail(h, VIO_ESTATE, "features exist from the second frame on");
  const int c = si.first_cam + camera;
  // the temporal records of the last frame are the previous keypoints, in slot order
  int32_t n = 0;
  const int prev_slot = (int)(si.frames & 1);  // state slot the last frame read
  HIP_CHECK(h, hipMemcpy(&n, &h->d_cnt->n_live[prev_slot][c], sizeof n, hipMemcpyDeviceToHost));
  *n_out = n;
  if (capacity < n * VIO_MLP_IN) return VIO_ETOOSMALL;
  if (n > 0) {
    if (!out) return VIO_EINVAL;
    HIP_CHECK(h, hipMemcpy(out, h->d_feat + (size_t)h->cams[c].row_off * VIO_MLP_IN, sizeof(float) * VIO_MLP_IN * n,
                           hipMemcpyDeviceToHost));
  }
  return VIO_OK;
}

int vio_frontend_get_stats(vio_frontend* h, vio_stats* out) {
  if (!h || !out) return VIO_EINVAL;
  *out = h->stats;
  return VIO_OK;
}

}  // extern "C"
