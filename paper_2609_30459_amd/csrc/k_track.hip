// Patch tracker for gfx950: inverse-compositional SE(2) alignment with a
// forward-backward check (Sec. III-E, eqs. 4-5, Fig. 4).
//
// One wave64 tracks one keypoint; lane i < 52 owns pattern point x_i (the 52
// half-integer offsets of the radius-4 disk, rows v = -3.5..3.5 of 4, 6, 8, 8,
// 8, 8, 6, 4 points), lanes 52..63 sit on an interior offset with weight 0 so
// every lane runs the same code. Every branch is taken on a wave vote, so a
// wave never diverges.
//
// A keypoint's time is its chain of dependent steps (2 passes x L levels x N
// iterations), each a gather, a reduction and a little wave-uniform math, with
// about one wave per SIMD at these sizes. The kernel is shaped for that chain:
//  * sums over the pattern: DPP inside each 16-lane row, then row_bcast:15/31
//    and one readlane of lane 63 -- a fixed tree, so results are deterministic;
//  * per iteration one fused reduction of (sum I'_i, sum G_i I'_i), since
//      delta = -sum_i G_i (I'_i / mean' - T_i) = c - (sum_i G_i I'_i) / mean'
//    with c = sum_i G_i T_i fixed per level;
//  * the templates of all levels of a pass are built together (they depend
//    only on the source image and the keypoint), so their gathers and
//    reductions overlap instead of sitting between the levels' iterations;
//  * wave-uniform math uses the hardware reciprocal and sine/cosine, and a
//    series for the SE(2) exponential;
//  * gathers read the pyramid through the L1 cache (the patch's lines stay hot
//    across a level's iterations).
// Decisions (template fit, degeneracy, leaving the image) are taken in the
// same order as a level-by-level pass, so the status is that of the paper's
// procedure.
//
// The same launch also runs the stereo matching of every detected cell winner
// (left camera -> right camera of the pair): those matches depend only on the
// current pyramids, so they run beside the temporal tracks instead of after the
// selection, and the selection kernel picks the ones it keeps.
#include <algorithm>

#include "fe_common.h"

namespace vio {
namespace {

constexpr int kW = 64;

template <int ctrl, int row_mask = 0xF>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, row_mask, 0xF, false));
}

// Sum over the 64 lanes, returned as a wave-uniform value: each 16-lane row is
// reduced with quad permutes and mirrors (every lane of a row then holds the
// row sum), row_bcast:15 adds row 0 into row 1 and row 2 into row 3,
// row_bcast:31 adds rows 0+1 into row 3; lane 63 holds (r2+r3)+(r0+r1).
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);       // row_half_mirror
  v += dpp<0x140>(v);       // row_mirror
  v += dpp<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v += dpp<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ bool wave_all(bool p) { return __all(p); }
__device__ __forceinline__ bool wave_any(bool p) { return __any(p); }

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ void pattern_of(int lane, float& u, float& v, float& w) {
  // rows v = -3.5 .. 3.5 hold 4, 6, 8, 8, 8, 8, 6, 4 points; row starts 0, 4,
  // 10, 18, 26, 34, 42, 48 (52 in all)
  int r, base, n;
  if (lane < 4) r = 0, base = 0, n = 4;
  else if (lane < 10) r = 1, base = 4, n = 6;
  else if (lane < 42) r = 2 + (lane - 10) / 8, base = 10 + 8 * ((lane - 10) / 8), n = 8;
  else if (lane < 48) r = 6, base = 42, n = 6;
  else if (lane < 52) r = 7, base = 48, n = 4;
  else r = -1, base = 0, n = 0;
  if (r < 0) {
    u = 0.5f;
    v = 0.5f;
    w = 0.f;
    return;
  }
  v = -3.5f + (float)r;
  u = -0.5f * (float)(n - 1) + (float)(lane - base);
  w = 1.f;
}

struct Level {
  const uint8_t* p;
  int pitch, w, h;
};

__device__ __forceinline__ bool in_dom(const Level& I, float x, float y) {
  return x >= 0.f && x <= (float)(I.w - 1) && y >= 0.f && y <= (float)(I.h - 1);
}

// bilinear interpolation on [0, W-1] x [0, H-1]: ix = min(floor(x), W-2),
// fx = x - ix (likewise y); the caller has checked the domain
__device__ __forceinline__ float bilinear(const Level& I, float x, float y) {
  const int ix = min((int)floorf(x), I.w - 2), iy = min((int)floorf(y), I.h - 2);
  const float fx = x - (float)ix, fy = y - (float)iy;
  const uint8_t* q = I.p + (size_t)iy * I.pitch + ix;
  const float a = q[0], b = q[1], c = q[I.pitch], d = q[I.pitch + 1];
  return (1.f - fy) * ((1.f - fx) * a + fx * b) + fy * ((1.f - fx) * c + fx * d);
}

// level l of pyramid slot `slot` of camera `cd` (scalar loads from the descriptor)
__device__ __forceinline__ Level level_of(const CamDesc& cd, int slot, int l) {
  Level L;
  L.p = cd.lvl[slot][l];
  L.pitch = cd.pitch[l];
  L.w = cd.w >> l;
  L.h = cd.h >> l;
  return L;
}

struct PassOut {
  int status;
  float tx, ty, th, resid;
};

// SE(2) exponential of (d0, d1, phi): translation V(phi) (d0, d1) with
// V = [[a, -b], [b, a]], a = sin(phi)/phi, b = (1 - cos(phi))/phi.
__device__ __forceinline__ void se2_v(float phi, float& a, float& b) {
  const float p2 = phi * phi;
  if (fabsf(phi) < 0.25f) {  // series, error below 2e-9 here
    a = 1.f - p2 * (1.f / 6.f - p2 * (1.f / 120.f - p2 * (1.f / 5040.f)));
    b = phi * (0.5f - p2 * (1.f / 24.f - p2 * (1.f / 720.f - p2 * (1.f / 40320.f))));
  } else {
    const float ip = rcp(phi);
    a = __sinf(phi) * ip;
    b = (1.f - __cosf(phi)) * ip;
  }
}

// One coarse-to-fine pass: template on `src` at (px, py), warp from (ix, iy,
// ith), N Gauss-Newton iterations per level, levels L-1 .. 0, translation
// doubled between levels, a level whose template does not fit is skipped.
template <int L>
__device__ PassOut klt_pass(const CamDesc& csrc, int ssrc, const CamDesc& cdst, int sdst, float px, float py,
                            float ix, float iy, float ith, int N, float u, float v, float wgt) {
  PassOut o{VIO_TRACKED, 0.f, 0.f, 0.f, 0.f};
  // ---- templates of all levels (Sec. III-E) ------------------------------
  bool fits[L], valid[L];
  float T[L], G0[L], G1[L], G2[L], k0[L], k1[L], k2[L];
  float I0[L], gxr[L], gyr[L];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const Level S = level_of(csrc, ssrc, l);
    const float sc = 1.f / (float)(1 << l);
    const float sx = px * sc + u, sy = py * sc + v;
    fits[l] = wave_all(in_dom(S, sx - 1.f, sy) && in_dom(S, sx + 1.f, sy) && in_dom(S, sx, sy - 1.f) &&
                       in_dom(S, sx, sy + 1.f));
    I0[l] = gxr[l] = gyr[l] = 0.f;
    if (fits[l]) {
      I0[l] = bilinear(S, sx, sy);
      gxr[l] = (bilinear(S, sx + 1.f, sy) - bilinear(S, sx - 1.f, sy)) * 0.5f;
      gyr[l] = (bilinear(S, sx, sy + 1.f) - bilinear(S, sx, sy - 1.f)) * 0.5f;
    }
  }
  float mean[L];
#pragma unroll
  for (int l = 0; l < L; ++l) mean[l] = wave_sum(wgt * I0[l]) * (1.f / 52.f);
  float J0[L], J1[L], J2[L];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const float im = rcp(mean[l]);
    T[l] = I0[l] * im;
    J0[l] = gxr[l] * im;
    J1[l] = gyr[l] * im;
    J2[l] = J1[l] * u - J0[l] * v;
  }
  float h00[L], h01[L], h02[L], h11[L], h12[L], h22[L];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    h00[l] = wave_sum(wgt * J0[l] * J0[l]);
    h01[l] = wave_sum(wgt * J0[l] * J1[l]);
    h02[l] = wave_sum(wgt * J0[l] * J2[l]);
    h11[l] = wave_sum(wgt * J1[l] * J1[l]);
    h12[l] = wave_sum(wgt * J1[l] * J2[l]);
    h22[l] = wave_sum(wgt * J2[l] * J2[l]);
  }
#pragma unroll
  for (int l = 0; l < L; ++l) {
    // 3x3 inverse by cofactors (H symmetric); degenerate when det <= 1e-6 (tr/3)^3
    const float c00 = h11[l] * h22[l] - h12[l] * h12[l];
    const float c01 = h12[l] * h02[l] - h01[l] * h22[l];
    const float c02 = h01[l] * h12[l] - h11[l] * h02[l];
    const float det = h00[l] * c00 + h01[l] * c01 + h02[l] * c02;
    const float tr3 = (h00[l] + h11[l] + h22[l]) * (1.f / 3.f);
    const float id = rcp(det);
    const float i00 = c00 * id, i01 = c01 * id, i02 = c02 * id;
    const float i11 = (h00[l] * h22[l] - h02[l] * h02[l]) * id;
    const float i12 = (h02[l] * h01[l] - h00[l] * h12[l]) * id;
    const float i22 = (h00[l] * h11[l] - h01[l] * h01[l]) * id;
    // weight folded into the gains: lanes 52..63 contribute nothing
    G0[l] = wgt * (i00 * J0[l] + i01 * J1[l] + i02 * J2[l]);
    G1[l] = wgt * (i01 * J0[l] + i11 * J1[l] + i12 * J2[l]);
    G2[l] = wgt * (i02 * J0[l] + i12 * J1[l] + i22 * J2[l]);
    valid[l] = mean[l] > 0.f && det > 1e-6f * tr3 * tr3 * tr3 &&
               wave_all(isfinite(G0[l]) && isfinite(G1[l]) && isfinite(G2[l]));
  }
#pragma unroll
  for (int l = 0; l < L; ++l) {
    k0[l] = wave_sum(G0[l] * T[l]);
    k1[l] = wave_sum(G1[l] * T[l]);
    k2[l] = wave_sum(G2[l] * T[l]);
  }
  // ---- coarse-to-fine Gauss-Newton (eqs. 4-5) ------------------------------
  const float s0 = 1.f / (float)(1 << (L - 1));
  float tx = ix * s0, ty = iy * s0, th = ith;
#pragma unroll
  for (int l = L - 1; l >= 0; --l) {
    if (l < L - 1) {
      tx = tx * 2.f;
      ty = ty * 2.f;
    }
    if (!fits[l]) {
      if (l == 0) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      continue;
    }
    if (!valid[l]) {
      o.status = VIO_LOST_DEGENERATE;
      return o;
    }
    const Level D = level_of(cdst, sdst, l);
    for (int it = 0; it < N; ++it) {
      const float cs = __cosf(th), sn = __sinf(th);
      const float wx = (cs * u - sn * v) + tx, wy = (sn * u + cs * v) + ty;
      if (wave_any(!in_dom(D, wx, wy))) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      const float Iw = bilinear(D, wx, wy);
      const float S0 = wave_sum(wgt * Iw);
      const float S1 = wave_sum(G0[l] * Iw), S2 = wave_sum(G1[l] * Iw), S3 = wave_sum(G2[l] * Iw);
      const float mw = S0 * (1.f / 52.f);
      if (!(mw > 0.f)) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      const float imw = rcp(mw);
      if (l == 0 && it == N - 1) {
        const float e = Iw * imw - T[l];
        o.resid = sqrtf(wave_sum(wgt * e * e) * (1.f / 52.f));
      }
      const float d0 = k0[l] - S1 * imw, d1 = k1[l] - S2 * imw, d2 = k2[l] - S3 * imw;
      float a, b;
      se2_v(d2, a, b);
      const float vx = a * d0 - b * d1, vy = b * d0 + a * d1;
      tx = tx + (cs * vx - sn * vy);
      ty = ty + (sn * vx + cs * vy);
      th = th + d2;
    }
  }
  o.tx = tx;
  o.ty = ty;
  o.th = th;
  return o;
}

template <int L>
__device__ TrackRes track_fb(const CamDesc& csrc, int ssrc, const CamDesc& cdst, int sdst, float px, float py,
                             float ix, float iy, int N, float fb_thr, float u, float v, float wgt) {
  TrackRes r;
  r.x = ix;
  r.y = iy;
  r.theta = 0.f;
  r.fb = 0.f;
  r.resid = 0.f;
  r.status = VIO_TRACKED;
  r.pad[0] = r.pad[1] = 0;
  const PassOut f = klt_pass<L>(csrc, ssrc, cdst, sdst, px, py, ix, iy, 0.f, N, u, v, wgt);
  if (f.status != VIO_TRACKED) {
    r.status = f.status;
    return r;
  }
  r.x = f.tx;
  r.y = f.ty;
  r.theta = f.th;
  r.resid = f.resid;
  const PassOut b = klt_pass<L>(cdst, sdst, csrc, ssrc, f.tx, f.ty, px, py, -f.th, N, u, v, wgt);
  if (b.status != VIO_TRACKED) {
    r.status = b.status;
    return r;
  }
  const float dx = b.tx - px, dy = b.ty - py;
  r.fb = sqrtf(dx * dx + dy * dy);
  r.status = r.fb > fb_thr ? VIO_LOST_FB : VIO_TRACKED;
  return r;
}

// Stores a wave-uniform 32-byte result without a branch on the lane id:
// lanes 0..7 write one dword each through a buffer resource whose range is
// exactly the record, and the hardware drops the other lanes' stores as out of
// range. (A lane-id branch inside the persistent loop would let the compiler
// split the wave across loop iterations; this keeps the loop body free of
// lane-dependent control flow.)
__device__ __forceinline__ void store_result(TrackRes* dst, const TrackRes& r, int lane) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)sizeof(TrackRes), kBufferWord3);
  const uint32_t w[8] = {__builtin_bit_cast(uint32_t, r.x),     __builtin_bit_cast(uint32_t, r.y),
                         __builtin_bit_cast(uint32_t, r.theta), __builtin_bit_cast(uint32_t, r.fb),
                         __builtin_bit_cast(uint32_t, r.resid), (uint32_t)r.status,
                         (uint32_t)r.pad[0],                    (uint32_t)r.pad[1]};
  uint32_t val = w[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) val = lane == k ? w[k] : val;
  __builtin_amdgcn_raw_buffer_store_b32(val, rs, lane * 4, 0, 0);
}

// One work item: a temporal track (camera c, slot j) or the stereo match of a
// cell winner (camera c, cell j). LL > 0: learned initialisation -- temporal
// tracks run LL levels from the network's guess and fall back to the plain
// L-level tracker from the constant-velocity guess unless kept with a
// residual RMS <= rho.
template <int L, int LL>
__device__ void process_item(const CamDesc* __restrict__ cams, const FrameTable* __restrict__ frame,
                             const Counters* __restrict__ cnt, const TrackSeg* __restrict__ segs, int n_segs,
                             const Prediction* __restrict__ pred, const Tuning& tune, int item, int lane, float u,
                             float v, float wgt) {
  // the last segment that begins at or before the item (begins ascend)
  int lo = 0, hi = n_segs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].begin <= item) lo = mid;
    else hi = mid - 1;
  }
  const TrackSeg sg = segs[lo];
  const int j = item - sg.begin;
  if (j < 0 || j >= sg.count) return;
  const int c = sg.cam;
  const CamDesc& cd = cams[c];
  const FrameCam& fc = frame->cam[c];
  if (!fc.active) return;
  const int P = fc.parity;
  if (sg.mode == kModeTemporal) {
    if (!fc.has_prev || j >= cnt->n_live[P ^ 1][c]) return;
    const Kp kp = cd.state[P ^ 1][j];
    float ix = kp.x + (kp.x - kp.px), iy = kp.y + (kp.y - kp.py);
    bool predicted = false;
    const int np = fc.n_pred;
    if (np > 0) {  // caller predictions, ascending id: binary search
      const Prediction* pp = pred + fc.pred_off;
      int lo = 0, hi = np - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int64_t mid_id = pp[mid].id;
        if (mid_id == kp.id) {
          ix = pp[mid].x;
          iy = pp[mid].y;
          predicted = true;
          break;
        }
        if (mid_id < kp.id) lo = mid + 1;
        else hi = mid - 1;
      }
    }
    TrackRes r;
    bool done = false;
    if constexpr (LL > 0) {
      if (!predicted) {
        const float* gs = tune.guess + (size_t)(cd.row_off + j) * 3;
        const float gx = kp.x + 16.f * gs[0], gy = kp.y + 16.f * gs[1];
        r = track_fb<LL>(cd, P ^ 1, cd, P, kp.x, kp.y, gx, gy, tune.liters, tune.fb_threshold, u, v, wgt);
        done = r.status == VIO_TRACKED && r.resid <= tune.rho;
      }
    }
    if (!done) {
      r = track_fb<L>(cd, P ^ 1, cd, P, kp.x, kp.y, ix, iy, tune.iters, tune.fb_threshold, u, v, wgt);
      r.pad[0] = (LL > 0 && !predicted) ? 1 : 0;
    }
    store_result(cd.res + j, r, lane);
  } else {
    // stereo match of a detection: speculative (item j = cell j's winner) or
    // deferred (item j = the frame's j-th selected detection)
    float x, y;
    if (tune.deferred) {
      if (j >= cnt->n_sel[c]) return;
      const Kp kp = cd.state[P][cnt->sel_base[c] + j];
      x = kp.x;
      y = kp.y;
    } else {
      const uint32_t key = cd.keys[P][j];
      if (key == 0) return;
      const int idx = 0xFFFFFF - (int)(key & 0xFFFFFFu);
      x = (float)(idx % cd.w);
      y = (float)(idx / cd.w);
    }
    TrackRes r = track_fb<L>(cd, P, cams[cd.partner], P, x, y, x - tune.disparity0, y, tune.iters,
                             tune.fb_threshold, u, v, wgt);
    r.pad[0] = 0;
    store_result(cd.sres + j, r, lane);
  }
}

// One wave per work item.
template <int L, int LL>
__global__ __launch_bounds__(kW* kTrackWaves) void k_track(const CamDesc* __restrict__ cams,
                                                          const FrameTable* __restrict__ frame,
                                                          const Counters* __restrict__ cnt,
                                                          const TrackSeg* __restrict__ segs, int n_segs,
                                                          int item_base, int n_items,
                                                          const Prediction* __restrict__ pred, Tuning tune) {
  const int lane = threadIdx.x & (kW - 1);
  const int k = (int)blockIdx.x * (int)(blockDim.x / kW) + (int)(threadIdx.x / kW);
  if (k >= n_items) return;
  float u, v, wgt;
  pattern_of(lane, u, v, wgt);
  process_item<L, LL>(cams, frame, cnt, segs, n_segs, pred, tune, item_base + k, lane, u, v, wgt);
}

// Persistent grid: every wave pops items from the frame's queue counter until
// it runs past n_items (each pop advances the counter, so every wave exits).
// The pop is branch-free: all lanes issue the atomic, lane 0 adding one and
// the others zero, and the first lane's (lane 0's) old value is the item, so
// no lane-dependent control flow enters the loop.
template <int L, int LL>
__global__ __launch_bounds__(kW* kTrackWaves) void k_track_persistent(const CamDesc* __restrict__ cams,
                                                                     FrameTable* __restrict__ frame,
                                                                     const Counters* __restrict__ cnt,
                                                                     const TrackSeg* __restrict__ segs, int n_segs,
                                                                     int item_base, int n_items,
                                                                     const Prediction* __restrict__ pred,
                                                                     Tuning tune, int queue) {
  const int lane = threadIdx.x & (kW - 1);
  float u, v, wgt;
  pattern_of(lane, u, v, wgt);
  for (;;) {
    const int k = __builtin_amdgcn_readfirstlane(atomicAdd(&frame->queue_head[queue], lane == 0 ? 1 : 0));
    if (k >= n_items) break;
    process_item<L, LL>(cams, frame, cnt, segs, n_segs, pred, tune, item_base + k, lane, u, v, wgt);
  }
}

template <int L, int LL>
hipError_t launch_L(const CamDesc* d_cams, FrameTable* d_frame, Counters* d_cnt, const TrackSeg* d_segs, int n_segs,
                    int item_base, int n_items, const Prediction* d_pred, Tuning tune, TrackShape sh, hipStream_t s) {
  const int bw = sh.block_waves;
  if (sh.waves_per_cu > 0) {
    const int waves = std::min(n_items, sh.waves_per_cu * sh.n_cus);
    const int blocks = (waves + bw - 1) / bw;
    launch_kernel(k_track_persistent<L, LL>, dim3(blocks), dim3(kW * bw), 0, s, d_cams, d_frame, d_cnt, d_segs,
                  n_segs, item_base, n_items, d_pred, tune, sh.queue);
  } else {
    const int blocks = (n_items + bw - 1) / bw;
    launch_kernel(k_track<L, LL>, dim3(blocks), dim3(kW * bw), 0, s, d_cams, d_frame, d_cnt, d_segs, n_segs,
                       item_base, n_items, d_pred, tune);
  }
  return hipGetLastError();
}

template <int L>
hipError_t launch_LL(const CamDesc* d_cams, FrameTable* d_frame, Counters* d_cnt, const TrackSeg* d_segs, int n_segs,
                     int item_base, int n_items, const Prediction* d_pred, Tuning tune, TrackShape sh, hipStream_t s) {
  const int ll = tune.learned ? tune.llevels : 0;
  switch (ll) {
    case 0: return launch_L<L, 0>(d_cams, d_frame, d_cnt, d_segs, n_segs, item_base, n_items, d_pred, tune, sh, s);
    case 1: return launch_L<L, 1>(d_cams, d_frame, d_cnt, d_segs, n_segs, item_base, n_items, d_pred, tune, sh, s);
    case 2: return launch_L<L, 2>(d_cams, d_frame, d_cnt, d_segs, n_segs, item_base, n_items, d_pred, tune, sh, s);
    case 3: return launch_L<L, 3>(d_cams, d_frame, d_cnt, d_segs, n_segs, item_base, n_items, d_pred, tune, sh, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_track(const CamDesc* d_cams, FrameTable* d_frame, Counters* d_cnt, const TrackSeg* d_segs, int n_segs,
                        int item_base, int n_items, const Prediction* d_pred, Tuning tune, TrackShape shape,
                        hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (shape.block_waves < 1 || shape.block_waves > kTrackWaves || shape.n_cus < 1 || shape.waves_per_cu < 0 ||
      shape.queue < 0 || shape.queue >= 4)
    return hipErrorInvalidValue;
  switch (tune.levels) {
#define VIO_TRACK_CASE(LV) \
  case LV: return launch_LL<LV>(d_cams, d_frame, d_cnt, d_segs, n_segs, item_base, n_items, d_pred, tune, shape, s);
    VIO_TRACK_CASE(1)
    VIO_TRACK_CASE(2)
    VIO_TRACK_CASE(3)
    VIO_TRACK_CASE(4)
    VIO_TRACK_CASE(5)
    VIO_TRACK_CASE(6)
#undef VIO_TRACK_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vio
