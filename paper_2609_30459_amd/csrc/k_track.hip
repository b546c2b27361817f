// Patch tracker for gfx950: inverse-compositional SE(2) alignment with a
// forward-backward check (Sec. III-E, eqs. 4-5, Fig. 4).
//
// One wave64 tracks one keypoint; lane i < 52 owns pattern point x_i (the 52
// half-integer offsets of the radius-4 disk, rows v = -3.5..3.5 of 4, 6, 8, 8,
// 8, 8, 6, 4 points), lanes 52..63 sit on an interior offset with weight 0 so
// every lane runs the same code. Sums over the pattern use DPP inside each
// 16-lane row plus four readlanes, a fixed tree that is identical in every
// lane, so the result is deterministic and wave-uniform. Every branch is taken
// on a wave vote, so a wave never diverges.
//
// Per iteration only four sums are needed: since
//   delta = -sum_i G_i (I'_i / mean' - T_i) = c - (sum_i G_i I'_i) / mean'
// with c = sum_i G_i T_i fixed per level, one fused reduction of
// (sum I'_i, sum G_i I'_i) gives both the warped mean and the update.
//
// The same launch also runs the stereo matching of every detected cell winner
// (left camera -> right camera of the pair): those matches depend only on the
// current pyramids, so they run beside the temporal tracks instead of after the
// selection, and the selection kernel picks the ones it keeps.
#include "fe_common.h"

namespace vio {
namespace {

constexpr int kW = 64;

template <int ctrl>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
}

__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Sum over the 64 lanes, returned in every lane (wave-uniform).
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
}

__device__ __forceinline__ bool wave_all(bool p) { return __all(p); }
__device__ __forceinline__ bool wave_any(bool p) { return __any(p); }

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

// bilinear interpolation on [0, W-1] x [0, H-1]; the caller has checked the domain
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

// One coarse-to-fine pass: template on `src` at (px, py), warp from (ix, iy,
// ith), N Gauss-Newton iterations per level, levels L-1 .. 0, translation
// doubled between levels, a level whose template does not fit is skipped.
__device__ PassOut klt_pass(const CamDesc& csrc, int ssrc, const CamDesc& cdst, int sdst, float px, float py,
                            float ix, float iy, float ith, int L, int N, float u, float v, float wgt) {
  PassOut o{VIO_TRACKED, 0.f, 0.f, 0.f, 0.f};
  const float s0 = 1.f / (float)(1 << (L - 1));
  float tx = ix * s0, ty = iy * s0, th = ith;
  for (int l = L - 1; l >= 0; --l) {
    if (l < L - 1) {
      tx = tx * 2.f;
      ty = ty * 2.f;
    }
    const float sc = 1.f / (float)(1 << l);
    const Level S = level_of(csrc, ssrc, l);
    const float sx = px * sc + u, sy = py * sc + v;
    const bool fits = in_dom(S, sx - 1.f, sy) && in_dom(S, sx + 1.f, sy) && in_dom(S, sx, sy - 1.f) &&
                      in_dom(S, sx, sy + 1.f);
    if (!wave_all(fits)) {
      if (l == 0) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      continue;
    }
    // template (Sec. III-E): mean-normalised samples and gradients
    const float I0 = bilinear(S, sx, sy);
    const float gxr = (bilinear(S, sx + 1.f, sy) - bilinear(S, sx - 1.f, sy)) / 2.f;
    const float gyr = (bilinear(S, sx, sy + 1.f) - bilinear(S, sx, sy - 1.f)) / 2.f;
    const float mean = wave_sum(wgt * I0) / 52.f;
    if (!(mean > 0.f)) {
      o.status = VIO_LOST_DEGENERATE;
      return o;
    }
    const float T = I0 / mean;
    const float nx = gxr / mean, ny = gyr / mean;
    const float J0 = nx, J1 = ny, J2 = ny * u - nx * v;
    const float h00 = wave_sum(wgt * J0 * J0), h01 = wave_sum(wgt * J0 * J1), h02 = wave_sum(wgt * J0 * J2);
    const float h11 = wave_sum(wgt * J1 * J1), h12 = wave_sum(wgt * J1 * J2), h22 = wave_sum(wgt * J2 * J2);
    // 3x3 inverse by cofactors (H symmetric)
    const float c00 = h11 * h22 - h12 * h12;
    const float c01 = h12 * h02 - h01 * h22;
    const float c02 = h01 * h12 - h11 * h02;
    const float det = h00 * c00 + h01 * c01 + h02 * c02;
    const float tr3 = (h00 + h11 + h22) / 3.f;
    if (!(det > 1e-6f * tr3 * tr3 * tr3)) {
      o.status = VIO_LOST_DEGENERATE;
      return o;
    }
    const float id = 1.f / det;
    const float i00 = c00 * id, i01 = (h02 * h12 - h01 * h22) * id, i02 = (h01 * h12 - h02 * h11) * id;
    const float i10 = c01 * id, i11 = (h00 * h22 - h02 * h02) * id, i12 = (h02 * h01 - h00 * h12) * id;
    const float i20 = c02 * id, i21 = (h01 * h02 - h00 * h12) * id, i22 = (h00 * h11 - h01 * h01) * id;
    const float G0 = i00 * J0 + i01 * J1 + i02 * J2;
    const float G1 = i10 * J0 + i11 * J1 + i12 * J2;
    const float G2 = i20 * J0 + i21 * J1 + i22 * J2;
    if (wave_any(!(isfinite(G0) && isfinite(G1) && isfinite(G2)))) {
      o.status = VIO_LOST_DEGENERATE;
      return o;
    }
    const float k0 = wave_sum(wgt * G0 * T), k1 = wave_sum(wgt * G1 * T), k2 = wave_sum(wgt * G2 * T);
    const Level D = level_of(cdst, sdst, l);
    for (int it = 0; it < N; ++it) {
      const float cs = cosf(th), sn = sinf(th);
      const float wx = (cs * u - sn * v) + tx, wy = (sn * u + cs * v) + ty;
      if (wave_any(!in_dom(D, wx, wy))) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      const float Iw = bilinear(D, wx, wy);
      const float S0 = wave_sum(wgt * Iw);
      const float S1 = wave_sum(wgt * G0 * Iw), S2 = wave_sum(wgt * G1 * Iw), S3 = wave_sum(wgt * G2 * Iw);
      const float mw = S0 / 52.f;
      if (!(mw > 0.f)) {
        o.status = VIO_LOST_OOB;
        return o;
      }
      if (l == 0 && it == N - 1) {
        const float e = Iw / mw - T;
        o.resid = sqrtf(wave_sum(wgt * e * e) / 52.f);
      }
      const float d0 = k0 - S1 / mw, d1 = k1 - S2 / mw, d2 = k2 - S3 / mw;
      // SE(2) exponential: translation V(phi) (d0, d1)
      float a, b;
      if (fabsf(d2) < 1e-4f) {
        a = 1.f - d2 * d2 / 6.f;
        b = d2 / 2.f;
      } else {
        a = sinf(d2) / d2;
        b = (1.f - cosf(d2)) / d2;
      }
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

__device__ TrackRes track_fb(const CamDesc& csrc, int ssrc, const CamDesc& cdst, int sdst, float px, float py,
                             float ix, float iy, int L, int N, float fb_thr, float u, float v, float wgt) {
  TrackRes r;
  r.x = ix;
  r.y = iy;
  r.theta = 0.f;
  r.fb = 0.f;
  r.resid = 0.f;
  r.status = VIO_TRACKED;
  r.pad[0] = r.pad[1] = 0;
  const PassOut f = klt_pass(csrc, ssrc, cdst, sdst, px, py, ix, iy, 0.f, L, N, u, v, wgt);
  if (f.status != VIO_TRACKED) {
    r.status = f.status;
    return r;
  }
  r.x = f.tx;
  r.y = f.ty;
  r.theta = f.th;
  r.resid = f.resid;
  const PassOut b = klt_pass(cdst, sdst, csrc, ssrc, f.tx, f.ty, px, py, -f.th, L, N, u, v, wgt);
  if (b.status != VIO_TRACKED) {
    r.status = b.status;
    return r;
  }
  const float dx = b.tx - px, dy = b.ty - py;
  r.fb = sqrtf(dx * dx + dy * dy);
  r.status = r.fb > fb_thr ? VIO_LOST_FB : VIO_TRACKED;
  return r;
}

__global__ __launch_bounds__(kW* kTrackWaves) void k_track(const CamDesc* __restrict__ cams,
                                                          const FrameTable* __restrict__ frame,
                                                          const Counters* __restrict__ cnt,
                                                          const TrackSeg* __restrict__ segs, int n_segs,
                                                          const Prediction* __restrict__ pred, Tuning tune) {
  const int lane = threadIdx.x & (kW - 1);
  const int item = (int)blockIdx.x * kTrackWaves + (int)(threadIdx.x / kW);
  int si = 0;
  while (si + 1 < n_segs && segs[si + 1].begin <= item) ++si;
  const TrackSeg sg = segs[si];
  const int j = item - sg.begin;
  if (j < 0 || j >= sg.count) return;
  const int c = sg.cam;
  const CamDesc& cd = cams[c];
  const FrameCam& fc = frame->cam[c];
  if (!fc.active) return;
  float u, v, wgt;
  pattern_of(lane, u, v, wgt);
  const int P = fc.parity;
  if (sg.mode == kModeTemporal) {
    if (!fc.has_prev || j >= cnt->n_live[P ^ 1][c]) return;
    const Kp kp = cd.state[P ^ 1][j];
    float ix = kp.x + (kp.x - kp.px), iy = kp.y + (kp.y - kp.py);
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
          break;
        }
        if (mid_id < kp.id) lo = mid + 1;
        else hi = mid - 1;
      }
    }
    const TrackRes r =
        track_fb(cd, P ^ 1, cd, P, kp.x, kp.y, ix, iy, tune.levels, tune.iters, tune.fb_threshold, u, v, wgt);
    if (lane == 0) cd.res[j] = r;
  } else {
    const uint32_t key = cd.keys[P][j];
    if (key == 0) return;
    const int idx = 0xFFFFFF - (int)(key & 0xFFFFFFu);
    const float x = (float)(idx % cd.w), y = (float)(idx / cd.w);
    const TrackRes r = track_fb(cd, P, cams[cd.partner], P, x, y, x - tune.disparity0, y, tune.levels, tune.iters,
                                tune.fb_threshold, u, v, wgt);
    if (lane == 0) cd.sres[j] = r;
  }
}

}  // namespace

hipError_t launch_track(const CamDesc* d_cams, const FrameTable* d_frame, Counters* d_cnt, const TrackSeg* d_segs,
                        int n_segs, int n_items, const Prediction* d_pred, Tuning tune, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const int blocks = (n_items + kTrackWaves - 1) / kTrackWaves;
  hipLaunchKernelGGL(k_track, dim3(blocks), dim3(kW * kTrackWaves), 0, s, d_cams, d_frame, d_cnt, d_segs, n_segs,
                     d_pred, tune);
  return hipGetLastError();
}

}  // namespace vio
