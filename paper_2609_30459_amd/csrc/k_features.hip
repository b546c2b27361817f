// Features of the learned initialisation for the live keypoints of the
// previous frame (32 inputs per keypoint, row row_off + j of the feature
// matrix):
//  * inputs 0..15: the previous flows (x - px, y - py) / 16 of the 8 live
//    tracks of the camera nearest to the keypoint with a flow (age >= 1; its
//    own track, at distance 0, comes first when it has one), nearest first by
//    (squared distance, id), zero when fewer exist;
//  * inputs 16..31: the previous frame's level-0 patch of 16x16 pixels around
//    round(p), clamped to the image, pooled over 4x4 cells:
//    cell_sum * 16 / patch_sum - 1 (integer sums, one correctly rounded
//    division).
//
// Two launches. k_grid (one workgroup per camera) buckets the camera's tracks
// that have a flow into a uniform grid of integer cells of 2.5 mean track
// spacings (about 6 tracks a cell, and well beyond the expected distance to
// the 8th neighbour): counts in LDS, a workgroup scan, and a scatter of
// (position, index) into the camera's grid arrays. k_features (one wave64 per
// keypoint) gives every track of the (2R+1)^2 cells around its keypoint an
// exact key (squared distance, index), one per lane, and sorts the keys over
// the wave with a bitonic network (lane exchanges by DPP, swizzle and
// permlane, no LDS); windows with more than 64 tracks go in chunks, the best
// eight riding along in lanes 0..7. A window is accepted when its 8th
// distance is below the distance to the window's nearest open side (no track
// outside can be as close) or it covers the grid, else R grows. The live set
// is sorted by id, so index order is id order; squared distances are taken in
// double, where differences and squares of float positions are exact, so the
// neighbour order is reproducible bit for bit. The same wave then pools the
// patch.
#include "fe_common.h"
#include "wave_ops.h"

namespace vio {
namespace {

constexpr int kGridThreads = 1024;
constexpr int kFeatWaves = 4;
constexpr int kNone = 0x7FFFFFFF;
static_assert(kFeatGridMax <= kGridThreads, "one cell per thread in the scan");

// Cell edge (px) and grid size for n tracks on a w x h image: about
// 2.5 sqrt(area / n), at most kFeatGridMax cells.
__device__ __forceinline__ void grid_geometry(int w, int h, int n, int& cs, int& gx, int& gy) {
  cs = max(8, (int)ceilf(2.5f * sqrtf((float)w * (float)h / (float)max(n, 1))));
  gx = (w + cs - 1) / cs;
  gy = (h + cs - 1) / cs;
  while (gx * gy > kFeatGridMax) {
    cs += cs / 4 + 1;
    gx = (w + cs - 1) / cs;
    gy = (h + cs - 1) / cs;
  }
}

__global__ __launch_bounds__(kGridThreads) void k_grid(const CamDesc* __restrict__ cams,
                                                      const FrameTable* __restrict__ frame,
                                                      const Counters* __restrict__ cnt, int cam_begin, FeatGrid fg) {
  __shared__ int s_cnt[kFeatGridMax];
  __shared__ int s_wsum[kGridThreads / 64];
  const int c = cam_begin + (int)blockIdx.x;
  const CamDesc& cd = cams[c];
  const FrameCam& fc = frame->cam[c];
  if (!fc.active || !fc.has_prev) return;
  const int Q = fc.parity ^ 1;
  const int n = cnt->n_live[Q][c];
  const Kp* live = cd.state[Q];
  int cs, gx, gy;
  grid_geometry(cd.w, cd.h, n, cs, gx, gy);
  const int G = gx * gy;
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int* start = fg.start + (size_t)c * (kFeatGridMax + 1);
  if (tid == 0) fg.hdr[c] = make_int4(cs, gx, gy, 0);
  for (int t = tid; t < G; t += kGridThreads) s_cnt[t] = 0;
  __syncthreads();
  auto cell_of = [&](const Kp& o) {
    const int cx = min(max((int)floorf(o.x) / cs, 0), gx - 1);
    const int cy = min(max((int)floorf(o.y) / cs, 0), gy - 1);
    return cy * gx + cx;
  };
  for (int i = tid; i < n; i += kGridThreads) {
    const Kp o = live[i];
    if (o.age >= 1) atomicAdd(&s_cnt[cell_of(o)], 1);
  }
  __syncthreads();
  {  // exclusive scan of the counts, one cell per thread
    const int v = tid < G ? s_cnt[tid] : 0;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      x += lane >= o ? y : 0;
    }
    if (lane == 63) s_wsum[wave] = x;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < kGridThreads / 64; ++w) before += w < wave ? s_wsum[w] : 0;
    const int excl = x - v + before;
    if (tid < G) {
      start[tid] = excl;
      s_cnt[tid] = excl;  // becomes the fill cursor
    }
    if (tid == G - 1) start[G] = excl + v;
  }
  __syncthreads();
  float2* pos = fg.pos + cd.row_off;
  int* idx = fg.idx + cd.row_off;
  for (int i = tid; i < n; i += kGridThreads) {
    const Kp o = live[i];
    if (o.age >= 1) {
      const int slot = atomicAdd(&s_cnt[cell_of(o)], 1);
      pos[slot] = make_float2(o.x, o.y);
      idx[slot] = i;
    }
  }
}

// Exact neighbour key: the squared distance as the bits of a non-negative
// double (their unsigned order is the numeric order), then the index.
struct NKey {
  uint64_t d;
  int ix;
};

__device__ __forceinline__ bool nkey_less(const NKey& a, const NKey& b) {
  return a.d < b.d || (a.d == b.d && a.ix < b.ix);
}

// The value of lane (lane ^ J) (every lane active). J = 1, 2 by quad
// permutes, 8 by a rotation of the 16-lane row by 8, 4 and 16 by swizzles
// inside 32-lane halves, 32 by a permlane32 swap.
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int lane) {
  if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
  if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
  if constexpr (J == 4) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);
  if constexpr (J == 8) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);
  if constexpr (J == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
  if constexpr (J == 32) {
    // swap(v, v): the first result holds lanes 0..31 twice, the second 32..63
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    const uint32_t lo = p[0], hi = p[1];
    return lane < 32 ? hi : lo;
  }
  return v;
}

// One compare-exchange stage of a bitonic sort over the 64 lanes: partner
// lane ^ J; in blocks of K lanes sorted ascending when (lane & K) == 0, the
// lower lane of a pair keeps the smaller key.
template <int K, int J>
__device__ __forceinline__ void bitonic_stage(NKey& k, int lane) {
  NKey p;
  const uint32_t lo = xor_lane<J>((uint32_t)k.d, lane), hi = xor_lane<J>((uint32_t)(k.d >> 32), lane);
  p.d = ((uint64_t)hi << 32) | lo;
  p.ix = (int)xor_lane<J>((uint32_t)k.ix, lane);
  const bool want_min = ((lane & J) == 0) == ((lane & K) == 0);
  const bool take = want_min ? nkey_less(p, k) : nkey_less(k, p);
  // field by field: a select of the whole struct goes through private memory
  k.d = take ? p.d : k.d;
  k.ix = take ? p.ix : k.ix;
}

template <int K, int J>
__device__ __forceinline__ void bitonic_merge(NKey& k, int lane) {
  bitonic_stage<K, J>(k, lane);
  if constexpr (J > 1) bitonic_merge<K, J / 2>(k, lane);
}

// Sorts the 64 lanes' keys ascending by lane (21 compare-exchange stages).
template <int K = 2>
__device__ __forceinline__ void bitonic_sort64(NKey& k, int lane) {
  bitonic_merge<K, K / 2>(k, lane);
  if constexpr (K < 64) bitonic_sort64<K * 2>(k, lane);
}

__global__ __launch_bounds__(64 * kFeatWaves) void k_features(const CamDesc* __restrict__ cams,
                                                             const FrameTable* __restrict__ frame,
                                                             const Counters* __restrict__ cnt, int cam_begin,
                                                             int cam_end, FeatGrid fg, float* __restrict__ feat) {
  // the wave's camera and keypoint: ceil(cap / kFeatWaves) workgroups per camera
  int c = cam_begin, b = (int)blockIdx.x;
  for (; c < cam_end; ++c) {
    const int nb = (cams[c].cap + kFeatWaves - 1) / kFeatWaves;
    if (b < nb) break;
    b -= nb;
  }
  if (c >= cam_end) return;
  const CamDesc& cd = cams[c];
  const FrameCam& fc = frame->cam[c];
  if (!fc.active || !fc.has_prev) return;
  const int Q = fc.parity ^ 1;
  const int n = cnt->n_live[Q][c];
  const int lane = threadIdx.x & 63;
  const int j = b * kFeatWaves + (int)(threadIdx.x >> 6);
  if (j >= n) return;  // no barrier in this kernel
  const Kp* live = cd.state[Q];
  const Kp me = live[j];
  const double mx = (double)me.x, my = (double)me.y;
  const int4 gh = fg.hdr[c];
  const int cs = gh.x, gx = gh.y, gy = gh.z;
  const int* start = fg.start + (size_t)c * (kFeatGridMax + 1);
  const float2* pos = fg.pos + cd.row_off;
  const int* idx = fg.idx + cd.row_off;

  // ---- the 8 nearest tracks with a flow: growing windows of cells --------
  // Every candidate of the window gets an exact key; lanes 0..7 keep the best
  // eight so far, and each chunk of candidates (64, then 56 at a time in
  // lanes 8..63) is merged in by a bitonic sort over the wave.
  const int mcx = min(max((int)floorf(me.x) / cs, 0), gx - 1);
  const int mcy = min(max((int)floorf(me.y) / cs, 0), gy - 1);
  const NKey none{0x7FF0000000000000ull, kNone};  // +inf, no track
  NKey best = none;
  for (int R = 1;; ++R) {
    const int ax = max(0, mcx - R), bx = min(gx - 1, mcx + R);
    const int ay = max(0, mcy - R), by = min(gy - 1, mcy + R);
    // the cells of a window row are contiguous in the sorted order
    int total = 0;
    for (int row = ay; row <= by; ++row) total += start[row * gx + bx + 1] - start[row * gx + ax];
    best = none;
    for (int t0 = 0; t0 == 0 || t0 < total; t0 += t0 == 0 ? 64 : 56) {
      // after the first chunk, lanes 0..7 carry the best eight so far
      const int t = t0 == 0 ? lane : (lane < 8 ? -1 : t0 + lane - 8);
      const bool carry = t0 != 0 && lane < 8;
      NKey k;
      k.d = carry ? best.d : none.d;
      k.ix = carry ? best.ix : none.ix;
      if (t >= 0 && t < total) {
        int q = 0, acc = 0;
        for (int row = ay; row <= by; ++row) {
          const int rb = start[row * gx + ax], n = start[row * gx + bx + 1] - rb;
          q = (t >= acc && t < acc + n) ? rb + (t - acc) : q;
          acc += n;
        }
        const float2 p = pos[q];
        const double dx = (double)p.x - mx, dy = (double)p.y - my;
        k.d = (uint64_t)__double_as_longlong(dx * dx + dy * dy);
        k.ix = idx[q];
      }
      bitonic_sort64(k, lane);
      best = k;
    }
    if (ax == 0 && bx == gx - 1 && ay == 0 && by == gy - 1) break;
    // no track outside the window lies closer than its nearest open side
    double bnd = INFINITY;
    if (ax > 0) bnd = fmin(bnd, mx - (double)(ax * cs));
    if (bx < gx - 1) bnd = fmin(bnd, (double)((bx + 1) * cs) - mx);
    if (ay > 0) bnd = fmin(bnd, my - (double)(ay * cs));
    if (by < gy - 1) bnd = fmin(bnd, (double)((by + 1) * cs) - my);
    const int ix7 = __builtin_amdgcn_readlane(best.ix, 7);
    const uint32_t d7lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)best.d, 7);
    const uint32_t d7hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(best.d >> 32), 7);
    const double d7 = __longlong_as_double((long long)(((uint64_t)d7hi << 32) | d7lo));
    if (ix7 != kNone && d7 < bnd * bnd) break;
  }
  float* f = feat + (size_t)(cd.row_off + j) * 32;
  {
    // lane r < 8 holds the r-th neighbour (nearest first)
    float fx = 0.f, fy = 0.f;
    if (lane < 8 && best.ix != kNone) {
      const Kp o = live[best.ix];
      fx = (o.x - o.px) * 0.0625f;
      fy = (o.y - o.py) * 0.0625f;
    }
    if (lane < 8) reinterpret_cast<float2*>(f)[lane] = make_float2(fx, fy);
  }

  // ---- pooled patch of the previous frame --------------------------------
  const int rx = (int)floorf(me.x + 0.5f), ry = (int)floorf(me.y + 0.5f);
  const uint8_t* img = cd.lvl[fc.pyr_prev][0];
  const int pitch = cd.pitch[0];
  const int prow = lane >> 2, col4 = (lane & 3) * 4;
  const int yy = min(max(ry - 8 + prow, 0), cd.h - 1);
  int ps = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) ps += img[(size_t)yy * pitch + min(max(rx - 8 + col4 + k, 0), cd.w - 1)];
  // cell (row / 4, lane & 3): the four lanes of a 16-lane row that agree in
  // bits 0..1 share a cell (rotations by 8 and 4 sum them)
  int csum = ps + dpp_i<0x128>(ps);
  csum += dpp_i<0x124>(csum);
  const int tot = wave_total_i(ps);
  if (((lane >> 2) & 3) == 0) {
    const int cell = (prow >> 2) * 4 + (lane & 3);
    f[16 + cell] = tot > 0 ? (float)(csum * 16) / (float)tot - 1.f : 0.f;
  }
}

}  // namespace

hipError_t launch_grid(const CamDesc* d_cams, const FrameTable* d_frame, const Counters* d_cnt, int cam_begin,
                       int cam_end, const FeatGrid& fg, hipStream_t s) {
  if (cam_end <= cam_begin) return hipSuccess;
  launch_kernel(k_grid, dim3(cam_end - cam_begin), dim3(kGridThreads), 0, s, d_cams, d_frame, d_cnt, cam_begin, fg);
  return hipGetLastError();
}

hipError_t launch_features(const CamDesc* d_cams, const FrameTable* d_frame, const Counters* d_cnt,
                           const CamDesc* h_cams, int cam_begin, int cam_end, const FeatGrid& fg, float* d_feat,
                           hipStream_t s) {
  if (cam_end <= cam_begin) return hipSuccess;
  int blocks = 0;
  for (int c = cam_begin; c < cam_end; ++c) blocks += (h_cams[c].cap + kFeatWaves - 1) / kFeatWaves;
  launch_kernel(k_features, dim3(blocks), dim3(64 * kFeatWaves), 0, s, d_cams, d_frame, d_cnt, cam_begin, cam_end,
                fg, d_feat);
  return hipGetLastError();
}

}  // namespace vio
