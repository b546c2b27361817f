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
// that have a flow into a uniform grid of integer cells of about twice the
// expected distance to the 8th neighbour: counts in LDS, a workgroup scan,
// and a scatter of (position, index) into the camera's grid arrays.
// k_features (one wave64 per keypoint) scans the (2R+1)^2 cells around its
// keypoint -- every lane keeping a sorted top-8 of (squared distance, index)
// over its share of the window's tracks -- and merges the lanes' heads in
// eight wave-wide minimum rounds. A window is accepted when its 8th distance
// is below the distance to the window's nearest open side (no track outside
// can be as close) or it covers the grid, else R grows. The live set is
// sorted by id, so index order is id order; squared distances are taken in
// double, where differences and squares of float positions are exact, so the
// neighbour order is reproducible bit for bit. The same wave then pools the
// patch.
#include "fe_common.h"

namespace vio {
namespace {

constexpr int kGridThreads = 1024;
constexpr int kFeatWaves = 4;
constexpr int kNone = 0x7FFFFFFF;
static_assert(kFeatGridMax <= kGridThreads, "one cell per thread in the scan");

__device__ __forceinline__ bool less_di(double da, int ia, double db, int ib) {
  return da < db || (da == db && ia < ib);
}

// Cell edge (px) and grid size for n tracks on a w x h image: about
// 1.9 sqrt(area / n), at most kFeatGridMax cells.
__device__ __forceinline__ void grid_geometry(int w, int h, int n, int& cs, int& gx, int& gy) {
  cs = max(8, (int)ceilf(1.9f * sqrtf((float)w * (float)h / (float)max(n, 1))));
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

// Inserts (dd, qi) into the lane's ascending top-8 (a NaN distance never enters).
__device__ __forceinline__ void top8_insert(double (&d)[8], int (&ix)[8], double dd, int qi) {
  if (!less_di(dd, qi, d[7], ix[7])) return;
  d[7] = dd;
  ix[7] = qi;
#pragma unroll
  for (int k = 7; k > 0; --k) {
    const bool sw = less_di(d[k], ix[k], d[k - 1], ix[k - 1]);
    const double td = d[k];
    const int ti = ix[k];
    d[k] = sw ? d[k - 1] : d[k];
    ix[k] = sw ? ix[k - 1] : ix[k];
    d[k - 1] = sw ? td : d[k - 1];
    ix[k - 1] = sw ? ti : ix[k - 1];
  }
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
  const int mcx = min(max((int)floorf(me.x) / cs, 0), gx - 1);
  const int mcy = min(max((int)floorf(me.y) / cs, 0), gy - 1);
  float nfx = 0.f, nfy = 0.f;  // lane r keeps the r-th neighbour's flow
  for (int R = 1;; ++R) {
    const int ax = max(0, mcx - R), bx = min(gx - 1, mcx + R);
    const int ay = max(0, mcy - R), by = min(gy - 1, mcy + R);
    double d[8];
    int ix[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) d[k] = INFINITY, ix[k] = kNone;
    for (int row = ay; row <= by; ++row) {
      // the cells of a row are contiguous in the sorted order
      const int hi = start[row * gx + bx + 1];
      for (int q = start[row * gx + ax] + lane; q < hi; q += 64) {
        const float2 p = pos[q];
        const double dx = (double)p.x - mx, dy = (double)p.y - my;
        top8_insert(d, ix, dx * dx + dy * dy, idx[q]);
      }
    }
    // merge: eight rounds of the wave-wide minimum of the lanes' heads
    int found = 0;
    double dlast = 0.0;
    nfx = nfy = 0.f;
    for (int r = 0; r < 8; ++r) {
      double bd = d[0];
      int bi = ix[0];
#pragma unroll
      for (int msk = 1; msk < 64; msk <<= 1) {
        const double od = __shfl_xor(bd, msk);
        const int oi = __shfl_xor(bi, msk);
        const bool take = less_di(od, oi, bd, bi);
        bd = take ? od : bd;
        bi = take ? oi : bi;
      }
      if (bi == kNone) break;  // wave-uniform
      const bool pop = ix[0] == bi;  // the lane holding the winner drops it
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        d[k] = pop ? d[k + 1] : d[k];
        ix[k] = pop ? ix[k + 1] : ix[k];
      }
      d[7] = pop ? INFINITY : d[7];
      ix[7] = pop ? kNone : ix[7];
      const Kp o = live[bi];
      nfx = lane == r ? (o.x - o.px) * 0.0625f : nfx;
      nfy = lane == r ? (o.y - o.py) * 0.0625f : nfy;
      found = r + 1;
      dlast = bd;
    }
    if (ax == 0 && bx == gx - 1 && ay == 0 && by == gy - 1) break;
    // no track outside the window lies closer than its nearest open side
    double bnd = INFINITY;
    if (ax > 0) bnd = fmin(bnd, mx - (double)(ax * cs));
    if (bx < gx - 1) bnd = fmin(bnd, (double)((bx + 1) * cs) - mx);
    if (ay > 0) bnd = fmin(bnd, my - (double)(ay * cs));
    if (by < gy - 1) bnd = fmin(bnd, (double)((by + 1) * cs) - my);
    if (found == 8 && dlast < bnd * bnd) break;
  }
  float* f = feat + (size_t)(cd.row_off + j) * 32;
  {
    const float fx = __shfl(nfx, (lane >> 1) & 7), fy = __shfl(nfy, (lane >> 1) & 7);
    if (lane < 16) f[lane] = (lane & 1) ? fy : fx;
  }

  // ---- pooled patch of the previous frame --------------------------------
  const int rx = (int)floorf(me.x + 0.5f), ry = (int)floorf(me.y + 0.5f);
  const uint8_t* img = cd.lvl[Q][0];
  const int pitch = cd.pitch[0];
  const int prow = lane >> 2, col4 = (lane & 3) * 4;
  const int yy = min(max(ry - 8 + prow, 0), cd.h - 1);
  int ps = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) ps += img[(size_t)yy * pitch + min(max(rx - 8 + col4 + k, 0), cd.w - 1)];
  // cell (row / 4, lane & 3): lanes differing in bits 2 and 3 share a cell
  const int csum = ps + __shfl_xor(ps, 4) + __shfl_xor(ps, 8) + __shfl_xor(ps, 12);
  int tot = ps;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) tot += __shfl_xor(tot, m);
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
