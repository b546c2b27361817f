// Features of the learned initialisation, one wave64 per live keypoint of the
// previous frame, kFeatWaves keypoints of one camera per workgroup:
//  * the previous flows (x - px, y - py) / 16 of the 8 live tracks of the
//    camera nearest to the keypoint with a flow (age >= 1; its own track, at
//    distance 0, comes first when it has one), nearest first by (squared
//    distance, id), zero when fewer exist;
//  * the previous frame's level-0 patch of 16x16 pixels around round(p),
//    clamped to the image, pooled over 4x4 cells: cell_sum * 16 / patch_sum - 1
//    (integer sums, one correctly rounded division).
//
// Neighbour search: the workgroup stages the camera's track positions in LDS
// (8 bytes per track, chunks of kFeatChunk, a track without a flow stored as
// NaN so it never wins), each lane keeps a sorted top-8 of (squared distance,
// index) over its share of the candidates in one pass, and eight wave-wide
// minimum rounds merge the lanes' heads. The live set is sorted by id, so
// index order is id order. Squared distances are taken in double, where the
// differences and squares of float positions are exact, so the neighbour
// order is reproducible bit for bit.
#include "fe_common.h"

namespace vio {
namespace {

constexpr int kFeatWaves = 16;
constexpr int kFeatChunk = 4096;
constexpr int kNone = 0x7FFFFFFF;

__device__ __forceinline__ bool less_di(double da, int ia, double db, int ib) {
  return da < db || (da == db && ia < ib);
}

__global__ __launch_bounds__(64 * kFeatWaves) void k_features(const CamDesc* __restrict__ cams,
                                                             const FrameTable* __restrict__ frame,
                                                             const Counters* __restrict__ cnt, int cam_begin,
                                                             int cam_end, float* __restrict__ feat) {
  __shared__ float2 s_pos[kFeatChunk];
  // the workgroup's camera and first keypoint: ceil(cap / kFeatWaves) workgroups per camera
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
  const int j0 = b * kFeatWaves;
  if (j0 >= n) return;  // workgroup-uniform: before any barrier
  const int lane = threadIdx.x & 63;
  const int j = j0 + (int)(threadIdx.x >> 6);
  const bool has = j < n;  // wave-uniform
  const Kp* live = cd.state[Q];
  const Kp me = live[has ? j : j0];
  const double mx = (double)me.x, my = (double)me.y;

  // ---- per-lane top-8 over the candidates, one pass -----------------------
  double d[8];
  int ix[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) d[k] = INFINITY, ix[k] = kNone;
  for (int base = 0; base < n; base += kFeatChunk) {
    const int m = min(kFeatChunk, n - base);
    __syncthreads();  // the previous chunk is consumed
    for (int i = (int)threadIdx.x; i < m; i += (int)blockDim.x) {
      const Kp o = live[base + i];
      s_pos[i] = o.age >= 1 ? make_float2(o.x, o.y) : make_float2(NAN, NAN);
    }
    __syncthreads();
    if (has) {
      for (int q = lane; q < m; q += 64) {
        const float2 p = s_pos[q];
        const double dx = (double)p.x - mx, dy = (double)p.y - my;
        const double dd = dx * dx + dy * dy;  // NaN for a track without a flow: never less
        const int qi = base + q;
        if (less_di(dd, qi, d[7], ix[7])) {
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
      }
    }
  }
  if (!has) return;  // no barrier follows
  float* f = feat + (size_t)(cd.row_off + j) * 32;

  // ---- merge: eight rounds of the wave-wide minimum of the lanes' heads ----
  float nfx = 0.f, nfy = 0.f;  // lane r keeps the r-th neighbour's flow
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
    if (bi == kNone) break;  // wave-uniform: fewer than r + 1 neighbours, the rest stay zero
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
  }
  {
    const float fx = __shfl(nfx, (lane >> 1) & 7), fy = __shfl(nfy, (lane >> 1) & 7);
    if (lane < 16) f[lane] = (lane & 1) ? fy : fx;
  }

  // ---- pooled patch of the previous frame --------------------------------
  const int rx = (int)floorf(me.x + 0.5f), ry = (int)floorf(me.y + 0.5f);
  const uint8_t* img = cd.lvl[Q][0];
  const int pitch = cd.pitch[0];
  const int row = lane >> 2, col4 = (lane & 3) * 4;
  const int yy = min(max(ry - 8 + row, 0), cd.h - 1);
  int s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += img[(size_t)yy * pitch + min(max(rx - 8 + col4 + k, 0), cd.w - 1)];
  // cell (row / 4, lane & 3): lanes differing in bits 2 and 3 share a cell
  const int cs = s + __shfl_xor(s, 4) + __shfl_xor(s, 8) + __shfl_xor(s, 12);
  int tot = s;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) tot += __shfl_xor(tot, m);
  if (((lane >> 2) & 3) == 0) {
    const int cell = (row >> 2) * 4 + (lane & 3);
    f[16 + cell] = tot > 0 ? (float)(cs * 16) / (float)tot - 1.f : 0.f;
  }
}

}  // namespace

hipError_t launch_features(const CamDesc* d_cams, const FrameTable* d_frame, const Counters* d_cnt,
                           const CamDesc* h_cams, int cam_begin, int cam_end, float* d_feat, hipStream_t s) {
  int blocks = 0;
  for (int c = cam_begin; c < cam_end; ++c) blocks += (h_cams[c].cap + kFeatWaves - 1) / kFeatWaves;
  if (blocks <= 0) return hipSuccess;
  launch_kernel(k_features, dim3(blocks), dim3(64 * kFeatWaves), 0, s, d_cams, d_frame, d_cnt, cam_begin, cam_end,
                d_feat);
  return hipGetLastError();
}

}  // namespace vio
