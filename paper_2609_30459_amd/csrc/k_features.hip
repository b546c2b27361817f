// Features of the learned initialisation for the live keypoints of the
// previous frame (32 inputs per keypoint, row row_off + j of the feature
// matrix), and the network's guesses from them:
//  * inputs 0..15: the previous flows (x - px, y - py) / 16 of the 8 live
//    tracks of the camera nearest to the keypoint with a flow (age >= 1; its
//    own track, at distance 0, comes first when it has one), nearest first by
//    (squared distance, id), zero when fewer exist;
//  * inputs 16..31: the previous frame's level-0 patch of 16x16 pixels around
//    round(p), clamped to the image, pooled over 4x4 cells:
//    cell_sum * 16 / patch_sum - 1 (integer sums, one correctly rounded
//    division).
//
// One launch (k_learn): a workgroup takes W keypoints of one camera (one wave
// each; W = 4, 8 or 16), stages the camera's tracks in LDS chunk by chunk, and
// every wave searches all of them for its keypoint: each lane keeps a sorted list of
// its best eight exact keys (squared distance in double, where the
// differences and squares of float positions are exact, then index) over
// the tracks it visits, and eight rounds of a wave minimum over the lanes'
// list heads take the eight nearest in order. The live set is
// sorted by id, so index order is id order and the neighbour order is the
// brute-force one, bit for bit. The same wave then pools the patch.
#include "fe_common.h"
#include "learn_ops.h"
#include "mfma_ops.h"
#include "wave_ops.h"

namespace vio {
namespace {

constexpr int kTileRows = 16;     // rows of one MFMA tile: at most 16 keypoints per workgroup
constexpr int kHidTiles = MH / 16;  // 16-unit output tiles of a hidden layer
constexpr int kCandChunk = 2048;  // tracks staged in LDS at a time (16 KB)

// The features and the network's output for W keypoints of one camera per
// workgroup (rows 0..W-1 of one MFMA tile; the other rows are zero). Wave w
// computes keypoint j0 + w's features (exact 8 nearest tracks, pooled patch)
// into the feature matrix and, rounded to bfloat16, into the workgroup's input
// tile; then wave w computes hidden tiles w, w + W, ... (16 units each, K = 32
// for layer 1 and 4 x 32 for layer 2) and wave 0 the three outputs, with the
// same MFMA sequence as the network kernel of vio_mlp.h (so the same results
// row by row). Each wave loads its weight slices into registers before the
// feature search, so their L2 latency hides behind it. Fewer waves per
// workgroup spread a camera over more compute units, each wave with a larger
// share of its SIMD.
template <int W>
__global__ __launch_bounds__(64 * W) void k_learn(const CamDesc* __restrict__ cams, const FrameTable* __restrict__ frame,
                                                  const Counters* __restrict__ cnt, int cam_begin, int cam_end,
                                                  MlpDev M, float* __restrict__ feat, float* __restrict__ guess) {
  static_assert(W >= 1 && W <= kTileRows, "one tile of keypoints per workgroup");
  constexpr int kTPW = (kHidTiles + W - 1) / W;  // hidden tiles per wave
  __shared__ float2 sCand[kCandChunk];                   // a chunk of the camera's tracks
  // bf16 inputs (one row per keypoint) and h1, then h2; rows padded by 8
  // entries, so that the 16 rows of an MFMA operand read (16 bytes per lane)
  // start 4 banks apart instead of in the same bank
  __shared__ __align__(16) uint16_t sX[kTileRows][MI + 8];
  __shared__ __align__(16) uint16_t sH[kTileRows][MH + 8];
  // the workgroup's camera and keypoints: ceil(cap / W) workgroups per camera
  int c = cam_begin, b = (int)blockIdx.x;
  for (; c < cam_end; ++c) {
    const int nb = (cams[c].cap + W - 1) / W;
    if (b < nb) break;
    b -= nb;
  }
  if (c >= cam_end) return;  // the conditions below are uniform over the workgroup: no barrier is skipped
  const CamDesc& cd = cams[c];
  const FrameCam& fc = frame->cam[c];
  if (!fc.active || !fc.has_prev) return;
  const int Q = fc.parity ^ 1;
  const int n = cnt->n_live[Q][c];
  const int j0 = b * W;
  if (j0 >= n) return;
  const int lane = threadIdx.x & 63, wv = (int)(threadIdx.x >> 6);
  const int r = lane & 15, g = lane >> 4;

  // rows past the workgroup's keypoints stay zero
  if constexpr (W < kTileRows) {
    for (int i = (int)threadIdx.x; i < (kTileRows - W) * MI; i += 64 * W) sX[W + i / MI][i % MI] = 0;
  }

  // ---- the 8 nearest tracks with a flow (keypoint j = j0 + wave) -----------
  const int j = j0 + wv;
  const Kp* live = cd.state[Q];
  Kp me{};
  if (j < n) me = live[j];
  const double mx = (double)me.x, my = (double)me.y;
  // the patch's pixels of the previous frame, loaded now so that they arrive
  // during the search
  int px4[4];
  patch_load(cd.lvl[fc.pyr_prev][0], cd.pitch[0], cd.w, cd.h, me.x, me.y, lane, j < n, px4);
  // this wave's weight slices (hidden tiles wv, wv + W, ...): loaded behind
  // the first chunk's staging loads, so the search (LDS only) does not wait
  // for them and their latency hides behind it
  const uint16_t z8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bf16x8 w1[kTPW], w2[kTPW][MH / 32], w3[MH / 32];
  float b1[kTPW], b2[kTPW], b3 = 0.f;
  // this lane's best eight exact keys. The camera's tracks are staged in LDS
  // chunk by chunk (no flow: NaN); the lane visits tracks lane, lane + 64, ...
  // of a chunk, so indices rise along its visits
  Top8 top;
  top.clear();
  for (int c0 = 0; c0 < n; c0 += kCandChunk) {
    const int nc = min(kCandChunk, n - c0);
    __syncthreads();  // the previous chunk has been read
    for (int i = (int)threadIdx.x; i < nc; i += 64 * W) {
      const Kp o = live[c0 + i];
      sCand[i] = o.age >= 1 ? make_float2(o.x, o.y) : make_float2(__int_as_float(0x7FC00000), 0.f);
    }
    __syncthreads();
    if (c0 == 0) {
#pragma unroll
      for (int t = 0; t < kTPW; ++t) {
        const int tile = wv + W * t;
        w1[t] = pack8(z8);
        b1[t] = b2[t] = 0.f;
#pragma unroll
        for (int kc = 0; kc < MH / 32; ++kc) w2[t][kc] = pack8(z8);
        if (tile < kHidTiles) {
          const int jn = 16 * tile + r;
          w1[t] = load8(M.W1b + (size_t)jn * MI + 8 * g);
#pragma unroll
          for (int kc = 0; kc < MH / 32; ++kc) w2[t][kc] = load8(M.W2b + (size_t)jn * MH + 32 * kc + 8 * g);
          b1[t] = M.P[OFF_B1 + jn];
          b2[t] = M.P[OFF_B2 + jn];
        }
      }
#pragma unroll
      for (int kc = 0; kc < MH / 32; ++kc) w3[kc] = pack8(z8);
      if (wv == 0 && r < MO) {
#pragma unroll
        for (int kc = 0; kc < MH / 32; ++kc) w3[kc] = load8(M.W3b + (size_t)r * MH + 32 * kc + 8 * g);
        b3 = M.P[OFF_B3 + r];
      }
    }
    if (j < n) {
      for (int k0 = 0; k0 < nc; k0 += 64) {
        const int k = k0 + lane;
        if (k < nc) {
          const float2 e = sCand[k];
          if (e.x == e.x) top.offer(e.x, e.y, mx, my, c0 + k);  // a track with a flow
        }
      }
    }
  }
  // lane r < 8: the r-th nearest track (nearest first)
  const int best_ix = j < n ? top.extract(lane) : kNone;
  if (j < n) {
    float* f = feat + (size_t)(cd.row_off + j) * MI;
    {
      // lane r < 8 holds the r-th neighbour (nearest first)
      float fx = 0.f, fy = 0.f;
      if (lane < 8 && best_ix != kNone) {
        const Kp o = live[best_ix];
        fx = (o.x - o.px) * 0.0625f;
        fy = (o.y - o.py) * 0.0625f;
      }
      if (lane < 8) {
        reinterpret_cast<float2*>(f)[lane] = make_float2(fx, fy);
        sX[wv][2 * lane] = bf16_bits(fx);
        sX[wv][2 * lane + 1] = bf16_bits(fy);
      }
    }

    // pooled patch of the previous frame
    float v;
    const int cell = patch_pool(px4, lane, v);
    if (cell >= 0) {
      f[16 + cell] = v;
      sX[wv][16 + cell] = bf16_bits(v);
    }
  } else if (lane < MI) {
    sX[wv][lane] = 0;  // a row past the live keypoints (its output is not stored)
  }
  __syncthreads();

  // ---- network: 32 -> 128 -> 128 -> 3 --------------------------------------
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < kTPW; ++t) {
    const int tile = wv + W * t;
    if (tile < kHidTiles) {
      const f32x4 acc = mfma(load8(&sX[r][8 * g]), w1[t], zero);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 4 * g + q;
        sH[row][16 * tile + r] = row < W && j0 + row < n ? bf16_bits(fmaxf(acc[q] + b1[t], 0.f)) : (uint16_t)0;
      }
    }
  }
  __syncthreads();
  f32x4 acc2[kTPW];
#pragma unroll
  for (int t = 0; t < kTPW; ++t) {
    acc2[t] = zero;
    if (wv + W * t < kHidTiles) {
#pragma unroll
      for (int kc = 0; kc < MH / 32; ++kc) acc2[t] = mfma(load8(&sH[r][32 * kc + 8 * g]), w2[t][kc], acc2[t]);
    }
  }
  __syncthreads();  // every wave has read h1
#pragma unroll
  for (int t = 0; t < kTPW; ++t) {
    const int tile = wv + W * t;
    if (tile < kHidTiles) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 4 * g + q;
        sH[row][16 * tile + r] = row < W && j0 + row < n ? bf16_bits(fmaxf(acc2[t][q] + b2[t], 0.f)) : (uint16_t)0;
      }
    }
  }
  __syncthreads();
  if (wv == 0) {
    f32x4 acc = zero;
#pragma unroll
    for (int kc = 0; kc < MH / 32; ++kc) acc = mfma(load8(&sH[r][32 * kc + 8 * g]), w3[kc], acc);
    if (r < MO) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 4 * g + q;
        if (row < W && j0 + row < n) guess[(size_t)(cd.row_off + j0 + row) * MO + r] = acc[q] + b3;
      }
    }
  }
}

}  // namespace

template <int W>
static hipError_t launch_learn_w(const CamDesc* d_cams, const FrameTable* d_frame, const Counters* d_cnt,
                                 const CamDesc* h_cams, int cam_begin, int cam_end, const MlpDev& M, float* d_feat,
                                 float* d_guess, hipStream_t s) {
  int blocks = 0;
  for (int c = cam_begin; c < cam_end; ++c) blocks += (h_cams[c].cap + W - 1) / W;
  launch_kernel(k_learn<W>, dim3(blocks), dim3(64 * W), 0, s, d_cams, d_frame, d_cnt, cam_begin, cam_end, M, d_feat,
                d_guess);
  return hipGetLastError();
}

hipError_t launch_learn(const CamDesc* d_cams, const FrameTable* d_frame, const Counters* d_cnt, const CamDesc* h_cams,
                        int cam_begin, int cam_end, const MlpDev& M, float* d_feat, float* d_guess, int waves,
                        hipStream_t s) {
  if (cam_end <= cam_begin) return hipSuccess;
  switch (waves) {
    case 4: return launch_learn_w<4>(d_cams, d_frame, d_cnt, h_cams, cam_begin, cam_end, M, d_feat, d_guess, s);
    case 8: return launch_learn_w<8>(d_cams, d_frame, d_cnt, h_cams, cam_begin, cam_end, M, d_feat, d_guess, s);
    case 16: return launch_learn_w<16>(d_cams, d_frame, d_cnt, h_cams, cam_begin, cam_end, M, d_feat, d_guess, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vio
