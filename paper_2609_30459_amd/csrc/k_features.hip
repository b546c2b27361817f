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
#include "mfma_ops.h"
#include "wave_ops.h"

namespace vio {
namespace {

constexpr int kTileRows = 16;     // rows of one MFMA tile: at most 16 keypoints per workgroup
constexpr int kHidTiles = MH / 16;  // 16-unit output tiles of a hidden layer
constexpr int kCandChunk = 2048;  // tracks staged in LDS at a time (16 KB)
constexpr int kNone = 0x7FFFFFFF;
constexpr uint64_t kInfBits = 0x7FF0000000000000ull;  // +inf as a key: an empty place

}  // namespace

namespace {

// Exact neighbour key: the squared distance as the bits of a non-negative
// double (their unsigned order is the numeric order), then the index.
struct NKey {
  uint64_t d;
  int ix;
};

__device__ __forceinline__ bool nkey_less(const NKey& a, const NKey& b) {
  return a.d < b.d || (a.d == b.d && a.ix < b.ix);
}

// The smallest key over the 64 lanes, in every lane (every lane must be
// active): a minimum over each quad (quad permutes), over each 16-lane row
// (rotations by 4 and 8), then across the rows (permlane32 and permlane16
// swaps) -- DPP and permlane moves only, no LDS round trip.
template <int Ctrl>
__device__ __forceinline__ void min_dpp(NKey& k) {
  NKey p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)k.d, Ctrl, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(k.d >> 32), Ctrl, 0xF, 0xF, false);
  p.d = ((uint64_t)hi << 32) | lo;
  p.ix = __builtin_amdgcn_update_dpp(0, k.ix, Ctrl, 0xF, 0xF, false);
  const bool take = nkey_less(p, k);
  // field by field: a select of the whole struct goes through private memory
  k.d = take ? p.d : k.d;
  k.ix = take ? p.ix : k.ix;
}

template <bool k32>
__device__ __forceinline__ void min_swap(NKey& k) {
  const uint32_t lo0 = (uint32_t)k.d, hi0 = (uint32_t)(k.d >> 32), ix0 = (uint32_t)k.ix;
  // swap(v, v) leaves the partner row's value in one of the two results, the
  // own value in the other; the minimum of the two is the same either way
  const auto a = k32 ? __builtin_amdgcn_permlane32_swap(lo0, lo0, false, false)
                     : __builtin_amdgcn_permlane16_swap(lo0, lo0, false, false);
  const auto b = k32 ? __builtin_amdgcn_permlane32_swap(hi0, hi0, false, false)
                     : __builtin_amdgcn_permlane16_swap(hi0, hi0, false, false);
  const auto c = k32 ? __builtin_amdgcn_permlane32_swap(ix0, ix0, false, false)
                     : __builtin_amdgcn_permlane16_swap(ix0, ix0, false, false);
  const uint32_t la = a[0], lb = a[1], ha = b[0], hb = b[1], ia = c[0], ib = c[1];
  NKey x{((uint64_t)ha << 32) | la, (int)ia}, y{((uint64_t)hb << 32) | lb, (int)ib};
  const bool take = nkey_less(y, x);
  k.d = take ? y.d : x.d;
  k.ix = take ? y.ix : x.ix;
}

__device__ __forceinline__ void wave_min_key(NKey& k) {
  min_dpp<0xB1>(k);   // quad lane ^ 1
  min_dpp<0x4E>(k);   // quad lane ^ 2
  min_dpp<0x124>(k);  // row rotate by 4
  min_dpp<0x128>(k);  // row rotate by 8
  min_swap<true>(k);  // rows 0, 1 <-> 2, 3
  min_swap<false>(k); // rows 0 <-> 1, 2 <-> 3
}

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
  __shared__ __align__(16) uint16_t sX[kTileRows][MI];  // bf16 inputs, one row per keypoint
  __shared__ __align__(16) uint16_t sH[kTileRows][MH];  // h1, then h2
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
  // during the search (lane: a row of the 16 x 16 patch, 4 columns)
  const int rx = (int)floorf(me.x + 0.5f), ry = (int)floorf(me.y + 0.5f);
  const uint8_t* img = cd.lvl[fc.pyr_prev][0];
  const int pitch = cd.pitch[0];
  const int prow = lane >> 2, col4 = (lane & 3) * 4;
  const int yy = min(max(ry - 8 + prow, 0), cd.h - 1);
  int px4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) px4[k] = j < n ? img[(size_t)yy * pitch + min(max(rx - 8 + col4 + k, 0), cd.w - 1)] : 0;
  // this wave's weight slices (hidden tiles wv, wv + W, ...): loaded behind
  // the first chunk's staging loads, so the search (LDS only) does not wait
  // for them and their latency hides behind it
  const uint16_t z8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bf16x8 w1[kTPW], w2[kTPW][MH / 32], w3[MH / 32];
  float b1[kTPW], b2[kTPW], b3 = 0.f;
  // this lane's best eight exact keys, ascending; +inf / kNone: empty. The
  // camera's tracks are staged in LDS chunk by chunk (no flow: NaN); the lane
  // visits tracks lane, lane + 64, ... of a chunk, so indices rise along its
  // visits and a tie in distance keeps the earlier (smaller id) key
  uint64_t ld[8];
  int li[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    ld[s] = kInfBits;
    li[s] = kNone;
  }
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
          if (e.x == e.x) {  // a track with a flow
            const double dx = (double)e.x - mx, dy = (double)e.y - my;
            const uint64_t kd = (uint64_t)__double_as_longlong(dx * dx + dy * dy);
            const int ki = c0 + k;
            if (kd < ld[7]) {
              bool lt[8];
#pragma unroll
              for (int s = 0; s < 8; ++s) lt[s] = kd < ld[s];
#pragma unroll
              for (int s = 7; s > 0; --s) {
                ld[s] = lt[s - 1] ? ld[s - 1] : (lt[s] ? kd : ld[s]);
                li[s] = lt[s - 1] ? li[s - 1] : (lt[s] ? ki : li[s]);
              }
              ld[0] = lt[0] ? kd : ld[0];
              li[0] = lt[0] ? ki : li[0];
            }
          }
        }
      }
    }
  }
  // eight rounds: the wave minimum of the lanes' heads is the next nearest;
  // its lane drops it (indices are unique, so exactly one lane does)
  int best_ix = kNone;
  if (j < n) {
#pragma unroll 1
    for (int r8 = 0; r8 < 8; ++r8) {
      NKey m{ld[0], li[0]};
      wave_min_key(m);
      if (lane == r8) best_ix = m.ix;
      const bool pop = li[0] == m.ix && m.ix != kNone;
#pragma unroll
      for (int s = 0; s < 7; ++s) {
        ld[s] = pop ? ld[s + 1] : ld[s];
        li[s] = pop ? li[s + 1] : li[s];
      }
      ld[7] = pop ? kInfBits : ld[7];
      li[7] = pop ? kNone : li[7];
    }
  }
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
    const int ps = px4[0] + px4[1] + px4[2] + px4[3];
    // cell (row / 4, lane & 3): the four lanes of a 16-lane row that agree in
    // bits 0..1 share a cell (rotations by 8 and 4 sum them)
    int csum = ps + dpp_i<0x128>(ps);
    csum += dpp_i<0x124>(csum);
    const int tot = wave_total_i(ps);
    if (((lane >> 2) & 3) == 0) {
      const int cell = (prow >> 2) * 4 + (lane & 3);
      const float v = tot > 0 ? (float)(csum * 16) / (float)tot - 1.f : 0.f;
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
