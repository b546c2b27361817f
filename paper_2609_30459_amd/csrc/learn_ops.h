// Wave-level pieces of the learned initialisation's inputs (the eight nearest
// tracks with a flow, the pooled patch) and of the network on one row,
// shared by the learned-stage kernel (several keypoints per workgroup, the
// network on 16-row tiles) and the tracker's fused prologue (one keypoint per
// wave, the network on one row). Both compute bit-identical features and
// network outputs: the same exact keys, the same pooling arithmetic, and the
// same MFMA sequence per row (an MFMA's output row depends only on its own
// input row).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fe_common.h"
#include "mfma_ops.h"
#include "wave_ops.h"

namespace vio {

constexpr int kNone = 0x7FFFFFFF;
constexpr uint64_t kInfBits = 0x7FF0000000000000ull;  // +inf as a key: an empty place

// Exact neighbour key: the squared distance as the bits of a non-negative
// double (their unsigned order is the numeric order), then the index; keys are
// compared lexicographically.

// Minimum of an unsigned value over the 64 lanes, in every lane: quads, rows
// (rotations by 4 and 8), then the row swaps.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad lane ^ 1
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad lane ^ 2
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));  // row rotate by 4
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));  // row rotate by 8
  const auto a = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  v = min((uint32_t)a[0], (uint32_t)a[1]);
  const auto b = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return min((uint32_t)b[0], (uint32_t)b[1]);
}

// The index of the smallest key (d, ix) over the 64 lanes, in every lane (every
// lane must be active), taken word by word.
// The high words of d first; when a single lane holds their minimum (the usual
// case: a tie needs equal exponents and top 20 mantissa bits) its key is the
// minimum and its index is read from it; otherwise the low words among the
// tied lanes, then the indices among the lanes tied on both (indices are
// non-negative, so their unsigned order is their order).
__device__ __forceinline__ int wave_min_head(uint64_t d, int ix) {
  const uint32_t hi = (uint32_t)(d >> 32), lo = (uint32_t)d;
  const uint32_t mh = wave_min_u32(hi);
  const uint64_t tied = __ballot(hi == mh);
  if (__popcll(tied) == 1) return __builtin_amdgcn_readlane(ix, (int)__ffsll((long long)tied) - 1);
  const uint32_t ml = wave_min_u32(hi == mh ? lo : 0xFFFFFFFFu);
  return (int)wave_min_u32(hi == mh && lo == ml ? (uint32_t)ix : 0xFFFFFFFFu);
}

// A lane's best eight keys so far, ascending (+inf / kNone: an empty place).
struct Top8 {
  uint64_t d[8];
  int ix[8];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      d[s] = kInfBits;
      ix[s] = kNone;
    }
  }
  // Offers the track at index ki, position (ex, ey), to the keypoint at
  // (mx, my); the differences and squares of float positions are exact in
  // double. A lane offers its tracks in rising index order, so a tie in
  // distance keeps the earlier (smaller id) key.
  __device__ __forceinline__ void offer(float ex, float ey, double mx, double my, int ki) {
    const double dx = (double)ex - mx, dy = (double)ey - my;
    const uint64_t kd = (uint64_t)__double_as_longlong(dx * dx + dy * dy);
    if (kd < d[7]) {
      bool lt[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) lt[s] = kd < d[s];
#pragma unroll
      for (int s = 7; s > 0; --s) {
        d[s] = lt[s - 1] ? d[s - 1] : (lt[s] ? kd : d[s]);
        ix[s] = lt[s - 1] ? ix[s - 1] : (lt[s] ? ki : ix[s]);
      }
      d[0] = lt[0] ? kd : d[0];
      ix[0] = lt[0] ? ki : ix[0];
    }
  }
  // Eight rounds: the wave minimum of the lanes' heads is the next nearest;
  // its lane drops it (indices are unique, so exactly one lane does). Lane
  // r < 8 receives the r-th nearest index (kNone: fewer tracks). Every lane
  // of the wave must take part.
  __device__ __forceinline__ int extract(int lane) {
    int best = kNone;
#pragma unroll 1
    for (int r8 = 0; r8 < 8; ++r8) {
      const int mix = wave_min_head(d[0], ix[0]);
      if (lane == r8) best = mix;
      const bool pop = ix[0] == mix && mix != kNone;
#pragma unroll
      for (int s = 0; s < 7; ++s) {
        d[s] = pop ? d[s + 1] : d[s];
        ix[s] = pop ? ix[s + 1] : ix[s];
      }
      d[7] = pop ? kInfBits : d[7];
      ix[7] = pop ? kNone : ix[7];
    }
    return best;
  }
};

// The previous frame's level-0 patch of 16 x 16 pixels around round(p),
// clamped to the image: lane l loads row l / 4, columns 4 (l % 4) .. + 3.
__device__ __forceinline__ void patch_load(const uint8_t* img, int pitch, int w, int h, float x, float y, int lane,
                                           bool valid, int px4[4]) {
  const int rx = (int)floorf(x + 0.5f), ry = (int)floorf(y + 0.5f);
  const int prow = lane >> 2, col4 = (lane & 3) * 4;
  const int yy = min(max(ry - 8 + prow, 0), h - 1);
#pragma unroll
  for (int k = 0; k < 4; ++k) px4[k] = valid ? img[(size_t)yy * pitch + min(max(rx - 8 + col4 + k, 0), w - 1)] : 0;
}

// Pooled patch: cell_sum * 16 / patch_sum - 1 over 4 x 4 cells (integer sums,
// one correctly rounded division). Returns the cell this lane reports
// (-1: none) and its value; the four lanes of a 16-lane row that agree in
// bits 0..1 share a cell (rotations by 8 and 4 sum them). Every lane of the
// wave must take part.
__device__ __forceinline__ int patch_pool(const int px4[4], int lane, float& v) {
  const int ps = px4[0] + px4[1] + px4[2] + px4[3];
  int csum = ps + dpp_i<0x128>(ps);
  csum += dpp_i<0x124>(csum);
  const int tot = wave_total_i(ps);
  v = tot > 0 ? (float)(csum * 16) / (float)tot - 1.f : 0.f;
  return ((lane >> 2) & 3) == 0 ? ((lane >> 4) * 4 + (lane & 3)) : -1;
}

// The network's weights as one wave's MFMA B operands for one row: lane l
// holds W1[16 t + l % 16][8 (l / 16) .. + 7] for hidden tile t, the same for
// W2 and its four 32-wide K chunks, and W3's row l % 16 (zero past the three
// outputs). Loaded in two parts, so that the first can be in flight during
// the neighbour search and the second during the extraction.
struct RowWeights {
  bf16x8 w1[MH / 16];
  bf16x8 w2[MH / 16][MH / 32];
  bf16x8 w3[MH / 32];
  __device__ __forceinline__ void load_first(const uint16_t* __restrict__ W1b, const uint16_t* __restrict__ W2b,
                                             int lane) {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < MH / 16; ++t) w1[t] = load8(W1b + (size_t)(16 * t + r) * MI + 8 * g);
#pragma unroll
    for (int t = 0; t < MH / 32; ++t)
#pragma unroll
      for (int kc = 0; kc < MH / 32; ++kc) w2[t][kc] = load8(W2b + (size_t)(16 * t + r) * MH + 32 * kc + 8 * g);
  }
  __device__ __forceinline__ void load_second(const uint16_t* __restrict__ W2b, const uint16_t* __restrict__ W3b,
                                              int lane) {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = MH / 32; t < MH / 16; ++t)
#pragma unroll
      for (int kc = 0; kc < MH / 32; ++kc) w2[t][kc] = load8(W2b + (size_t)(16 * t + r) * MH + 32 * kc + 8 * g);
    const uint16_t z8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < MH / 32; ++kc) w3[kc] = r < MO ? load8(W3b + (size_t)r * MH + 32 * kc + 8 * g) : pack8(z8);
  }
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The network on one row by one wave, with the MFMA sequence of the 16-row
// kernels (row 0 of each tile is the row; the other rows are zero). x: the
// row's 32 bf16 inputs and h: 128 bf16 of scratch, both in the wave's own LDS
// (16-byte aligned); W: the loaded weights; returns the outputs in every lane.
__device__ __forceinline__ void mlp_row(const RowWeights& W, const float* __restrict__ P, uint16_t* x, uint16_t* h,
                                        int lane, float out[3]) {
  const int r = lane & 15, g = lane >> 4;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  const uint16_t z8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bf16x8 zb = pack8(z8);
  float b1[MH / 16], b2[MH / 16];
#pragma unroll
  for (int t = 0; t < MH / 16; ++t) {
    b1[t] = lane < 16 ? P[OFF_B1 + 16 * t + lane] : 0.f;
    b2[t] = lane < 16 ? P[OFF_B2 + 16 * t + lane] : 0.f;
  }
  const float b3 = r < MO ? P[OFF_B3 + r] : 0.f;
  wave_sync_lds();
  // layer 1: lanes 16 g (row 0) carry inputs 8 g .. 8 g + 7
  const bf16x8 a1 = r == 0 ? load8(x + 8 * g) : zb;
#pragma unroll
  for (int t = 0; t < MH / 16; ++t) {
    const f32x4 acc = mfma(a1, W.w1[t], zero);
    if (lane < 16) h[16 * t + lane] = bf16_bits(fmaxf(acc[0] + b1[t], 0.f));
  }
  wave_sync_lds();
  // layer 2: h1 as four 32-wide K chunks, read before h2 overwrites them
  bf16x8 a2[MH / 32];
#pragma unroll
  for (int kc = 0; kc < MH / 32; ++kc) a2[kc] = r == 0 ? load8(h + 32 * kc + 8 * g) : zb;
  wave_sync_lds();
#pragma unroll
  for (int t = 0; t < MH / 16; ++t) {
    f32x4 acc = zero;
#pragma unroll
    for (int kc = 0; kc < MH / 32; ++kc) acc = mfma(a2[kc], W.w2[t][kc], acc);
    if (lane < 16) h[16 * t + lane] = bf16_bits(fmaxf(acc[0] + b2[t], 0.f));
  }
  wave_sync_lds();
  // layer 3: output columns 0..2
  f32x4 acc = zero;
#pragma unroll
  for (int kc = 0; kc < MH / 32; ++kc) acc = mfma(r == 0 ? load8(h + 32 * kc + 8 * g) : zb, W.w3[kc], acc);
  const float o = acc[0] + b3;
#pragma unroll
  for (int k = 0; k < MO; ++k) out[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, o), k));
}

}  // namespace vio
