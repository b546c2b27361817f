// Wave-level helpers for gfx950 (wave64): DPP lane exchanges and sums of
// several values at once over the 64 lanes of a wave. Every helper must be
// called by the whole wave (all 64 lanes active).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vio {

template <int ctrl>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
}

// One exchange stage inside the 16-lane rows: the partner of a lane differs
// from it in lane bit BIT and agrees below it (CTRL: quad_perm [1,0,3,2] for
// bit 0, quad_perm [2,3,0,1] for bit 1, row_ror:4 for bit 2, row_ror:8 for
// bit 3). With N > 1 values, value pair (2i, 2i+1) becomes value i: a lane
// keeps the member its bit selects and adds the partner's copy of it (the
// partner, with the other bit, sends exactly that member).
template <int CTRL, int BIT, int N>
__device__ __forceinline__ void xstage(float* v, int lane) {
  if constexpr (N == 1) {
    v[0] += dpp<CTRL>(v[0]);
  } else {
    const bool b = (lane >> BIT) & 1;
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      const float keep = b ? v[2 * i + 1] : v[2 * i];
      const float send = b ? v[2 * i] : v[2 * i + 1];
      v[i] = keep + dpp<CTRL>(send);
    }
  }
}

// Sum of a row with its partner row: permlane32 swaps lanes 32..63 of one copy
// with lanes 0..31 of the other (rows 0,1 <-> 2,3), permlane16 the odd rows of
// one copy with the even rows of the other (rows 0 <-> 1, 2 <-> 3); the two
// results, added, give every lane its value plus the partner row's value in
// the same position.
__device__ __forceinline__ float rowswap_sum32(float x) {
  const auto p = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, x),
                                                  false, false);
  const unsigned a = p[0], b = p[1];  // (a bit cast of p[1] itself would read p[0])
  return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
}
__device__ __forceinline__ float rowswap_sum16(float x) {
  const auto p = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, x),
                                                  false, false);
  const unsigned a = p[0], b = p[1];  // (a bit cast of p[1] itself would read p[0])
  return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
}

// The four exchange stages over N values (N = 1, 2, 4, 8 or 16): returns, in
// lane j of every 16-lane row, sum (j mod N) of the row.
template <int N>
__device__ __forceinline__ float row_sums_pow2(const float* v, int lane) {
  static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "power of two up to 16");
  float w[N];
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = v[i];
  xstage<0xB1, 0, N>(w, lane);
  xstage<0x4E, 1, (N > 2 ? N / 2 : 1)>(w, lane);
  xstage<0x124, 2, (N > 4 ? N / 4 : 1)>(w, lane);
  xstage<0x128, 3, (N > 8 ? N / 8 : 1)>(w, lane);
  return w[0];
}

// v[i] <- sum of v[i] over the 64 lanes, i < N (N = 1, 2, 4, 8 or 16), as
// wave-uniform values.
template <int N>
__device__ __forceinline__ void wave_sums_pow2(float* v, int lane) {
  const float x = rowswap_sum16(rowswap_sum32(row_sums_pow2<N>(v, lane)));
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), i));
}

// v[i] <- wave sum of v[i] for i < M, in chunks of 16, 8, 4, 2, 1
template <int M>
__device__ __forceinline__ void wave_sums(float* v, int lane) {
  if constexpr (M > 0) {
    constexpr int C = M >= 16 ? 16 : M >= 8 ? 8 : M >= 4 ? 4 : M >= 2 ? 2 : 1;
    wave_sums_pow2<C>(v, lane);
    wave_sums<M - C>(v + C, lane);
  }
}

__device__ __forceinline__ float wave_sum(float x, int lane) {
  wave_sums_pow2<1>(&x, lane);
  return x;
}

// Sums for two items per wave, one per 32-lane half, each lane of a half
// carrying two values of its item: a[i] at position g = lane mod 32 and b[i]
// at position g + 32 of the item's 64. a[i] <- the item's total of value i,
// uniform across the half, summed in exactly the order wave_sums_pow2 sums 64
// values held one per lane: the row stages run on a and on b alone (the rows
// of positions 0..31 and 32..63), a + b stands in for the permlane32 swap, and
// the permlane16 swap pairs the two rows of each half. row_newbcast:i then
// hands lane i's total to its row -- lane i's also for a single value (N = 1),
// which every lane holds but each through its own order of the row's terms:
// lane 0's is the one wave_sums_pow2 reads.
template <int ctrl>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
}
template <int N, int i = 0>
__device__ __forceinline__ void row_broadcasts(float* v, float x) {
  if constexpr (i < N) {
    v[i] = dpp_mov<0x150 + i>(x);
    row_broadcasts<N, i + 1>(v, x);
  }
}
template <int N>
__device__ __forceinline__ void half_sums_pow2(float* a, const float* b, int lane) {
  row_broadcasts<N>(a, rowswap_sum16(row_sums_pow2<N>(a, lane) + row_sums_pow2<N>(b, lane)));
}

// a[i] <- half-wave totals of (a[i], b[i]) for i < M, chunked as wave_sums<M>
template <int M>
__device__ __forceinline__ void half_sums(float* a, const float* b, int lane) {
  if constexpr (M > 0) {
    constexpr int C = M >= 16 ? 16 : M >= 8 ? 8 : M >= 4 ? 4 : M >= 2 ? 2 : 1;
    half_sums_pow2<C>(a, b, lane);
    half_sums<M - C>(a + C, b + C, lane);
  }
}

// out[i] <- half-wave totals of gen(i, 0) + gen(i, 1) for i in [OFF, OFF + M),
// chunked and summed as half_sums (and so as wave_sums<M> on out + OFF), each
// chunk's values made just before its stages (a's, then b's), so only one
// chunk of one position is held at a time.
template <int M, int OFF, class Gen>
__device__ __forceinline__ void half_sums_of(float* out, const Gen& gen, int lane) {
  if constexpr (M > 0) {
    constexpr int C = M >= 16 ? 16 : M >= 8 ? 8 : M >= 4 ? 4 : M >= 2 ? 2 : 1;
    float w[C];
#pragma unroll
    for (int i = 0; i < C; ++i) w[i] = gen(OFF + i, 0);
    const float xa = row_sums_pow2<C>(w, lane);
#pragma unroll
    for (int i = 0; i < C; ++i) w[i] = gen(OFF + i, 1);
    row_broadcasts<C>(out + OFF, rowswap_sum16(xa + row_sums_pow2<C>(w, lane)));
    half_sums_of<M - C, OFF + C>(out, gen, lane);
  }
}

__device__ __forceinline__ float half_sum(float a, float b, int lane) {
  half_sums_pow2<1>(&a, &b, lane);
  return a;
}

// Votes over each 32-lane half (all 64 lanes active): the half's all / any,
// decided on the scalar unit from the ballot and handed back to the lanes as a
// lane mask.
__device__ __forceinline__ uint64_t half_mask(bool h0, bool h1) {
  return (h0 ? 0x00000000FFFFFFFFull : 0ull) | (h1 ? 0xFFFFFFFF00000000ull : 0ull);
}
__device__ __forceinline__ bool half_all(bool p, int) {
  const uint64_t m = __ballot(p);
  return __builtin_amdgcn_inverse_ballot_w64(half_mask((uint32_t)m == 0xFFFFFFFFu, (uint32_t)(m >> 32) == 0xFFFFFFFFu));
}
__device__ __forceinline__ bool half_any(bool p, int) {
  const uint64_t m = __ballot(p);
  return __builtin_amdgcn_inverse_ballot_w64(half_mask((uint32_t)m != 0u, (uint32_t)(m >> 32) != 0u));
}

template <int ctrl>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, ctrl, 0xF, 0xF, false);
}

// Integer total over the 64 lanes (the tree of wave_sums_pow2<1>), as a
// wave-uniform value.
__device__ __forceinline__ int wave_total_i(int x) {
  x += dpp_i<0xB1>(x);
  x += dpp_i<0x4E>(x);
  x += dpp_i<0x124>(x);
  x += dpp_i<0x128>(x);
  {
    const auto p = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
    const unsigned a = p[0], b = p[1];
    x = (int)(a + b);
  }
  {
    const auto p = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
    const unsigned a = p[0], b = p[1];
    x = (int)(a + b);
  }
  return __builtin_amdgcn_readfirstlane(x);
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4, 8
// inside each 16-lane row, then row_bcast:15 and row_bcast:31 carry the row
// totals forward (lanes without a source add the old value 0).
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return x;
}

}  // namespace vio
