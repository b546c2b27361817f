// BF16 MFMA helpers of the learned-initialisation network (gfx950,
// v_mfma_f32_16x16x32_bf16, FP32 accumulation) and its parameter layout,
// shared by the network kernels and the fused feature + network kernel.
//
// Operand layout (16x16x32): lane l holds A[l%16][8(l/16) .. +7] (a row
// segment of 8 bf16), B[8(l/16) .. +7][l%16] (a column segment) and returns
// D[4(l/16) + q][l%16], q = 0..3.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vio_mlp.h"

namespace vio {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MI = VIO_MLP_IN, MH = VIO_MLP_HIDDEN, MO = VIO_MLP_OUT, NP = VIO_MLP_NPARAM;
constexpr int OFF_W1 = 0, OFF_B1 = MH * MI, OFF_W2 = OFF_B1 + MH, OFF_B2 = OFF_W2 + MH * MH, OFF_W3 = OFF_B2 + MH,
              OFF_B3 = OFF_W3 + MO * MH;
static_assert(OFF_B3 + MO == NP, "parameter layout");

// float -> bfloat16 bits, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ bf16x8 pack8(const uint16_t v[8]) {
  uint4 u;
  u.x = v[0] | ((uint32_t)v[1] << 16);
  u.y = v[2] | ((uint32_t)v[3] << 16);
  u.z = v[4] | ((uint32_t)v[5] << 16);
  u.w = v[6] | ((uint32_t)v[7] << 16);
  return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

}  // namespace vio
