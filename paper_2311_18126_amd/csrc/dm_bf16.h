// dm_bf16.h -- bfloat16 rounding and the bfloat16 matrix-core product, shared by the network
// kernels (dm_mlp.hip) and the warm start inside the step kernel (dm_warm.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 dm_bf16x8 __attribute__((ext_vector_type(8)));
typedef float dm_f32x4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bit pattern, round to nearest, ties to even; NaN -> quiet NaN.
__device__ __forceinline__ uint16_t dm_bf16_bits(float v) {
  const uint32_t b = __float_as_uint(v);
  if (v != v) return 0x7FC0;
  return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// C += A B for one 16 x 16 x 32 tile (v_mfma_f32_16x16x32_bf16).  Lane l supplies
// A[l % 16][8 (l / 16) + 0..7] and B[8 (l / 16) + 0..7][l % 16] and holds
// C[4 (l / 16) + j][l % 16], j = 0..3.
__device__ __forceinline__ dm_f32x4 dm_mfma_bf16(dm_bf16x8 a, dm_bf16x8 b, dm_f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
