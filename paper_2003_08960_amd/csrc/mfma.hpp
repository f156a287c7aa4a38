// MFMA operand types and helpers shared by the depth-transform kernels.
// v_mfma_f32_32x32x2_f32: lane l holds A[l % 32][l / 32] and B[l / 32][l % 32];
// v_mfma_f32_32x32x16_{f16,bf16}: lane l holds A[l % 32][8 (l / 32) + 0..7]
// and B[8 (l / 32) + 0..7][l % 32]; both leave D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
// in accumulator register r of lane l.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace ssoct {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int PREC>
struct PrecTraits {
  static constexpr bool F32 = PREC == DP_F32;
  static constexpr bool SPLIT = PREC == DP_F16_SPLIT || PREC == DP_BF16_SPLIT;
  static constexpr bool BF = PREC == DP_BF16 || PREC == DP_BF16_SPLIT;
};

template <bool BF>
__device__ __forceinline__ v16f mfma_x16(uint4 a, uint4 b, v16f c) {
  if constexpr (BF) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), c, 0, 0,
                                                  0);
  }
}

// lo 16 bits of x0, x1 packed, and hi 16 bits packed
__device__ __forceinline__ uint32_t pack_lo(uint32_t x0, uint32_t x1) { return __builtin_amdgcn_perm(x1, x0, 0x05040100u); }
__device__ __forceinline__ uint32_t pack_hi(uint32_t x0, uint32_t x1) { return __builtin_amdgcn_perm(x1, x0, 0x07060302u); }

}  // namespace ssoct
