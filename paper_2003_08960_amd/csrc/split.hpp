// Two-term splits of an FP32 value into 16-bit formats (hi = RNE(x),
// lo = RNE(x - hi)), the operand storage of the split-precision depth
// transforms: hi*hi + hi*lo + lo*hi carries about 16 significant bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace ssoct {

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// hi + lo split of one real value, packed as hi | lo << 16 (FMT = HF_F16 or HF_BF16)
template <int FMT>
__device__ __forceinline__ uint32_t split_pack(float x) {
  if constexpr (FMT == HF_F16) {
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)(x - (float)h);
    return (uint32_t)__builtin_bit_cast(uint16_t, h) | ((uint32_t)__builtin_bit_cast(uint16_t, l) << 16);
  } else {
    const uint16_t h = bf16_rne(x);
    const uint16_t l = bf16_rne(x - bf16_val(h));
    return (uint32_t)h | ((uint32_t)l << 16);
  }
}

}  // namespace ssoct
