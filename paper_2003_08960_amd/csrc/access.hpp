// Global loads and stores of data that one kernel touches exactly once
// (streamed frames, the hologram stack, the volume).  With NT = true they
// are non-temporal (the streaming hint: no reuse expected in the caches).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssoct {

typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef uint32_t nt_u2 __attribute__((ext_vector_type(2)));
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ float2 ld_once(const float2* p) {
  if constexpr (NT) {
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
    return make_float2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ uint2 ld_once(const uint2* p) {
  if constexpr (NT) {
    const nt_u2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u2*>(p));
    return make_uint2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ uint4 ld_once(const uint4* p) {
  if constexpr (NT) {
    const nt_u4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ void st_once(float2* p, float2 v) {
  if constexpr (NT) {
    nt_f2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f2*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void st_once(uint2* p, uint2 v) {
  if constexpr (NT) {
    nt_u2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<nt_u2*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void st_once(float* p, float v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

}  // namespace ssoct
