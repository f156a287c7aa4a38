// Depth transform of Eq. 7 as a radix FFT along the sweep axis (FP32), the
// HBM-bound alternative to the dense DFT-matrix product: the paper computes
// this transform with a 1-D FFT per pixel, and on gfx950 its 5 T log2 T
// flops per pixel are far below what the 16 B/voxel of traffic allow.
//
// Four-step split T = 16 T2 (T2 = 1..16): t = t1 + 16 t2, q = q2 + T2 q1,
//   V[q2 + T2 q1] = sum_t1 w16^(q1 t1) [ wT^(q2 t1) sum_t2 wT2^(q2 t2) h[t1 + 16 t2] ]
// with w_n = exp(-2 pi i / n) (forward; the adjoint conjugates every factor).
// A workgroup owns PX consecutive pixels and all T frames; thread (t1, px)
// does the T2-point DFTs of stage A, the twiddles go on in registers, the
// products cross LDS once, and thread (q2, px) does the 16-point DFT of
// stage B.  Every global access is PX consecutive pixels of one frame or bin.
#include "access.hpp"
#include "fft_engine.hpp"
#include "internal.hpp"

namespace ssoct {

#ifndef SSOCT_DFFT_PX
#define SSOCT_DFFT_PX 32         // pixels per workgroup (threads = 16 PX)
#endif
#ifndef SSOCT_DFFT_NT
#define SSOCT_DFFT_NT 1          // non-temporal loads of H and stores of the volume (both touched once)
#endif

template <int T2, int DIR, int EPI, int PX>
__global__ __launch_bounds__(16 * PX) void k_depth_fft(const float2* __restrict__ H, const float2* __restrict__ wt,
                                                        void* __restrict__ out, int P) {
  constexpr int T = 16 * T2;
  constexpr int ED = -DIR;           // engine sign: forward depth DFT has exponent -2 pi i q t / T
  __shared__ float2 lds[T * PX];     // [q2][t1][px]
  const int px = threadIdx.x % PX, r = threadIdx.x / PX;   // r = t1 in stage A, q2 in stage B
  const int base = blockIdx.x * PX;
  const bool live = base + px < P;

  // stage A: DFT over t2 of h[r + 16 t2]
  float2 a[T2];
#pragma unroll
  for (int t2 = 0; t2 < T2; ++t2)
    a[t2] = live ? ld_once<SSOCT_DFFT_NT>(H + (size_t)(r + 16 * t2) * P + base + px) : make_float2(0.f, 0.f);
  if constexpr (T2 > 1) dft_small<T2, ED>(a);
#pragma unroll
  for (int q2 = 0; q2 < T2; ++q2) {
    float2 w = wt[(q2 * r) % T];     // exp(-2 pi i q2 t1 / T), FP64-derived
    if constexpr (DIR < 0) w = cconj(w);
    lds[(q2 * 16 + r) * PX + px] = q2 == 0 ? a[q2] : cmul(a[q2], w);
  }
  __syncthreads();
  if (r >= T2) return;

  // stage B: DFT over t1 for bin column q2 = r
  float2 b[16];
#pragma unroll
  for (int t1 = 0; t1 < 16; ++t1) b[t1] = lds[(r * 16 + t1) * PX + px];
  dft16<ED>(b);
  if (!live) return;
#pragma unroll
  for (int q1 = 0; q1 < 16; ++q1) {
    const size_t idx = (size_t)(r + T2 * q1) * P + base + px;
    if constexpr (EPI == EPI_ABS)
      st_once<SSOCT_DFFT_NT>(reinterpret_cast<float*>(out) + idx, sqrtf(b[q1].x * b[q1].x + b[q1].y * b[q1].y));
    else
      st_once<SSOCT_DFFT_NT>(reinterpret_cast<float2*>(out) + idx, b[q1]);
  }
}

template <int T2, int DIR, int EPI>
static hipError_t depth_fft_t(int P, const float2* H, const float2* wt, void* out, hipStream_t s) {
  constexpr int PX = SSOCT_DFFT_PX;
  hipLaunchKernelGGL((k_depth_fft<T2, DIR, EPI, PX>), dim3((P + PX - 1) / PX), dim3(16 * PX), 0, s, H, wt, out, P);
  return hipGetLastError();
}

template <int DIR, int EPI>
static hipError_t depth_fft_d(int T, int P, const float2* H, const float2* wt, void* out, hipStream_t s) {
  switch (T) {
    case 16: return depth_fft_t<1, DIR, EPI>(P, H, wt, out, s);
    case 32: return depth_fft_t<2, DIR, EPI>(P, H, wt, out, s);
    case 64: return depth_fft_t<4, DIR, EPI>(P, H, wt, out, s);
    case 128: return depth_fft_t<8, DIR, EPI>(P, H, wt, out, s);
    case 256: return depth_fft_t<16, DIR, EPI>(P, H, wt, out, s);
    default: return hipErrorInvalidValue;
  }
}

bool depth_fft_supported(int T) { return T == 16 || T == 32 || T == 64 || T == 128 || T == 256; }

hipError_t launch_depth_fft(int T, int P, int dir, int epi, const float2* H, const float2* wt, void* out,
                            hipStream_t s) {
  if (P <= 0) return hipSuccess;
  if (dir > 0) {
    if (epi == EPI_ABS) return depth_fft_d<+1, EPI_ABS>(T, P, H, wt, out, s);
    return depth_fft_d<+1, EPI_STORE>(T, P, H, wt, out, s);
  }
  if (epi != EPI_STORE) return hipErrorInvalidValue;
  return depth_fft_d<-1, EPI_STORE>(T, P, H, wt, out, s);
}

// wt[k] = exp(-2 pi i k / T), k = 0..T-1, from FP64 (sincospi) rounded to FP32
__global__ void k_depth_twiddles(int T, float2* __restrict__ wt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  double s, c;
  sincospi(-2.0 * (double)k / (double)T, &s, &c);
  wt[k] = make_float2((float)c, (float)s);
}

hipError_t launch_depth_twiddles(int T, float2* wt, hipStream_t s) {
  hipLaunchKernelGGL(k_depth_twiddles, dim3((T + 255) / 256), dim3(256), 0, s, T, wt);
  return hipGetLastError();
}

}  // namespace ssoct
