// Table kernels: every phase argument is formed in FP64 on the GPU and
// reduced modulo one cycle before the sine and cosine, then rounded to FP32.
//
//  * axis tables   : bilinear positions of Eq. 5 and the separable chirp of
//                    Eq. 6 per frame (with dispersion and Eq. 6 prefactor on
//                    the row table)
//  * misc tables   : FFT twiddles, Eq. 6 output phase, aberration screen
//  * depth tables  : the T x T real form of the Eq. 7 DFT matrix, packed in
//                    MFMA register order (FP32, and FP16/BF16 hi+lo pairs)
#include "fft_engine.hpp"
#include "internal.hpp"

namespace ssoct {

__device__ __forceinline__ double frac_cycles(double c) { return c - rint(c); }

// exp(2 pi i cyc) for an already reduced cycle count, in FP64
__device__ __forceinline__ float2 expi_cycles(double cyc, double amp) {
  double s, c;
  sincospi(2.0 * cyc, &s, &c);
  return make_float2((float)(amp * c), (float)(amp * s));
}

__global__ void k_axis_tables(const double* __restrict__ params, int T, int N,
                              AxisTab* __restrict__ rows, AxisTab* __restrict__ cols) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (i >= N || t >= T) return;
  const double* pf = params + (size_t)ParamLayout::PER_FRAME * t;
  const double s_t = pf[0], kappa = pf[1], rowcyc = pf[2], amp = pf[3];
  const int half = N >> 1;
  const int ip = (i + half) & (N - 1);     // original sample of FFT position i
  const int c = ip - half;                 // centred index
  // source position N/2 + c s_t, rounded exactly as written (no contraction)
  const double P = __dadd_rn(__dmul_rn((double)c, s_t), (double)half);
  double p0 = floor(P);
  int i0 = (int)p0;
  if (i0 < 0) i0 = 0;
  if (i0 > N - 1) i0 = N - 1;
  const float f = (float)(P - p0);
  const double cc = (double)c * (double)c;
  const double sign = (i & 1) ? -1.0 : 1.0;   // (-1)^i' == (-1)^i since N/2 is even
  double col_cyc = frac_cycles(-kappa * cc);
  double row_cyc = frac_cycles(-kappa * cc + rowcyc);
  AxisTab a;
  a.i0 = i0;
  a.f = f;
  a.fac = expi_cycles(col_cyc, sign);
  cols[(size_t)t * N + i] = a;
  a.fac = expi_cycles(row_cyc, sign * amp);
  rows[(size_t)t * N + i] = a;
}

__device__ __forceinline__ int mono_a(int k) {
  const int A[N_MONO] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
  return A[k];
}

__device__ __forceinline__ double mono(int k, double x, double y) {
  // (a, b) in the fixed monomial order
  const int A[N_MONO] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
  const int B[N_MONO] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4};
  double r = 1.0;
  for (int a = 0; a < A[k]; ++a) r *= x;
  for (int b = 0; b < B[k]; ++b) r *= y;
  return r;
}

// Per-thread twiddle table of the FFT engine (layout: TwPlan in fft_engine.hpp)
// for radix order PL.
template <int N, int PL>
__global__ void k_twiddles(float2* __restrict__ tw) {
  using P = TwPlan<N, PL>;
  using S = FFTShape<N>;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P::SIZE) return;
  long long num;
  if (idx < P::OFF_L) {
    // radix-16 pass p (counted from 0 over all of them) has stride
    // Ns = 16^p, or L 16^p when the small radix runs first
    const int p = idx / (P::G * P::E16) + (P::SMALL_FIRST ? 0 : 1), rem = idx % (P::G * P::E16);
    const int j = rem / P::E16, r = rem % P::E16 + 1;
    const int Ns = (P::SMALL_FIRST ? S::L : 1) << (4 * p);
    num = (long long)((j % Ns) * (N / (Ns * 16))) * r;
  } else {
    const int rem = idx - P::OFF_L, j = rem / P::EL, e = rem % P::EL;
    const int i = e / (S::L - 1), k = e % (S::L - 1) + 1;
    num = (long long)(j + P::G * i) * k;
  }
  double s, c;
  sincospi(2.0 * (double)(num % N) / (double)N, &s, &c);
  tw[idx] = make_float2((float)c, (float)s);
}

template <int N>
static hipError_t twiddles_n(float2* tw, int pl, hipStream_t s) {
  const int n = pl ? TwPlan<N, 1>::SIZE : TwPlan<N, 0>::SIZE;
  if (n == 0) return hipSuccess;
  if (pl)
    hipLaunchKernelGGL((k_twiddles<N, 1>), dim3((n + 255) / 256), dim3(256), 0, s, tw);
  else
    hipLaunchKernelGGL((k_twiddles<N, 0>), dim3((n + 255) / 256), dim3(256), 0, s, tw);
  return hipGetLastError();
}

hipError_t launch_twiddles(int N, float2* tw, hipStream_t s, int pl) {
  if (pl != 0 && pl != 1) return hipErrorInvalidValue;
  switch (N) {
    case 16: return twiddles_n<16>(tw, pl, s);
    case 32: return twiddles_n<32>(tw, pl, s);
    case 64: return twiddles_n<64>(tw, pl, s);
    case 128: return twiddles_n<128>(tw, pl, s);
    case 256: return twiddles_n<256>(tw, pl, s);
    case 512: return twiddles_n<512>(tw, pl, s);
    case 1024: return twiddles_n<1024>(tw, pl, s);
    case 2048: return twiddles_n<2048>(tw, pl, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
static size_t tw_size_n(int pl) {
  return pl ? TwPlan<N, 1>::SIZE : TwPlan<N, 0>::SIZE;
}

size_t twiddle_table_size(int N, int pl) {
  switch (N) {
    case 16: return tw_size_n<16>(pl);
    case 32: return tw_size_n<32>(pl);
    case 64: return tw_size_n<64>(pl);
    case 128: return tw_size_n<128>(pl);
    case 256: return tw_size_n<256>(pl);
    case 512: return tw_size_n<512>(pl);
    case 1024: return tw_size_n<1024>(pl);
    case 2048: return tw_size_n<2048>(pl);
    default: return 0;
  }
}

__global__ void k_misc_tables(const double* __restrict__ params, int T, int N, float2* __restrict__ outfac,
                              float* __restrict__ apoly) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;   // column (Eq. 6 output phase) or row (screen)
  if (n >= N) return;
  const double* g = params + ParamLayout::globals(T);
  if (outfac) {
    const double cu = (double)(n - (N >> 1));
    outfac[n] = expi_cycles(frac_cycles(-g[ParamLayout::G_KAPPA_OUT] * cu * cu), 1.0);
  }
  if (apoly && g[ParamLayout::G_HAS_ABERR] != 0.0) {
    // aberration phase on FFT row n as a quartic in x: sum_a p_a x^a with
    // p_a = sum_b poly(a, b) y^b, in cycles; p_0 reduced to one cycle (exact
    // in FP64); x, y = centred original index * sqrt 2 / N (rho = r / (N / sqrt 2))
    const int half = N >> 1;
    const double y = (double)(((n + half) & (N - 1)) - half) * (1.4142135623730950488 / (double)N);
    double pa[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < N_MONO; ++k) pa[mono_a(k)] += g[ParamLayout::G_POLY + k] * mono(k, 1.0, y);
    float* dst = apoly + (size_t)n * APOLY_STRIDE;
    for (int a = 0; a < 5; ++a) {
      const double c = pa[a] * 0.15915494309189533577;
      dst[a] = (float)(a == 0 ? frac_cycles(c) : c);
    }
    for (int a = 5; a < APOLY_STRIDE; ++a) dst[a] = 0.0f;
  }
}

// Aberration screen exp(i sum_k c_k Z_k) at every FFT position (FP64 phase,
// reduced in cycles), read by the adjoint row pass
__global__ void k_aberr_screen(const double* __restrict__ params, int T, int N, float2* __restrict__ screen) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;   // column (FFT position)
  const int m = blockIdx.y;                              // row (FFT position)
  if (n >= N || m >= N) return;
  const double* g = params + ParamLayout::globals(T);
  const int half = N >> 1;
  const double inv = 1.4142135623730950488 / (double)N;   // rho = r / (N / sqrt 2)
  const double x = (double)(((n + half) & (N - 1)) - half) * inv;
  const double y = (double)(((m + half) & (N - 1)) - half) * inv;
  double ph = 0.0;
  for (int k = 0; k < N_MONO; ++k) ph += g[ParamLayout::G_POLY + k] * mono(k, x, y);
  screen[(size_t)m * N + n] = expi_cycles(frac_cycles(ph * 0.15915494309189533577), 1.0);
}

hipError_t launch_aberr_screen(const double* params, int T, int N, float2* screen, hipStream_t s) {
  hipLaunchKernelGGL(k_aberr_screen, dim3((N + 255) / 256, N), dim3(256), 0, s, params, T, N, screen);
  return hipGetLastError();
}

DepthLayout depth_layout(int T, bool general) {
  DepthLayout L;
  L.T = T;
  const int t32 = (T + 31) / 32 * 32;
  L.KC = 32;                                   // chunk of 32, 64, 128 or 256 frames
  while (L.KC < t32 && L.KC < 256) L.KC *= 2;
  L.T_pad = (T + L.KC - 1) / L.KC * L.KC;
  L.rows = general ? 2 * T : ((T % 2 == 0) ? T : T + 1);
  L.M_pad = (L.rows + 31) / 32 * 32;
  L.nrb = L.M_pad / 32;
  L.waves = 1;                                 // 1, 2, 4 or 8 waves of 32 rows each
  while (L.waves < L.nrb && L.waves < 8) L.waves *= 2;
  L.slabs = (L.nrb + L.waves - 1) / L.waves;
  L.nrb = L.slabs * L.waves;                   // row blocks allocated (extra rows are zero)
  return L;
}

// Real form of the DFT matrix of Eq. 7.  Row pair k holds (Re W_q, Im W_q) for
// q = k >= 1 (W_q[t] = exp(-2 pi i q t / T)); pair 0 holds (W_0, W_{T/2}) for
// even T and (W_0, 0) for odd T.  Rows past the last pair and columns t >= T
// are zero.
__device__ __forceinline__ double depth_entry(int row, int t, int T) {
  const int k = row >> 1, which = row & 1;
  const int h = T / 2;
  if (t >= T || k >= T - h) return 0.0;
  if (k == 0) {
    if (which == 0) return 1.0;
    return (T % 2 == 0) ? ((t & 1) ? -1.0 : 1.0) : 0.0;
  }
  const long long idx = ((long long)k * t) % T;
  double s, c;
  sincospi(2.0 * (double)idx / (double)T, &s, &c);
  return which == 0 ? c : -s;
}

// General matrix W[q][t] = exp(-2 pi i q kappa_t / T) (sweeps not linear in
// k): row pair q holds (Re W_q, Im W_q) for every q = 0 .. T-1; the phase
// q kappa_t is reduced modulo T in FP64 before the sine and cosine.
__device__ __forceinline__ double depth_entry_general(int row, int t, int T, const double* __restrict__ kappa) {
  const int q = row >> 1, which = row & 1;
  if (t >= T || q >= T) return 0.0;
  const double x = (double)q * kappa[t];
  const double r = x - (double)T * floor(x / (double)T);
  double s, c;
  sincospi(2.0 * r / (double)T, &s, &c);
  return which == 0 ? c : -s;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One thread per (row block, k-step, lane).
//   f32 : value A[row = 32 rb + l % 32][t = 2 s + l / 32]       -> a_f32[(rb * T_pad/2 + s) * 64 + l]
//   f16 : 8 halves A[row][t = 16 s + 8 (l / 32) + i], hi and lo -> a_x[((rb * T_pad/16 + s) * 2 + hl) * 64 + l]
// kappa == nullptr: the DFT matrix in its paired real form; else the general matrix
__global__ void k_depth_tables(int T, int T_pad, int nrb, const double* __restrict__ kappa, float* __restrict__ a_f32,
                               uint4* __restrict__ a_f16, uint4* __restrict__ a_bf16) {
  const int l = threadIdx.x;          // lane 0..63
  const int s = blockIdx.x;           // k-step of 2 (f32)
  const int rb = blockIdx.y;
  if (rb >= nrb) return;
  const int row = 32 * rb + (l & 31);
  auto entry = [&](int t) { return kappa ? depth_entry_general(row, t, T, kappa) : depth_entry(row, t, T); };
  if (s < T_pad / 2) {
    const int t = 2 * s + (l >> 5);
    a_f32[((size_t)rb * (T_pad / 2) + s) * 64 + l] = (float)entry(t);
  }
  if (s < T_pad / 16) {
    uint32_t h16[2][4], b16[2][4];
    for (int i = 0; i < 8; i += 2) {
      uint16_t hh[2], hl[2], bh[2], bl[2];
      for (int u = 0; u < 2; ++u) {
        const int t = 16 * s + 8 * (l >> 5) + i + u;
        const float x = (float)entry(t);
        const _Float16 h = (_Float16)x;
        const _Float16 lo = (_Float16)(x - (float)h);
        hh[u] = __builtin_bit_cast(uint16_t, h);
        hl[u] = __builtin_bit_cast(uint16_t, lo);
        const uint16_t bhi = f32_to_bf16_rne(x);
        bh[u] = bhi;
        bl[u] = f32_to_bf16_rne(x - bf16_to_f32(bhi));
      }
      h16[0][i / 2] = (uint32_t)hh[0] | ((uint32_t)hh[1] << 16);
      h16[1][i / 2] = (uint32_t)hl[0] | ((uint32_t)hl[1] << 16);
      b16[0][i / 2] = (uint32_t)bh[0] | ((uint32_t)bh[1] << 16);
      b16[1][i / 2] = (uint32_t)bl[0] | ((uint32_t)bl[1] << 16);
    }
    for (int hl = 0; hl < 2; ++hl) {
      const size_t o = (((size_t)rb * (T_pad / 16) + s) * 2 + hl) * 64 + l;
      a_f16[o] = make_uint4(h16[hl][0], h16[hl][1], h16[hl][2], h16[hl][3]);
      a_bf16[o] = make_uint4(b16[hl][0], b16[hl][1], b16[hl][2], b16[hl][3]);
    }
  }
}

hipError_t launch_axis_tables(const double* params, int T, int N, AxisTab* rows, AxisTab* cols,
                              hipStream_t s) {
  dim3 block(256), grid((N + 255) / 256, T);
  hipLaunchKernelGGL(k_axis_tables, grid, block, 0, s, params, T, N, rows, cols);
  return hipGetLastError();
}

hipError_t launch_misc_tables(const double* params, int T, int N, float2* outfac, float* apoly, hipStream_t s) {
  if (!outfac && !apoly) return hipSuccess;
  hipLaunchKernelGGL(k_misc_tables, dim3((N + 255) / 256), dim3(256), 0, s, params, T, N, outfac, apoly);
  return hipGetLastError();
}

hipError_t launch_depth_tables(int T, const double* kappa, float* a_f32, uint4* a_f16, uint4* a_bf16,
                               hipStream_t s) {
  DepthLayout L = depth_layout(T, kappa != nullptr);
  dim3 block(64), grid(L.T_pad / 2, L.nrb);
  hipLaunchKernelGGL(k_depth_tables, grid, block, 0, s, T, L.T_pad, L.nrb, kappa, a_f32, a_f16, a_bf16);
  return hipGetLastError();
}

}  // namespace ssoct
