// Fresnel stage (steps 1-2 of the flowchart, Fig. 3): chromatic rescale by
// linear interpolation (Eq. 5) fused with the chirp of Eq. 6 into the row
// DFT, then the column DFT, which writes the hologram stack H[t][pixel] in the
// operand format of the depth transform.  Adjoint kernels (DIR = -1) serve
// the gradient of the sharpness loss.
//
// Index conventions: FFT position i carries original sample (i + N/2) mod N;
// the tables already hold (-1)^i' and the chirp, so both passes are plain
// positive-exponent DFTs and the output lands at natural (u, v).
//
// Both passes are persistent loops with register prefetch: a row group loads
// the source rows of its next output row while it transforms the current
// one, and a column workgroup loads its next column tile while it transforms
// the current one.  The per-frame column table of Eq. 5/6 is staged in LDS
// once per row workgroup.
#include "access.hpp"
#include "fft_engine.hpp"
#include "internal.hpp"
#include "split.hpp"

namespace ssoct {

// Tuning knobs (compile-time; the defaults are the tuned values)
#ifndef SSOCT_ROW_RPG
#define SSOCT_ROW_RPG 8          // rows per row group and workgroup iteration count
#endif
#ifndef SSOCT_ROW_WAVESYNC
#define SSOCT_ROW_WAVESYNC 1     // single-wave row groups exchange with wave-level ordering
#endif
#ifndef SSOCT_AS_XCD
#define SSOCT_AS_XCD 1           // transfer-function column pass: contiguous runs of tiles per XCD
#endif
#ifndef SSOCT_AS_GROUP
#define SSOCT_AS_GROUP 0         // > 0: phase evaluations scheduled in groups of this many
#endif
#ifndef SSOCT_AS_PF
#define SSOCT_AS_PF 1            // 1: transfer-function column pass loads its next tile while transforming
#endif
#ifndef SSOCT_AS_WPE
#define SSOCT_AS_WPE 0           // > 0: waves per SIMD the transfer-function column pass is compiled for
#endif
#if SSOCT_AS_WPE > 0
#define SSOCT_AS_OCC __attribute__((amdgpu_waves_per_eu(SSOCT_AS_WPE)))
#else
#define SSOCT_AS_OCC
#endif
#ifndef SSOCT_AS_THREADS
#define SSOCT_AS_THREADS 256     // transfer-function column pass: at most this many threads per workgroup
#endif
#ifndef SSOCT_COL_MIN
#define SSOCT_COL_MIN 16         // minimum adjacent columns per column workgroup (128 B row segments)
#endif
#ifndef SSOCT_COL_PREFETCH
#define SSOCT_COL_PREFETCH 0     // load the next column tile while transforming the current one (always on
                                 // where the twiddles are in LDS, see SSOCT_COL_TWL)
#endif
#ifndef SSOCT_COL_TWL
#define SSOCT_COL_TWL 1          // column passes (Fresnel and angular-spectrum): twiddles in LDS where the
                                 // exchange buffer leaves room, and the next tile prefetched into registers
#endif
#ifndef SSOCT_ROW_NT
#define SSOCT_ROW_NT 0           // row pass: non-temporal stores of the intermediate
#endif
#ifndef SSOCT_COL_NT
#define SSOCT_COL_NT 1           // column pass: non-temporal stores of H
#endif
#ifndef SSOCT_COL_NT_LD
#define SSOCT_COL_NT_LD 1        // column pass: non-temporal loads of the intermediate
#endif
#ifndef SSOCT_ADJ_NT
#define SSOCT_ADJ_NT 0           // adjoint column pass: non-temporal stores of the intermediate the
                                 // adjoint row pass reads back (a chunk sized to stay in MALL)
#endif
#ifndef SSOCT_ROWG_WPE
#define SSOCT_ROWG_WPE 2          // waves per SIMD the bin-pair row pass is held to (no aberration, no Eq. 6 factor)
#endif
#ifndef SSOCT_ROW_WAVES_PER_EU
#define SSOCT_ROW_WAVES_PER_EU 0  // > 0: ask the compiler to fit this many row-pass waves per SIMD
#endif
#if SSOCT_ROW_WAVES_PER_EU > 0
#define SSOCT_ROW_OCC __attribute__((amdgpu_waves_per_eu(SSOCT_ROW_WAVES_PER_EU)))
#else
#define SSOCT_ROW_OCC
#endif

// Row pass geometry: GR groups of G = N/16 threads, each group owns RPG
// consecutive rows; a workgroup covers GR * RPG rows of one frame.
template <int N>
struct RowCfg {
  static constexpr int G = FFTShape<N>::G;
  static constexpr int GR = (256 / G) < N ? (256 / G) : N;
  static constexpr int RPG = (N / GR) < SSOCT_ROW_RPG ? (N / GR) : SSOCT_ROW_RPG;
  static constexpr int ROWS = GR * RPG;                  // rows per workgroup
  static constexpr int THREADS = GR * G;
  static constexpr bool WAVE = G <= 64 && SSOCT_ROW_WAVESYNC;  // a group lives inside one wavefront
};
// Column pass geometry: C adjacent columns (>= SSOCT_COL_MIN, so row segments
// are >= 64 B), at most 1024 threads
template <int N>
struct ColCfg {
  static constexpr int G = FFTShape<N>::G;
  static constexpr int C0 = 4096 / N;
  static constexpr int C1 = C0 < SSOCT_COL_MIN ? SSOCT_COL_MIN : (C0 > N ? N : C0);
  static constexpr int C = C1 * G > 1024 ? 1024 / G : C1;
  static constexpr int THREADS = C * G;
};
// Narrower tiles (C/2 and C/4 adjacent columns, for N >= 512) are tuning
// alternatives of the Fresnel column passes: fewer threads and less LDS per
// workgroup, so more workgroups per CU, at the price of shorter row segments.
template <int N>
struct ColTiles {
  static constexpr int C = ColCfg<N>::C;
  static constexpr bool ALT = N >= 512 && C >= 4;
  static constexpr int C2 = ALT ? C / 2 : C;
  static constexpr int C4 = ALT ? C / 4 : C;
};
// LDS of the column pass: the exchange buffer of CT columns, plus the twiddle
// table of radix order PL where the two fit in one CU's 160 KB (every N <= 1024)
template <int N, int CT, int PL = 0>
struct ColLdsT {
  static constexpr int XB = FFTShape<N>::LDS * CT;
  static constexpr int TWN = TwPlan<N, PL>::SIZE > 0 ? TwPlan<N, PL>::SIZE : 1;
  static constexpr bool TWL = SSOCT_COL_TWL && (XB + TWN) * 8 <= 163840;
  static constexpr bool PF = TWL || SSOCT_COL_PREFETCH;    // next tile prefetched into registers
  static constexpr int BYTES = (XB + (TWL ? TWN : 1)) * 8;
};
template <int N>
using ColLds = ColLdsT<N, ColCfg<N>::C>;

// Source rows y0 and y0 + 1 of Eq. 5 for one output row: thread j of a group
// holds columns [s N/4 + 4 j, s N/4 + 4 j + 4) for s = 0..3, so every load
// instruction of a group covers a contiguous N/2-byte span and the LDS stores
// of the y-lerped row are conflict free.
struct RowSrc {
  uint2 a[4], b[4];
};

template <int N>
__device__ __forceinline__ RowSrc load_rows(const uint16_t* __restrict__ I, int y0, int j) {
  const int y1 = y0 + 1 < N ? y0 + 1 : N - 1;
  const uint16_t* r0 = I + (size_t)y0 * N + 4 * j;
  const uint16_t* r1 = I + (size_t)y1 * N + 4 * j;
  RowSrc s;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    s.a[q] = *reinterpret_cast<const uint2*>(r0 + q * (N / 4));
    s.b[q] = *reinterpret_cast<const uint2*>(r1 + q * (N / 4));
  }
  return s;
}

// y-lerp of the two source rows into rbuf (same column split as load_rows);
// the last thread also zeroes rbuf[N], the right tap of the last sample, which
// only occurs with weight 0 (s_t <= 1 keeps every position inside [0, N-1])
template <int N>
__device__ __forceinline__ void lerp_rows(const RowSrc& s, float fy, float* rbuf, int j) {
  if (j == N / 16 - 1) rbuf[N] = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t wa[2] = {s.a[q].x, s.a[q].y};
    const uint32_t wb[2] = {s.b[q].x, s.b[q].y};
    float out[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float a0 = (float)(wa[h] & 0xffffu), a1 = (float)(wa[h] >> 16);
      const float b0 = (float)(wb[h] & 0xffffu), b1 = (float)(wb[h] >> 16);
      out[2 * h] = a0 + fy * (b0 - a0);
      out[2 * h + 1] = a1 + fy * (b1 - a1);
    }
    *reinterpret_cast<float4*>(rbuf + q * (N / 4) + 4 * j) = make_float4(out[0], out[1], out[2], out[3]);
  }
}

// Aberration phase of one row as a quartic in x (cycles), from the per-row table
struct ARow {
  float p0, p1, p2, p3, p4;
};

template <bool ABERR>
__device__ __forceinline__ ARow load_arow(const float* __restrict__ apoly, int m) {
  ARow a{0.f, 0.f, 0.f, 0.f, 0.f};
  if constexpr (ABERR) {
    const float4 lo = *reinterpret_cast<const float4*>(apoly + (size_t)m * APOLY_STRIDE);
    a = ARow{lo.x, lo.y, lo.z, lo.w, apoly[(size_t)m * APOLY_STRIDE + 4]};
  }
  return a;
}

// exp(2 pi i phase) of the aberration at FFT column n: Horner in FP32, the
// phase reduced to one cycle, then the hardware sine and cosine, which take
// their argument in cycles (measured on gfx950 over [-1/2, 1/2]: at most
// 1.3e-7 from the FP64 values)
template <int N>
__device__ __forceinline__ float2 aberr_factor(const ARow& a, int n) {
  constexpr float inv = 1.41421356237309505f / (float)N;   // rho = r / (N / sqrt 2)
  const float x = (float)(((n + N / 2) & (N - 1)) - N / 2) * inv;
  const float ph = fmaf(fmaf(fmaf(fmaf(a.p4, x, a.p3), x, a.p2), x, a.p1), x, a.p0);
  const float f = ph - rintf(ph);
  return make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
}

// Row input z[m][n] of the DFT at FFT position n (x-lerp of the y-lerped row,
// times the separable chirp, dispersion, sign and optional aberration).
template <int N, bool ABERR>
__device__ __forceinline__ float2 row_input(const float* rbuf, const AxisTab& ct, float2 rowfac, const ARow& ar,
                                            int n) {
  const int x0 = ct.i0;
  const float r0 = rbuf[x0], r1 = rbuf[x0 + 1];   // rbuf[N] is a zero pad
  const float J = r0 + ct.f * (r1 - r0);
  float2 fac = cmul(ct.fac, rowfac);
  if constexpr (ABERR) fac = cmul(fac, aberr_factor<N>(ar, n));
  return make_float2(J * fac.x, J * fac.y);
}

template <int N>
struct RowLds {
  static constexpr int XS = (FFTShape<N>::LDS + 1) & ~1;  // row stride kept a multiple of 16 bytes
  AxisTab ctab[N];
  float2 xbuf[RowCfg<N>::GR][XS];   // exchange buffer; the y-lerped row (float4 stores) aliases its start
};

// stage the frame's column table in LDS (all threads)
template <int N>
__device__ __forceinline__ void stage_ctab(AxisTab* ctab, const AxisTab* __restrict__ src) {
  for (int i = threadIdx.x; i < N; i += RowCfg<N>::THREADS) ctab[i] = src[i];
}

// ------------------------------------------------------------------ forward row pass
template <int N, bool ABERR, bool EQ6>
__global__ __launch_bounds__(RowCfg<N>::THREADS) SSOCT_ROW_OCC void k_row_pass(
    const uint16_t* __restrict__ frames, int t0, const AxisTab* __restrict__ rows,
    const AxisTab* __restrict__ cols, const float2* __restrict__ tw, const float* __restrict__ apoly,
    const float2* __restrict__ outfac, float2* __restrict__ inter) {
  using S = FFTShape<N>;
  using R = RowCfg<N>;
  constexpr int G = S::G;
  __shared__ RowLds<N> lds;
  __shared__ AxisTab rtab_s[R::ROWS];   // row table entries of this workgroup's rows
  // output factor of Eq. 6, read between the row's stores; kept in LDS up to
  // N = 1024 (at N = 2048 it would leave room for one workgroup per CU)
  constexpr bool OFS = EQ6 && N <= 1024;
  __shared__ float2 ofac_s[OFS ? N : 1];
  const int g = threadIdx.x / G, j = threadIdx.x % G;
  const int f = blockIdx.y;
  const int t = t0 + f;
  const int m0 = blockIdx.x * R::ROWS + g * R::RPG;
  const uint16_t* I = frames + (size_t)t * N * N;
  const AxisTab* rtab = rows + (size_t)t * N;
  float* rbuf = reinterpret_cast<float*>(lds.xbuf[g]);
  // The first row's source loads, the twiddles and the table staging are in
  // flight together.  The twiddles stay in registers and the staging waits
  // complete their loads, so no twiddle load is outstanding inside the row
  // loop.  Inside the loop the next row's table entry comes from LDS: a
  // global load there would have to wait for the previous row's stores,
  // which the vector memory counter counts together with the loads.
  AxisTab rt = rtab[m0];
  RowSrc src = load_rows<N>(I, rt.i0, j);
  ARow an = load_arow<ABERR>(apoly, m0);
  const TwRegs<N> twr = load_tw_regs<N>(tw, j);
  stage_ctab<N>(lds.ctab, cols + (size_t)t * N);
  for (int i = threadIdx.x; i < R::ROWS; i += R::THREADS) rtab_s[i] = rtab[blockIdx.x * R::ROWS + i];
  if constexpr (OFS) {
    for (int i = threadIdx.x; i < N; i += R::THREADS) ofac_s[i] = outfac[i];
  }
  // Everything above has landed here (the first lerp needs it at once), so
  // the loop is entered with no load outstanding and its header, shared with
  // the back edge, does not wait for the stores of the previous row.
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unchanged
  __syncthreads();  // column and row tables visible
#pragma unroll 1
  for (int i = 0; i < R::RPG; ++i) {
    const int m = m0 + i;
    const RowSrc cur = src;
    const AxisTab rc = rt;
    const ARow ar = an;
    if (i + 1 < R::RPG) {  // prefetch the next row of this group
      rt = rtab_s[g * R::RPG + i + 1];
      src = load_rows<N>(I, rt.i0, j);
      an = load_arow<ABERR>(apoly, m + 1);
    }
    exchange_sync<R::WAVE>();  // previous row's FFT reads are done
    lerp_rows<N>(cur, rc.f, rbuf, j);
    exchange_sync<R::WAVE>();
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int n = j + k * G;
      v[k] = row_input<N, ABERR>(rbuf, lds.ctab[n], rc.fac, ar, n);
    }
    fft_group_tw<N, +1, 1, R::WAVE>(v, j, lds.xbuf[g], twr);
    float2* dst = inter + ((size_t)f * N + m) * N;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int vv = j + out_offset<N>(e);
      float2 val = v[e];
      if constexpr (EQ6) val = cmul(val, OFS ? ofac_s[vv] : outfac[vv]);
      st_once<SSOCT_ROW_NT>(dst + vv, val);
    }
  }
}

// ------------------------------------------------------------------ bin-pair row pass (depth-first order)
// Row m of G_q (q = qa + f, FFT positions, from the depth DFT of the rescaled
// frames) times the frame-independent chirp, sign and optional aberration:
// DFT of fac G_q into chunk frame f, and for 0 < q < T/2 DFT of fac conj(G_q)
// into chunk frame Fh + f.  The column pass turns these into V[q] and
// V[T - q] (Eq. 6 is linear and its chirp does not depend on the frame when
// lambda_1 is used for every frame and no per-frame phase is applied).
// Without the aberration factor the kernel fits two waves per SIMD; the
// compiler is held to that (with the Eq. 6 output factor it would otherwise
// take a few registers more and keep one).
template <int N, bool ABERR, bool EQ6, int RPG>
__global__ __launch_bounds__(RowCfg<N>::THREADS)
__attribute__((amdgpu_waves_per_eu(ABERR ? 1 : (EQ6 ? 2 : SSOCT_ROWG_WPE)))) void k_row_pass_g(
    const float2* __restrict__ Gq, int qa, int T, const AxisTab* __restrict__ rows0,
    const AxisTab* __restrict__ cols0, const float2* __restrict__ tw, const float* __restrict__ apoly,
    const float2* __restrict__ outfac, float2* __restrict__ inter, int Fh) {
  using S = FFTShape<N>;
  using R = RowCfg<N>;
  constexpr int G = S::G;
  // column factors only (contiguous 8-byte entries: a 16-byte table entry read for its factor
  // alone would put two lanes on one LDS bank)
  __shared__ float2 cfac[N];
  __shared__ float2 xbuf[R::GR][RowLds<N>::XS];
  constexpr int ROWS = R::GR * RPG;    // rows per workgroup
  __shared__ float2 rfac_s[ROWS];      // row factors of this workgroup's rows
  constexpr bool OFS = EQ6 && N <= 1024;  // output factor of Eq. 6 in LDS, as in k_row_pass
  __shared__ float2 ofac_s[OFS ? N : 1];
  const int g = threadIdx.x / G, j = threadIdx.x % G;
  const int f = blockIdx.y;
  const int q = qa + f;
  const bool both = q >= 1 && 2 * q < T;
  const int m0 = blockIdx.x * ROWS + g * RPG;
  float2 nxt[16];
  {
    const float2* src = Gq + ((size_t)q * N + m0) * N;
#pragma unroll
    for (int k = 0; k < 16; ++k) nxt[k] = ld_once<true>(src + j + k * G);
  }
  // as in k_row_pass: twiddles in registers, per-row table entries in LDS,
  // and no load outstanding when the loop is entered
  const TwRegs<N> twr = load_tw_regs<N>(tw, j);
  for (int i = threadIdx.x; i < N; i += R::THREADS) cfac[i] = cols0[i].fac;
  for (int i = threadIdx.x; i < ROWS; i += R::THREADS) rfac_s[i] = rows0[blockIdx.x * ROWS + i].fac;
  if constexpr (OFS) {
    for (int i = threadIdx.x; i < N; i += R::THREADS) ofac_s[i] = outfac[i];
  }
  ARow an = load_arow<ABERR>(apoly, m0);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unchanged
  __syncthreads();  // column table and row factors visible
#pragma unroll 1
  for (int i = 0; i < RPG; ++i) {
    const int m = m0 + i;
    float2 gv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) gv[k] = nxt[k];
    const ARow ar = an;
    if (i + 1 < RPG) {  // prefetch the next row of this group
      const float2* src = Gq + ((size_t)q * N + m + 1) * N;
#pragma unroll
      for (int k = 0; k < 16; ++k) nxt[k] = ld_once<true>(src + j + k * G);
      an = load_arow<ABERR>(apoly, m + 1);
    }
    const float2 rowfac = rfac_s[g * RPG + i];
#pragma unroll 1
    for (int h = 0; h < (both ? 2 : 1); ++h) {
      float2 v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int n = j + k * G;
        float2 fac = cmul(cfac[n], rowfac);
        if constexpr (ABERR) fac = cmul(fac, aberr_factor<N>(ar, n));
        v[k] = cmul(fac, h == 0 ? gv[k] : cconj(gv[k]));
      }
      exchange_sync<R::WAVE>();  // the previous transform's exchange reads are done
      fft_group_tw<N, +1, 1, R::WAVE>(v, j, xbuf[g], twr);
      float2* dst = inter + ((size_t)(h == 0 ? f : Fh + f) * N + m) * N;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int vv = j + out_offset<N>(e);
        float2 val = v[e];
        if constexpr (EQ6) val = cmul(val, OFS ? ofac_s[vv] : outfac[vv]);
        st_once<SSOCT_ROW_NT>(dst + vv, val);
      }
    }
  }
}

// ------------------------------------------------------------------ H storage formats
template <int FMT, int NT = SSOCT_COL_NT>
__device__ __forceinline__ void store_h(void* __restrict__ H, long long idx, float2 val, float scale) {
  if constexpr (FMT == HF_F32) {
    st_once<NT>(reinterpret_cast<float2*>(H) + idx, val);
  } else {
    uint2 w;
    w.x = split_pack<FMT>(val.x * scale);
    w.y = split_pack<FMT>(val.y * scale);
    st_once<NT>(reinterpret_cast<uint2*>(H) + idx, w);
  }
}

// ------------------------------------------------------------------ angular-spectrum passes
// Propagation of the sensor field by the angular spectrum (no rescale, no
// chirp, plain uncentred DFTs; pixel and frequency indices both natural):
//   pass 1 (k_as_row_fwd): DFT^- of every u16 frame row into the chunk buffer;
//   pass 2 (k_as_col): per column tile, DFT^- down the columns, times the
//     transfer function, DFT^+ back, in place;
//   pass 3 (k_as_row_inv): DFT^+ of every row into H (depth operand format).
// The per-frame block `asp` holds 1/lambda_t^2, a phase offset in cycles
// (dispersion) and an amplitude (gate / N^2) for each frame.
template <int N>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_as_row_fwd(const uint16_t* __restrict__ frames, int t0,
                                                                  const float2* __restrict__ tw,
                                                                  float2* __restrict__ inter) {
  using S = FFTShape<N>;
  using R = RowCfg<N>;
  constexpr int G = S::G;
  __shared__ float2 xbuf[R::GR][RowLds<N>::XS];
  const int g = threadIdx.x / G, j = threadIdx.x % G;
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * R::ROWS + g * R::RPG;
  const uint16_t* I = frames + (size_t)(t0 + f) * N * N;
  // As in k_row_pass: the next row loads while the current one is
  // transformed, the twiddles stay in registers, and nothing is outstanding
  // when the loop starts, so the loop waits for its prefetched row only
  // (loaded before the previous row's stores, which stay in flight).
  // held as 32-bit values: packing two samples per register would wait for
  // the loads (and with them the previous row's stores) right after issue
  uint32_t nx[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) nx[k] = I[(size_t)m0 * N + j + k * G];
  const TwRegs<N> twr = load_tw_regs<N>(tw, j);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unchanged
#pragma unroll 1
  for (int i = 0; i < R::RPG; ++i) {
    const int m = m0 + i;
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = make_float2((float)nx[k], 0.f);
    if (i + 1 < R::RPG) {
#pragma unroll
      for (int k = 0; k < 16; ++k) nx[k] = I[(size_t)(m + 1) * N + j + k * G];
    }
    exchange_sync<R::WAVE>();
    fft_group_tw<N, -1, 1, R::WAVE>(v, j, xbuf[g], twr);
    float2* dst = inter + ((size_t)f * N + m) * N;
#pragma unroll
    for (int e = 0; e < 16; ++e) dst[j + out_offset<N>(e)] = v[e];
  }
}

// The transfer-function column pass keeps 16 FP64 phase evaluations in flight
// per thread, so its tiles are narrower than the column pass's: at most 256
// threads (4 columns at N = 1024), which leaves room for two workgroups per
// CU (LDS: exchange buffer plus twiddle table, 48 KB at N = 1024) at up to 256
// VGPRs per thread; 8-column tiles hold one workgroup per CU.
template <int N>
struct AsColCfg {
  static constexpr int C = ColCfg<N>::C * FFTShape<N>::G > SSOCT_AS_THREADS ? SSOCT_AS_THREADS / FFTShape<N>::G
                                                                            : ColCfg<N>::C;
  static constexpr int THREADS = C * FFTShape<N>::G;
};

// Register of DFT^+ input element j + G m that the forward transform's output
// register e holds (element j + out_offset(e)): m = e / L + (e % L) (16 / L)
template <int N>
__device__ __forceinline__ constexpr int as_in_slot(int e) {
  constexpr int L = FFTShape<N>::L > 1 ? FFTShape<N>::L : 1;
  return e / L + (e % L) * (16 / L);
}
static_assert(as_in_slot<1024>(5) * FFTShape<1024>::G == out_offset<1024>(5), "register permutation of N = 1024");
static_assert(as_in_slot<2048>(7) * FFTShape<2048>::G == out_offset<2048>(7), "register permutation of N = 2048");
static_assert(as_in_slot<256>(9) * FFTShape<256>::G == out_offset<256>(9), "register permutation of N = 256");

// Square root of a positive normal FP64 value (no zero, subnormal, infinity or
// NaN, so none of the range scaling of the library root): the hardware
// reciprocal-root estimate, one Goldschmidt step and two Newton corrections
// of the root, which end within an ulp.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

template <int N>
__global__ __launch_bounds__(AsColCfg<N>::THREADS) SSOCT_AS_OCC void k_as_col(float2* __restrict__ buf, int t0,
                                                                const float2* __restrict__ tw,
                                                                const double* __restrict__ asp, double inv_nd,
                                                                double z, int ntiles) {
  using S = FFTShape<N>;
  constexpr int G = S::G;
  constexpr int C = AsColCfg<N>::C;
  constexpr int NCB = N / C;
  // As in k_col_pass, the twiddle table goes to LDS beside the exchange
  // buffer where it fits.  With SSOCT_AS_PF the freed registers hold the
  // next tile, loaded while the current one is transformed (tiles are
  // disjoint and each belongs to one workgroup, so the prefetch never reads
  // a column that is being written in place).  At N = 1024 the kernel then
  // holds 138 VGPRs, and three workgroups share a CU (the LDS allows three)
  // as they do without the prefetch at 165 VGPRs.
  constexpr int TWN = TwPlan<N>::SIZE > 0 ? TwPlan<N>::SIZE : 1;
  constexpr bool TWL = SSOCT_COL_TWL && (S::LDS * C + TWN) * 8 <= 163840;
  constexpr bool PF = TWL && SSOCT_AS_PF;
  __shared__ float2 xbuf[S::LDS * C];
  __shared__ float2 twl[TWL ? TWN : 1];
  const int c = threadIdx.x % C, j = threadIdx.x / C;
  float2 pf[16];
  auto issue = [&](int tl) {
    const float2* cs = buf + (size_t)(tl / NCB) * N * N + (tl % NCB) * C + c;
#pragma unroll
    for (int k = 0; k < 16; ++k) pf[k] = cs[(size_t)(j + k * G) * N];
  };
  // tiles tile0, tile0 + tstride, ... below tend: with SSOCT_AS_XCD each XCD
  // (workgroups are dispatched round-robin over the 8) walks a contiguous run,
  // so the workgroups of one L2 hold neighbouring column blocks
  int tile0 = blockIdx.x, tstride = gridDim.x, tend = ntiles;
  if (SSOCT_AS_XCD && gridDim.x % 8 == 0) {
    const int per = (ntiles + 7) / 8, x = blockIdx.x % 8;
    tile0 = x * per + (int)blockIdx.x / 8;
    tstride = gridDim.x / 8;
    tend = min(ntiles, (x + 1) * per);
  }
  if constexpr (TWL) {
    if (PF && tile0 < tend) issue(tile0);
    for (int i = threadIdx.x; i < TwPlan<N>::SIZE; i += AsColCfg<N>::THREADS) twl[i] = tw[i];
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the loop is entered with no load outstanding
    __syncthreads();  // twiddles visible
  }
  const TwMem<N> twm{TWL ? static_cast<const float2*>(twl) : tw, j};
#pragma unroll 1
  for (int tile = tile0; tile < tend; tile += tstride) {
    const int f = tile / NCB, kx = (tile % NCB) * C + c;
    float2* col = buf + (size_t)f * N * N + kx;
    float2 v[16];
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = pf[k];
      if (tile + tstride < tend) issue(tile + tstride);
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = col[(size_t)(j + k * G) * N];
    }
    fft_group_tw<N, -1, C, false>(v, j, xbuf + c, twm);
    const double* pf = asp + 3 * (size_t)(t0 + f);
    const double inv_l2 = pf[0], cyc0 = pf[1], amp = pf[2];
    // squared spatial frequency (kx'^2 + ky'^2) / (N d)^2 from the exact integer kx'^2 + ky'^2
    // (signed indices, at most N^2 / 2)
    const int sx = kx < N / 2 ? kx : kx - N;
    const int kx2 = sx * sx;
    const double inv_nd2 = inv_nd * inv_nd;
    const float famp = (float)amp;
    // propagating: exp(2 pi i (cyc0 - z sqrt(rad))) amp; evanescent (rad <= 0): 0
    // (exp(-i k z) for +z: the paper's fields carry exp(+i omega t), as the prefactor of Eq. 6
    // does).  The phase (up to ~1e5 cycles) is reduced to a fraction in FP64; the hardware sine
    // and cosine take the fraction in cycles (within 1.3e-7 of FP64 over one cycle on gfx950).
    // Evaluated without branches (an evanescent element takes a dummy root and is zeroed), so the
    // sixteen FP64 chains of a thread interleave.
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int ky = j + out_offset<N>(e);
      const int sy = ky < N / 2 ? ky : ky - N;
      const double rad = inv_l2 - (double)(kx2 + sy * sy) * inv_nd2;
      const bool prop = rad > 0.0;
      double cyc = cyc0 - z * sqrt_pos(prop ? rad : 1.0);
      cyc -= rint(cyc);
      const float fr = (float)cyc;
      const float2 h = make_float2(prop ? __builtin_amdgcn_cosf(fr) * famp : 0.f,
                                   prop ? __builtin_amdgcn_sinf(fr) * famp : 0.f);
      v[e] = cmul(v[e], h);
#if SSOCT_AS_GROUP > 0
      if ((e + 1) % SSOCT_AS_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
#endif
    }
    // back to the input order of DFT^+, which wants element j + k G in
    // register k: the forward output register e holds element
    // j + out_offset(e) = j + G m(e), m(e) = e / L + (e % L) (16 / L), so
    // the same thread already holds every element it needs and a register
    // permutation replaces an exchange (the transform's own first exchange
    // waits for the forward transform's last reads of xbuf)
    float2 w[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) w[as_in_slot<N>(e)] = v[e];
    fft_group_tw<N, +1, C, false>(w, j, xbuf + c, twm);
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = w[e];
#pragma unroll
    for (int e = 0; e < 16; ++e) col[(size_t)(j + out_offset<N>(e)) * N] = v[e];
    __syncthreads();   // this tile's exchange reads are done before the next tile writes LDS
  }
}

template <int N, int FMT>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_as_row_inv(const float2* __restrict__ inter, int t0,
                                                                  const float2* __restrict__ tw,
                                                                  void* __restrict__ H, float scale) {
  using S = FFTShape<N>;
  using R = RowCfg<N>;
  constexpr int G = S::G;
  __shared__ float2 xbuf[R::GR][RowLds<N>::XS];
  const int g = threadIdx.x / G, j = threadIdx.x % G;
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * R::ROWS + g * R::RPG;
  // next row prefetched, twiddles in registers, empty entry state (k_as_row_fwd)
  float2 nx[16];
  {
    const float2* src = inter + ((size_t)f * N + m0) * N;
#pragma unroll
    for (int k = 0; k < 16; ++k) nx[k] = src[j + k * G];
  }
  const TwRegs<N> twr = load_tw_regs<N>(tw, j);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unchanged
#pragma unroll 1
  for (int i = 0; i < R::RPG; ++i) {
    const int m = m0 + i;
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = nx[k];
    if (i + 1 < R::RPG) {
      const float2* src = inter + ((size_t)f * N + m + 1) * N;
#pragma unroll
      for (int k = 0; k < 16; ++k) nx[k] = src[j + k * G];
    }
    exchange_sync<R::WAVE>();
    fft_group_tw<N, +1, 1, R::WAVE>(v, j, xbuf[g], twr);
    const long long base = ((long long)(t0 + f) * N + m) * N;
#pragma unroll
    for (int e = 0; e < 16; ++e) store_h<FMT>(H, base + j + out_offset<N>(e), v[e], scale);
  }
}

// ------------------------------------------------------------------ column pass (both directions)
// Tiles are (frame f, block of C columns) over the F frames of the launch,
// walked persistently.  Frames f < nA read src + f N^2 and write frame
// f fstride of dst; frames f >= nA read src2 + (f - nA) N^2 and write frame
// (f - nA) fstride2 of dst2 (two runs of frames in one launch).
// DIR = +1 writes H in format FMT (and the Eq. 6 output phase when EQ6);
// DIR = -1 writes complex64.  PL is the radix order of the transforms.
template <int N, int DIR, int FMT, bool EQ6, int CT = ColCfg<N>::C, int PL = 0>
__global__ __launch_bounds__(CT * FFTShape<N>::G) void k_col_pass(const float2* __restrict__ src,
                                                                  const float2* __restrict__ tw,
                                                                  const float2* __restrict__ outfac,
                                                                  void* __restrict__ dst, float scale, int ntiles,
                                                                  int fstride, const float2* __restrict__ src2,
                                                                  void* __restrict__ dst2, int nA, int fstride2) {
  using S = FFTShape<N>;
  constexpr int G = S::G;
  constexpr int C = CT;
  constexpr int NCB = N / C;  // column blocks per frame
  // The twiddle table goes to LDS where the exchange buffer leaves room for
  // it (N <= 1024).  That frees the registers the twiddles would hold for a
  // prefetch of the next tile, which then loads while the current one is
  // transformed: one 1024-thread workgroup fills a CU, so without it the
  // CU's memory and ALUs take turns.
  using LT = ColLdsT<N, CT, PL>;
  constexpr bool TWL = LT::TWL;
  constexpr bool PF = LT::PF;
  __shared__ float2 xbuf[LT::XB];
  __shared__ float2 twl[TWL ? LT::TWN : 1];
  const int c = threadIdx.x % C, j = threadIdx.x / C;
  float2 pf[16];
  auto issue = [&](int tile) {
    const int f = tile / NCB, col = (tile % NCB) * C + c;
    const float2* s = (f < nA ? src + (size_t)f * N * N : src2 + (size_t)(f - nA) * N * N) + col;
#pragma unroll
    for (int k = 0; k < 16; ++k) pf[k] = ld_once<SSOCT_COL_NT_LD>(s + (size_t)(j + k * G) * N);
  };
  int tile = blockIdx.x;
  if (PF && tile < ntiles) issue(tile);
  if constexpr (TWL) {
    for (int i = threadIdx.x; i < TwPlan<N, PL>::SIZE; i += (CT * G)) twl[i] = tw[i];
    // the first tile has landed; the loop is entered with no load
    // outstanding, so waiting for a prefetched tile inside it leaves the
    // previous tile's stores in flight
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unchanged
    __syncthreads();  // twiddles visible
  }
#pragma unroll 1
  for (; tile < ntiles; tile += gridDim.x) {
    float2 v[16];
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = pf[k];
      if (tile + (int)gridDim.x < ntiles) issue(tile + gridDim.x);
    } else {
      issue(tile);
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = pf[k];
    }
    const int f = tile / NCB, col = (tile % NCB) * C + c;
    if constexpr (TWL) fft_group_tw<N, DIR, C, false>(v, j, xbuf + c, TwMem<N, PL>{twl, j});
    else fft_group_tw<N, DIR, C, false>(v, j, xbuf + c, TwMem<N, PL>{tw, j});
    void* d = f < nA ? dst : dst2;
    const long long fo = (f < nA ? (long long)f * fstride : (long long)(f - nA) * fstride2) * N * N;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int u = j + out_offset<N, PL>(e);
      float2 val = v[e];
      if constexpr (EQ6) val = cmul(val, outfac[u]);
      store_h<FMT, (DIR > 0 ? SSOCT_COL_NT : SSOCT_ADJ_NT)>(d, fo + (long long)u * N + col, val, scale);
    }
  }
}

// ------------------------------------------------------------------ adjoint row pass + moments
// g[m][n] = DFT^-_v inter[f][m][v]; u = Im(conj(g) z) with z recomputed as in
// the forward row pass; per-(frame, workgroup) FP64 moments sum u x^a y^b
// (a + b <= 4) at the original sample (x, y) = (c_n', c_m') sqrt(2) / N.
template <int N, bool ABERR>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void k_row_pass_adj(
    const uint16_t* __restrict__ frames, int t0, const AxisTab* __restrict__ rows,
    const AxisTab* __restrict__ cols, const float2* __restrict__ tw, const float2* __restrict__ screen,
    const float2* __restrict__ inter, double* __restrict__ partials) {
  using S = FFTShape<N>;
  using R = RowCfg<N>;
  constexpr int G = S::G;
  constexpr int NW = (R::THREADS + 63) / 64;
  constexpr int WIDTH = R::THREADS < 64 ? R::THREADS : 64;  // lanes that exist in a wave
  __shared__ RowLds<N> lds;
  __shared__ double red[NW][N_MONO];
  const int g = threadIdx.x / G, j = threadIdx.x % G;
  const int f = blockIdx.y;
  const int t = t0 + f;
  const int m0 = blockIdx.x * R::ROWS + g * R::RPG;
  const uint16_t* I = frames + (size_t)t * N * N;
  const AxisTab* rtab = rows + (size_t)t * N;
  float* rbuf = reinterpret_cast<float*>(lds.xbuf[g]);
  stage_ctab<N>(lds.ctab, cols + (size_t)t * N);
  const double inv = 1.4142135623730950488 / (double)N;
  const int half = N >> 1;
  double acc[N_MONO];
#pragma unroll
  for (int k = 0; k < N_MONO; ++k) acc[k] = 0.0;
  __syncthreads();
#pragma unroll 1
  for (int i = 0; i < R::RPG; ++i) {
    const int m = m0 + i;
    const AxisTab rc = rtab[m];
    const RowSrc cur = load_rows<N>(I, rc.i0, j);
    const float2* srow_ab = ABERR ? screen + (size_t)m * N : nullptr;
    const float2* srow = inter + ((size_t)f * N + m) * N;
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = srow[j + k * G];
    fft_group<N, -1, 1, R::WAVE>(v, j, lds.xbuf[g], tw);
    exchange_sync<R::WAVE>();   // FFT reads of xbuf done before rbuf (aliased) is written
    lerp_rows<N>(cur, rc.f, rbuf, j);
    exchange_sync<R::WAVE>();
    const double y = (double)(m < half ? m : m - N) * inv;
    const double y2 = y * y;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int n = j + out_offset<N>(e);
      float2 z = row_input<N, false>(rbuf, lds.ctab[n], rc.fac, ARow{}, n);
      if constexpr (ABERR) z = cmul(z, srow_ab[n]);
      const float2 gg = v[e];
      const double u = (double)gg.x * (double)z.y - (double)gg.y * (double)z.x;  // Im(conj(g) z)
      const double x = (double)(n < half ? n : n - N) * inv;
      const double x2 = x * x;
      const double ux = u * x, uy = u * y;
      acc[0] += u;
      acc[1] += ux;
      acc[2] += uy;
      acc[3] += ux * x;
      acc[4] += ux * y;
      acc[5] += uy * y;
      acc[6] += ux * x2;
      acc[7] += ux * x * y;
      acc[8] += ux * y2;
      acc[9] += uy * y2;
      acc[10] += ux * x * x2;
      acc[11] += ux * x2 * y;
      acc[12] += ux * x * y2;
      acc[13] += ux * y2 * y;
      acc[14] += uy * y * y2;
    }
    exchange_sync<R::WAVE>();   // rbuf reads done before the next FFT writes xbuf
  }
  // wave reduction, then across waves in fixed order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N_MONO; ++k) {
    double a = acc[k];
    for (int o = WIDTH / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, WIDTH);
    acc[k] = a;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N_MONO; ++k) red[wv][k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x < N_MONO) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w][threadIdx.x];
    partials[((size_t)t * gridDim.x + blockIdx.x) * N_MONO + threadIdx.x] = s;
  }
}

// ------------------------------------------------------------------ launchers
template <int N>
static hipError_t row_pass_n(int F, int t0, const uint16_t* frames, const AxisTab* rows, const AxisTab* cols,
                             const float2* tw, const float* apoly, const float2* outfac, float2* inter,
                             hipStream_t s) {
  using R = RowCfg<N>;
  dim3 grid(N / R::ROWS, F), block(R::THREADS);
  if (apoly && outfac)
    hipLaunchKernelGGL((k_row_pass<N, true, true>), grid, block, 0, s, frames, t0, rows, cols, tw, apoly, outfac, inter);
  else if (apoly)
    hipLaunchKernelGGL((k_row_pass<N, true, false>), grid, block, 0, s, frames, t0, rows, cols, tw, apoly, outfac, inter);
  else if (outfac)
    hipLaunchKernelGGL((k_row_pass<N, false, true>), grid, block, 0, s, frames, t0, rows, cols, tw, apoly, outfac, inter);
  else
    hipLaunchKernelGGL((k_row_pass<N, false, false>), grid, block, 0, s, frames, t0, rows, cols, tw, apoly, outfac, inter);
  return hipGetLastError();
}

// persistent column workgroups: `req` (from the tuner) or 512 (two per CU of the 256 on MI355X)
static int col_grid(int ntiles, int req) {
  const int g = req > 0 ? req : 512;
  return ntiles < g ? ntiles : g;
}

template <int N, int CT>
static int col_default_grid_nt(int cu) {
  // with the tile prefetch: one resident round of workgroups, each walking
  // its tiles; without it, two rounds
  constexpr int per_lds = 163840 / ColLdsT<N, CT>::BYTES;
  constexpr int per_thr = 2048 / (CT * FFTShape<N>::G);   // at most 32 waves per CU
  constexpr int per_cu = per_lds < per_thr ? per_lds : per_thr;
  return ColLdsT<N, CT>::PF ? cu * (per_cu > 0 ? per_cu : 1) : 512;
}

template <int N>
static int col_default_grid_n(int cu, int ct) {
  using K = ColTiles<N>;
  if (ct == K::C2 && K::ALT) return col_default_grid_nt<N, K::C2>(cu);
  if (ct == K::C4 && K::ALT) return col_default_grid_nt<N, K::C4>(cu);
  return col_default_grid_nt<N, K::C>(cu);
}

// Default persistent grid of the transfer-function column pass: one resident
// round of workgroups (its next tile is prefetched, so a second round only
// adds a tail), with the per-CU residency of the compiled kernel
template <int N>
static int as_col_default_grid_n(int cu) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(k_as_col<N>),
                                                   AsColCfg<N>::THREADS, 0) != hipSuccess || nb < 1)
    nb = 1;
  return cu * nb;
}

int as_col_default_grid(int N, int cu) {
  switch (N) {
    case 16: return as_col_default_grid_n<16>(cu);
    case 32: return as_col_default_grid_n<32>(cu);
    case 64: return as_col_default_grid_n<64>(cu);
    case 128: return as_col_default_grid_n<128>(cu);
    case 256: return as_col_default_grid_n<256>(cu);
    case 512: return as_col_default_grid_n<512>(cu);
    case 1024: return as_col_default_grid_n<1024>(cu);
    default: return as_col_default_grid_n<2048>(cu);
  }
}

int col_default_grid(int N, int cu, int ct) {
  switch (N) {
    case 16: return col_default_grid_n<16>(cu, ct);
    case 32: return col_default_grid_n<32>(cu, ct);
    case 64: return col_default_grid_n<64>(cu, ct);
    case 128: return col_default_grid_n<128>(cu, ct);
    case 256: return col_default_grid_n<256>(cu, ct);
    case 512: return col_default_grid_n<512>(cu, ct);
    case 1024: return col_default_grid_n<1024>(cu, ct);
    default: return col_default_grid_n<2048>(cu, ct);
  }
}

template <int N>
static void col_tiles_n(int* out) {
  using K = ColTiles<N>;
  out[0] = K::C;
  out[1] = K::ALT ? K::C2 : 0;
  out[2] = K::ALT ? K::C4 : 0;
}

void col_tiles(int N, int* out) {
  switch (N) {
    case 16: return col_tiles_n<16>(out);
    case 32: return col_tiles_n<32>(out);
    case 64: return col_tiles_n<64>(out);
    case 128: return col_tiles_n<128>(out);
    case 256: return col_tiles_n<256>(out);
    case 512: return col_tiles_n<512>(out);
    case 1024: return col_tiles_n<1024>(out);
    default: return col_tiles_n<2048>(out);
  }
}

// forward column pass of tile width CT and radix order PL (with the Eq. 6
// output phase when outfac is given)
template <int N, int CT, int PL>
static hipError_t col_pass_ntp(int F, const float2* inter, const float2* tw, const float2* outfac, void* dst, int fmt,
                               float scale, int req_grid, int fstride, hipStream_t s, int F2,
                               const float2* inter2, void* dst2, int fstride2) {
  const int ntiles = (F + F2) * (N / CT);
  dim3 grid(col_grid(ntiles, req_grid)), block(CT * FFTShape<N>::G);
#define SSOCT_COL(FMT, E)                                                                                            \
  hipLaunchKernelGGL((k_col_pass<N, +1, FMT, E, CT, PL>), grid, block, 0, s, inter, tw, outfac, dst, scale, ntiles, \
                     fstride, inter2, dst2, F, fstride2)
  if (fmt == HF_F32) { if (outfac) SSOCT_COL(HF_F32, true); else SSOCT_COL(HF_F32, false); }
  else if (fmt == HF_F16) { if (outfac) SSOCT_COL(HF_F16, true); else SSOCT_COL(HF_F16, false); }
  else { if (outfac) SSOCT_COL(HF_BF16, true); else SSOCT_COL(HF_BF16, false); }
#undef SSOCT_COL
  return hipGetLastError();
}

// the same for a runtime radix order (sizes that are a power of 16 have one)
template <int N, int CT>
static hipError_t col_pass_nt(int F, const float2* inter, const float2* tw, const float2* outfac, void* dst, int fmt,
                              float scale, int req_grid, int fstride, hipStream_t s, int F2 = 0,
                              const float2* inter2 = nullptr, void* dst2 = nullptr, int fstride2 = 0,
                              int radix = 0) {
  if constexpr (FFTShape<N>::L > 1) {
    if (radix == 1)
      return col_pass_ntp<N, CT, 1>(F, inter, tw, outfac, dst, fmt, scale, req_grid, fstride, s, F2, inter2, dst2,
                                    fstride2);
  }
  if (radix != 0) return hipErrorInvalidValue;
  return col_pass_ntp<N, CT, 0>(F, inter, tw, outfac, dst, fmt, scale, req_grid, fstride, s, F2, inter2, dst2,
                                fstride2);
}

// ctile: column tile width (the default ColCfg<N>::C, or one of the narrower
// ColTiles alternatives)
template <int N>
static hipError_t col_pass_n(int F, int t0, const float2* inter, const float2* tw, const float2* outfac, void* H,
                             int fmt, int sigma, int req_grid, int ctile, int radix, hipStream_t s) {
  using K = ColTiles<N>;
  const float scale = ldexpf(1.0f, -sigma);
  char* dst = reinterpret_cast<char*>(H) + (size_t)t0 * N * N * 8;
#define SSOCT_COLN(CT) col_pass_nt<N, CT>(F, inter, tw, outfac, dst, fmt, scale, req_grid, 1, s, 0, nullptr, nullptr, 0, radix)
  if (K::ALT && ctile == K::C2) return SSOCT_COLN(K::C2);
  if (K::ALT && ctile == K::C4) return SSOCT_COLN(K::C4);
  return SSOCT_COLN(K::C);
#undef SSOCT_COLN
}

template <int N>
static hipError_t col_pass_adj_n(int F, int t0, const float2* B, const float2* tw, float2* inter, int req_grid,
                                 hipStream_t s) {
  using C = ColCfg<N>;
  const int ntiles = F * (N / C::C);
  dim3 grid(col_grid(ntiles, req_grid)), block(C::THREADS);
  const float2* src = B + (size_t)t0 * N * N;
  hipLaunchKernelGGL((k_col_pass<N, -1, HF_F32, false>), grid, block, 0, s, src, tw, (const float2*)nullptr,
                     (void*)inter, 1.0f, ntiles, 1, (const float2*)nullptr, (void*)nullptr, F, 0);
  return hipGetLastError();
}

template <int N>
static hipError_t row_pass_adj_n(int F, int t0, const uint16_t* frames, const AxisTab* rows, const AxisTab* cols,
                                 const float2* tw, const float2* screen, const float2* inter, double* partials,
                                 hipStream_t s) {
  using R = RowCfg<N>;
  dim3 grid(N / R::ROWS, F), block(R::THREADS);
  if (screen)
    hipLaunchKernelGGL((k_row_pass_adj<N, true>), grid, block, 0, s, frames, t0, rows, cols, tw, screen, inter, partials);
  else
    hipLaunchKernelGGL((k_row_pass_adj<N, false>), grid, block, 0, s, frames, t0, rows, cols, tw, screen, inter, partials);
  return hipGetLastError();
}

#define SSOCT_DISPATCH_N(N, CALL)        \
  switch (N) {                           \
    case 16: return CALL(16);            \
    case 32: return CALL(32);            \
    case 64: return CALL(64);            \
    case 128: return CALL(128);          \
    case 256: return CALL(256);          \
    case 512: return CALL(512);          \
    case 1024: return CALL(1024);        \
    case 2048: return CALL(2048);        \
    default: return hipErrorInvalidValue; \
  }

template <int N, int RPG>
static hipError_t row_pass_g_rpg(int nb, int qa, int T, const float2* G, const AxisTab* rows0, const AxisTab* cols0,
                                 const float2* tw, const float* apoly, const float2* outfac, float2* inter, int Fh,
                                 hipStream_t s) {
  using R = RowCfg<N>;
  dim3 grid(N / (R::GR * RPG), nb), block(R::THREADS);
#define SSOCT_RG(A, E)                                                                                                \
  hipLaunchKernelGGL((k_row_pass_g<N, A, E, RPG>), grid, block, 0, s, G, qa, T, rows0, cols0, tw, apoly, outfac, inter, \
                     Fh)
  if (apoly && outfac) SSOCT_RG(true, true);
  else if (apoly) SSOCT_RG(true, false);
  else if (outfac) SSOCT_RG(false, true);
  else SSOCT_RG(false, false);
#undef SSOCT_RG
  return hipGetLastError();
}

// Rows per group of the bin-pair row pass: `rpg` if it is one of 8, 4, 2 (and
// leaves at least one row group per workgroup's share), else the largest of
// them that still gives two workgroups per CU for the launch's nb bins (a
// chunk of bins has half the frames of a Fresnel chunk, so its row pass
// launches half as many workgroups at the rows per group of k_row_pass).
template <int N>
static hipError_t row_pass_g_n(int nb, int qa, int T, const float2* G, const AxisTab* rows0, const AxisTab* cols0,
                               const float2* tw, const float* apoly, const float2* outfac, float2* inter, int Fh,
                               int rpg, int cu, hipStream_t s) {
  using R = RowCfg<N>;
  constexpr int MAXR = N / R::GR;   // rows per group cannot exceed the rows of one workgroup's share
  if (rpg != 8 && rpg != 4 && rpg != 2) {
    // 4 rows per group where that still gives two workgroups per CU, else 2
    // (8 rows measured slower at every launch size of the paper shape)
    rpg = (N / (R::GR * 4)) * nb >= 2 * cu ? 4 : 2;
  }
  if (rpg > MAXR) rpg = MAXR;
  if (rpg >= 8 && MAXR >= 8) return row_pass_g_rpg<N, (MAXR >= 8 ? 8 : 1)>(nb, qa, T, G, rows0, cols0, tw, apoly, outfac, inter, Fh, s);
  if (rpg >= 4 && MAXR >= 4) return row_pass_g_rpg<N, (MAXR >= 4 ? 4 : 1)>(nb, qa, T, G, rows0, cols0, tw, apoly, outfac, inter, Fh, s);
  if (rpg >= 2 && MAXR >= 2) return row_pass_g_rpg<N, (MAXR >= 2 ? 2 : 1)>(nb, qa, T, G, rows0, cols0, tw, apoly, outfac, inter, Fh, s);
  return row_pass_g_rpg<N, 1>(nb, qa, T, G, rows0, cols0, tw, apoly, outfac, inter, Fh, s);
}

template <int N>
static hipError_t col_pass_v_n(int F, const float2* inter, const float2* tw, const float2* outfac, float2* V,
                               int fstride, int req_grid, int ctile, hipStream_t s, int F2, const float2* inter2,
                               float2* V2, int fstride2, int radix) {
  using K = ColTiles<N>;
#define SSOCT_COLV(CT) \
  col_pass_nt<N, CT>(F, inter, tw, outfac, V, HF_F32, 1.0f, req_grid, fstride, s, F2, inter2, V2, fstride2, radix)
  if (K::ALT && ctile == K::C2) return SSOCT_COLV(K::C2);
  if (K::ALT && ctile == K::C4) return SSOCT_COLV(K::C4);
  return SSOCT_COLV(K::C);
#undef SSOCT_COLV
}

hipError_t launch_row_pass_g(int N, int nb, int qa, int T, const float2* G, const AxisTab* rows0,
                             const AxisTab* cols0, const float2* tw, const float* apoly, const float2* outfac,
                             float2* inter, int Fh, int rpg, int cu, hipStream_t s) {
#define CALL(n) row_pass_g_n<n>(nb, qa, T, G, rows0, cols0, tw, apoly, outfac, inter, Fh, rpg, cu, s)
  SSOCT_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_col_pass_v(int N, int F, const float2* inter, const float2* tw, const float2* outfac, float2* V,
                             int fstride, int grid, int ctile, hipStream_t s, int F2, const float2* inter2,
                             float2* V2, int fstride2, int radix) {
  if (F2 > 0 && !(inter2 && V2)) return hipErrorInvalidValue;
#define CALL(n) col_pass_v_n<n>(F, inter, tw, outfac, V, fstride, grid, ctile, s, F2, inter2, V2, fstride2, radix)
  SSOCT_DISPATCH_N(N, CALL)
#undef CALL
}

template <int N>
static hipError_t as_stage_n(int F, int t0, const uint16_t* frames, const float2* tw, const double* asp,
                             double inv_nd, double z, float2* inter, void* H, int fmt, int sigma, int req_grid,
                             hipStream_t s) {
  using R = RowCfg<N>;
  using C = AsColCfg<N>;
  dim3 rgrid(N / R::ROWS, F), rblock(R::THREADS);
  hipLaunchKernelGGL((k_as_row_fwd<N>), rgrid, rblock, 0, s, frames, t0, tw, inter);
  const int ntiles = F * (N / C::C);
  hipLaunchKernelGGL((k_as_col<N>), dim3(col_grid(ntiles, req_grid)), dim3(C::THREADS), 0, s, inter, t0, tw, asp,
                     inv_nd, z, ntiles);
  const float scale = ldexpf(1.0f, -sigma);
  if (fmt == HF_F32) hipLaunchKernelGGL((k_as_row_inv<N, HF_F32>), rgrid, rblock, 0, s, inter, t0, tw, H, scale);
  else if (fmt == HF_F16) hipLaunchKernelGGL((k_as_row_inv<N, HF_F16>), rgrid, rblock, 0, s, inter, t0, tw, H, scale);
  else hipLaunchKernelGGL((k_as_row_inv<N, HF_BF16>), rgrid, rblock, 0, s, inter, t0, tw, H, scale);
  return hipGetLastError();
}

hipError_t launch_as_stage(int N, int F, int t0, const uint16_t* frames, const float2* tw, const double* asp,
                           double inv_nd, double z, float2* inter, void* H, int fmt, int sigma, int grid,
                           hipStream_t s) {
#define CALL(n) as_stage_n<n>(F, t0, frames, tw, asp, inv_nd, z, inter, H, fmt, sigma, grid, s)
  SSOCT_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_row_pass(int N, int F, int t0, const uint16_t* frames, const AxisTab* rows, const AxisTab* cols,
                           const float2* tw, const float* apoly, const float2* outfac, float2* inter, hipStream_t s) {
#define CALL(n) row_pass_n<n>(F, t0, frames, rows, cols, tw, apoly, outfac, inter, s)
  SSOCT_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_col_pass(int N, int F, int t0, const float2* inter, const float2* tw, const float2* outfac, void* H,
                           int fmt, int sigma, int grid, hipStream_t s, int ctile, int radix) {
#define CALL(n) col_pass_n<n>(F, t0, inter, tw, outfac, H, fmt, sigma, grid, ctile, radix, s)
  SSOCT_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_col_pass_adj(int N, int F, int t0, const float2* B, const float2* tw, float2* inter, int grid,
                               hipStream_t s) {
#define CALL(n) col_pass_adj_n<n>(F, t0, B, tw, inter, grid, s)
  SSOCT_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_row_pass_adj(int N, int F, int t0, const uint16_t* frames, const AxisTab* rows,
                               const AxisTab* cols, const float2* tw, const float2* screen, const float2* inter,
                               double* partials, hipStream_t s) {
#define CALL(n) row_pass_adj_n<n>(F, t0, frames, rows, cols, tw, screen, inter, partials, s)
  SSOCT_DISPATCH_N(N, CALL)
#undef CALL
}

int row_adj_blocks(int N) {
  switch (N) {
    case 16: return 16 / RowCfg<16>::ROWS;
    case 32: return 32 / RowCfg<32>::ROWS;
    case 64: return 64 / RowCfg<64>::ROWS;
    case 128: return 128 / RowCfg<128>::ROWS;
    case 256: return 256 / RowCfg<256>::ROWS;
    case 512: return 512 / RowCfg<512>::ROWS;
    case 1024: return 1024 / RowCfg<1024>::ROWS;
    case 2048: return 2048 / RowCfg<2048>::ROWS;
    default: return 0;
  }
}

}  // namespace ssoct
