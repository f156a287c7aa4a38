// Depth transform of Eq. 7 as a two-factor DFT on MFMA (T = 16 T2,
// T2 = 2..16).  With t = t1 + 16 t2 and q = q2 + T2 q1,
//   V[q2 + T2 q1] = sum_t1 W16[q1][t1] wT^(q2 t1) sum_t2 WT2[q2][t2] h[t1 + 16 t2],
// W_n[a][b] = exp(-2 pi i a b / n), wT = exp(-2 pi i / T).  Each inner sum
// is the product of a small DFT matrix in real form with the stack viewed as
// reals, always with FP32 accumulation:
//  * FP16/BF16 (hi only, or split hi*hi + hi*lo + lo*hi): rows 2k, 2k + 1 =
//    Re W[k], Im W[k], padded to 32 rows, on v_mfma_f32_32x32x16_{f16,bf16};
//    2 x 32 x (T2 + 16) x 16 x 2 flops per pixel and product (65536 at
//    T = 256, 8x fewer than the dense real-form product);
//  * FP32: the paired form (16 rows: W_0, W_{n/2}, Re W_k and Im W_k for
//    k = 1 .. n/2 - 1, which give V[k] and V[n - k]) on
//    v_mfma_f32_16x16x4_f32, half that work again;
// so every precision is bound by the 16 B/voxel of the stack and the volume.
//
// A workgroup (8 waves) owns 32 pixels and all T frames.  Stage A: each
// wave takes MFMA tiles of columns (t1, pixel), K = t2, loading its operands
// from HBM straight into registers (each load covers consecutive pixels of
// one frame); the products, times the twiddle wT^(q2 t1), cross LDS once as
// [q2][t1][pixel] (split into hi/lo for the 16-bit forms).  Stage B: tiles
// of columns (q2, pixel), K = t1; the accumulator holds V for consecutive
// pixels of each bin, written with non-temporal stores.
#include "access.hpp"
#include "fft_engine.hpp"
#include "internal.hpp"
#include "mfma.hpp"
#include "split.hpp"

#ifndef SSOCT_F4_NT
#define SSOCT_F4_NT 1            // non-temporal loads of H and stores of the volume (both touched once)
#endif

namespace ssoct {

#ifndef SSOCT_F4_PX
#define SSOCT_F4_PX 32           // default pixels per tile: 128-byte (16) or 256-byte (32) rows of each frame
#endif
#ifndef SSOCT_F4_THREADS
#define SSOCT_F4_THREADS 512     // workgroup size (waves take 32-column MFMA tiles in turn)
#endif
constexpr int F4_THREADS = SSOCT_F4_THREADS;
constexpr int F4_PX = SSOCT_F4_PX;

// element (row k, column lane) of the real-form DFT matrix of size n:
// row 2a = Re W_n[a][k], row 2a + 1 = Im W_n[a][k]; zero outside a < n, k < n
__device__ __forceinline__ double dft_real_form(int row, int k, int n) {
  const int a = row >> 1;
  if (a >= n || k >= n) return 0.0;
  double s, c;
  sincospi(-2.0 * (double)((a * k) % n) / (double)n, &s, &c);
  return (row & 1) ? s : c;
}

// Paired real form of the n-point DFT matrix (n = 2..16, 16 rows): row 0 =
// W_0, row 1 = W_{n/2} (both real), rows 2k, 2k + 1 = Re W_k, Im W_k for
// k = 1 .. n/2 - 1; rows >= n and columns >= n are zero.  With the products
// A = R h_re and B = R h_im, V[k] = (A_2k - B_2k+1, B_2k + A_2k+1) and
// V[n - k] = (A_2k + B_2k+1, B_2k - A_2k+1): n real rows give all n outputs.
__device__ __forceinline__ double dft_pair_form(int row, int k, int n) {
  if (row >= n || k >= n) return 0.0;
  if (row == 0) return 1.0;
  if (row == 1) return (k & 1) ? -1.0 : 1.0;
  double s, c;
  sincospi(-2.0 * (double)(((row >> 1) * k) % n) / (double)n, &s, &c);
  return (row & 1) ? s : c;
}

// hi | lo << 16 of an FP64 value in FP16 or BF16 (hi = RNE(x), lo = RNE(x - hi))
template <bool BF>
__device__ __forceinline__ uint32_t split_pack64(double x) {
  if constexpr (BF) {
    const uint16_t h = bf16_rne((float)x);
    const uint16_t l = bf16_rne((float)(x - (double)bf16_val(h)));
    return (uint32_t)h | ((uint32_t)l << 16);
  } else {
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)(x - (double)(float)h);
    return (uint32_t)__builtin_bit_cast(uint16_t, h) | ((uint32_t)__builtin_bit_cast(uint16_t, l) << 16);
  }
}

// A operand of a 32x32x16 product for real-form rows `row` and k = k0..k0+7:
// hi halves in hi, lo halves in lo
template <bool BF>
__device__ __forceinline__ void a_operand16(int row, int k0, int n, uint4& hi, uint4& lo) {
  uint32_t p[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) p[i] = split_pack64<BF>(dft_real_form(row, k0 + i, n));
  hi = make_uint4(pack_lo(p[0], p[1]), pack_lo(p[2], p[3]), pack_lo(p[4], p[5]), pack_lo(p[6], p[7]));
  lo = make_uint4(pack_hi(p[0], p[1]), pack_hi(p[2], p[3]), pack_hi(p[4], p[5]), pack_hi(p[6], p[7]));
}

// acc_re/acc_im += A * (re, im of the 8 elements e) for the 16-bit forms
template <int PREC>
__device__ __forceinline__ void mfma16_step(const uint2 (&e)[8], uint4 ahi, uint4 alo, v16f& acc_re, v16f& acc_im) {
  using PT_ = PrecTraits<PREC>;
  uint4 re_hi, im_hi;
  re_hi.x = pack_lo(e[0].x, e[1].x); re_hi.y = pack_lo(e[2].x, e[3].x);
  re_hi.z = pack_lo(e[4].x, e[5].x); re_hi.w = pack_lo(e[6].x, e[7].x);
  im_hi.x = pack_lo(e[0].y, e[1].y); im_hi.y = pack_lo(e[2].y, e[3].y);
  im_hi.z = pack_lo(e[4].y, e[5].y); im_hi.w = pack_lo(e[6].y, e[7].y);
  if constexpr (PT_::SPLIT) {
    uint4 re_lo, im_lo;
    re_lo.x = pack_hi(e[0].x, e[1].x); re_lo.y = pack_hi(e[2].x, e[3].x);
    re_lo.z = pack_hi(e[4].x, e[5].x); re_lo.w = pack_hi(e[6].x, e[7].x);
    im_lo.x = pack_hi(e[0].y, e[1].y); im_lo.y = pack_hi(e[2].y, e[3].y);
    im_lo.z = pack_hi(e[4].y, e[5].y); im_lo.w = pack_hi(e[6].y, e[7].y);
    acc_re = mfma_x16<PT_::BF>(alo, re_hi, acc_re);
    acc_im = mfma_x16<PT_::BF>(alo, im_hi, acc_im);
    acc_re = mfma_x16<PT_::BF>(ahi, re_lo, acc_re);
    acc_im = mfma_x16<PT_::BF>(ahi, im_lo, acc_im);
  }
  acc_re = mfma_x16<PT_::BF>(ahi, re_hi, acc_re);
  acc_im = mfma_x16<PT_::BF>(ahi, im_hi, acc_im);
}

// Per-lane A operands of the T2-point (stage A) and 16-point (stage B) DFT
// matrices, as 16 dwords per lane.  FP32 (v_mfma_f32_16x16x4_f32, lane l
// holds A[l % 16][l / 16] of each K-step of 4): the paired form, a[s] at s,
// b[s] at 8 + s.  16-bit (32x32x16 tiles): the real form, row l % 32,
// ahi, alo, bhi, blo at 0, 4, 8, 12.  Built once per plan from FP64
// (F4_OPS_DWORDS per lane, 64 lanes) and loaded by every workgroup.
constexpr int F4_OPS_DWORDS = 16;

template <int T2>
struct PairSteps {
  static constexpr int KA = (T2 + 3) / 4;   // K-steps of stage A (K = T2, zero-padded to 4)
  static constexpr int KB = 4;              // K-steps of stage B (K = 16)
};

template <int T2, int PREC>
struct AOps {
  float a[PrecTraits<PREC>::F32 ? PairSteps<T2>::KA : 1], b[PrecTraits<PREC>::F32 ? 4 : 1];
  uint4 ahi, alo, bhi, blo;
  __device__ __forceinline__ void build(int l) {
    if constexpr (PrecTraits<PREC>::F32) {
#pragma unroll
      for (int s = 0; s < PairSteps<T2>::KA; ++s) a[s] = (float)dft_pair_form(l % 16, 4 * s + l / 16, T2);
#pragma unroll
      for (int s = 0; s < 4; ++s) b[s] = (float)dft_pair_form(l % 16, 4 * s + l / 16, 16);
    } else {
      a_operand16<PrecTraits<PREC>::BF>(l & 31, 8 * (l >> 5), T2, ahi, alo);
      a_operand16<PrecTraits<PREC>::BF>(l & 31, 8 * (l >> 5), 16, bhi, blo);
    }
  }
  __device__ __forceinline__ void store(uint32_t* dst) const {
    uint4 q[4];
    if constexpr (PrecTraits<PREC>::F32) {
      uint32_t w[16] = {};
#pragma unroll
      for (int s = 0; s < PairSteps<T2>::KA; ++s) w[s] = __float_as_uint(a[s]);
#pragma unroll
      for (int s = 0; s < 4; ++s) w[8 + s] = __float_as_uint(b[s]);
#pragma unroll
      for (int i = 0; i < 4; ++i) q[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
    } else {
      q[0] = ahi; q[1] = alo; q[2] = bhi; q[3] = blo;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) reinterpret_cast<uint4*>(dst)[i] = q[i];
  }
  __device__ __forceinline__ void load(const uint32_t* __restrict__ src) {
    uint4 q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = reinterpret_cast<const uint4*>(src)[i];
    if constexpr (PrecTraits<PREC>::F32) {
      const uint32_t w[16] = {q[0].x, q[0].y, q[0].z, q[0].w, q[1].x, q[1].y, q[1].z, q[1].w,
                              q[2].x, q[2].y, q[2].z, q[2].w, q[3].x, q[3].y, q[3].z, q[3].w};
#pragma unroll
      for (int s = 0; s < PairSteps<T2>::KA; ++s) a[s] = __uint_as_float(w[s]);
#pragma unroll
      for (int s = 0; s < 4; ++s) b[s] = __uint_as_float(w[8 + s]);
    } else {
      ahi = q[0]; alo = q[1]; bhi = q[2]; blo = q[3];
    }
  }
};

template <int T2, int PREC>
__global__ void k_4step_operands(uint32_t* __restrict__ ops) {
  const int l = threadIdx.x;   // 64 lanes
  AOps<T2, PREC> A;
  A.build(l);
  A.store(ops + (size_t)l * F4_OPS_DWORDS);
}

// Stage-A products of column tile j times the twiddle wT^(q2 t1), into the [q2][t1][pixel] tile `dst`
template <int T2, int PREC, int PX>
__device__ __forceinline__ void stage_a_store(uint2* dst, int j, int lc, int lh, const v16f& ar, const v16f& ai,
                                              const float2* __restrict__ wt, float mid_scale) {
  constexpr int T = 16 * T2;
  constexpr int HFMT = PrecTraits<PREC>::BF ? HF_BF16 : HF_F16;
  const int t1 = (32 * j + lc) / PX, px = (32 * j + lc) % PX;
#pragma unroll
  for (int r = 0; r < 16; r += 2) {
    const int q2 = (8 * (r >> 2) + 4 * lh + (r & 3)) >> 1;
    if (q2 >= T2) continue;
    const float2 a = make_float2(ar[r] - ai[r + 1], ai[r] + ar[r + 1]);
    const float2 b = q2 == 0 ? a : cmul(a, wt[(q2 * t1) % T]);
    dst[(q2 * 16 + t1) * PX + px] = make_uint2(split_pack<HFMT>(b.x * mid_scale), split_pack<HFMT>(b.y * mid_scale));
  }
}

// Stage B for column tile j (columns 32 j + lc of (q2, pixel)) of the [q2][t1][pixel] tile `in`,
// and the volume epilogue for pixels p0 + pixel
template <int T2, int PREC, int EPI, int PX>
__device__ __forceinline__ void stage_b(const uint2* in, int j, int lc, int lh, const AOps<T2, PREC>& A,
                                        void* __restrict__ out, int P, int p0, float out_scale) {
  const int q2 = (32 * j + lc) / PX, px = (32 * j + lc) % PX;
  v16f br, bi;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    br[r] = 0.f;
    bi[r] = 0.f;
  }
  uint2 e[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) e[i] = in[(q2 * 16 + 8 * lh + i) * PX + px];
  mfma16_step<PREC>(e, A.bhi, A.blo, br, bi);
#pragma unroll
  for (int r = 0; r < 16; r += 2) {
    const int q1 = (8 * (r >> 2) + 4 * lh + (r & 3)) >> 1;
    const int q = q2 + T2 * q1;
    float2 V = make_float2((br[r] - bi[r + 1]) * out_scale, (bi[r] + br[r + 1]) * out_scale);
    const size_t idx = (size_t)q * P + p0 + px;
    if constexpr (EPI == EPI_ABS)
      st_once<SSOCT_F4_NT>(reinterpret_cast<float*>(out) + idx, sqrtf(V.x * V.x + V.y * V.y));
    else
      st_once<SSOCT_F4_NT>(reinterpret_cast<float2*>(out) + idx, V);
  }
}

template <int T2, int PX>
struct F4Shape {
  static constexpr int T = 16 * T2;
  static constexpr int NW = F4_THREADS / 64;
  static constexpr int TA = 16 * PX / 32;                       // stage-A column tiles (t1, pixel)
  static constexpr int TB = (T2 * PX + 31) / 32;                // stage-B column tiles (q2, pixel)
  static constexpr int TA_W = (TA + NW - 1) / NW, TB_W = (TB + NW - 1) / NW;
  static constexpr int TA16 = PX, TB16 = T2 * PX / 16;       // 16-column tiles (FP32 paired form)
  static constexpr int TA16_W = (TA16 + NW - 1) / NW, TB16_W = (TB16 + NW - 1) / NW;
  static_assert(PX == 16 || PX == 32, "16 or 32 pixels per tile");
  static_assert(T2 >= 2 && T2 <= 16, "T = 32 .. 256");
};

// Stage-A operands of column tile j loaded straight from the stack: lane
// (lc, lh) takes frame t1 + 16 t2 at pixel p0 + px for its k values, so each
// half-wave load is PX consecutive pixels of one frame.
template <int T2, int PREC, int PX>
__device__ __forceinline__ void load_stage_a(const uint2* __restrict__ H, int P, int p0, int j, int lc, int lh,
                                             int shift, uint2 (&e)[8]) {
  constexpr int T = 16 * T2;
  const int t1 = (32 * j + lc) / PX, px = (32 * j + lc) % PX;
  const uint2* src = H + p0 + px;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int t2 = 8 * lh + i;   // k = 8 lh + i of the 32x32x16 step
    const int slot = (t1 + 16 * t2 + shift) & (T - 1);   // a ring window starting `shift` slots in
    e[i] = t2 < T2 ? ld_once<SSOCT_F4_NT>(src + (size_t)slot * P) : make_uint2(0u, 0u);
  }
}

template <int T2, int PREC>
__device__ __forceinline__ void stage_a_regs(const uint2 (&e)[8], const AOps<T2, PREC>& A, v16f& ar, v16f& ai) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    ar[r] = 0.f;
    ai[r] = 0.f;
  }
  mfma16_step<PREC>(e, A.ahi, A.alo, ar, ai);
}

// ------------------------------------------------------------------ FP32: paired form on 16x16x4 tiles
// A 16-column tile: lane l is column c = l % 16 of the tile and K-row
// l / 16 of every step; the accumulator rows 4 (l / 16) + r, r = 0..3, are
// two row pairs of the paired form.
typedef float v4f __attribute__((ext_vector_type(4)));

// outputs of the paired form held by lane group g = l / 16 for an n-point
// matrix: f(k, value) for each DFT index k it completes
template <typename F>
__device__ __forceinline__ void pair_outputs(const v4f& re, const v4f& im, int g, int n, F&& f) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float Ar = re[2 * h], Br = re[2 * h + 1], Ai = im[2 * h], Bi = im[2 * h + 1];
    if (g == 0 && h == 0) {          // rows W_0 and W_{n/2}
      f(0, make_float2(Ar, Ai));
      f(n / 2, make_float2(Br, Bi));
    } else {
      const int k = 2 * g + h;       // rows Re W_k, Im W_k
      if (k < n / 2) {
        f(k, make_float2(Ar - Bi, Ai + Br));
        f(n - k, make_float2(Ar + Bi, Ai - Br));
      }
    }
  }
}

// stage A, 16-column tile j of (t1, pixel): operands straight from the stack
template <int T2, int PX>
__device__ __forceinline__ void load_stage_a_pair(const uint2* __restrict__ H, int P, int p0, int j, int l,
                                                  int shift, uint2 (&e)[PairSteps<T2>::KA]) {
  constexpr int T = 16 * T2;
  const int t1 = (16 * j + l % 16) / PX, px = (16 * j + l % 16) % PX;
  const uint2* src = H + p0 + px;
#pragma unroll
  for (int s = 0; s < PairSteps<T2>::KA; ++s) {
    const int t2 = 4 * s + l / 16;
    const int slot = (t1 + 16 * t2 + shift) & (T - 1);   // a ring window starting `shift` slots in
    e[s] = t2 < T2 ? ld_once<SSOCT_F4_NT>(src + (size_t)slot * P) : make_uint2(0u, 0u);
  }
}

template <int T2, int PX>
__device__ __forceinline__ void stage_a_pair(const uint2 (&e)[PairSteps<T2>::KA], const AOps<T2, DP_F32>& A,
                                             uint2* dst, int j, int l, const float2* __restrict__ wt) {
  constexpr int T = 16 * T2;
  v4f re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < PairSteps<T2>::KA; ++s) {
    re = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[s], __uint_as_float(e[s].x), re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[s], __uint_as_float(e[s].y), im, 0, 0, 0);
  }
  const int t1 = (16 * j + l % 16) / PX, px = (16 * j + l % 16) % PX;
  pair_outputs(re, im, l / 16, T2, [&](int q2, float2 a) {
    const float2 b = q2 == 0 ? a : cmul(a, wt[(q2 * t1) % T]);
    dst[(q2 * 16 + t1) * PX + px] = make_uint2(__float_as_uint(b.x), __float_as_uint(b.y));
  });
}

template <int T2, int EPI, int PX>
__device__ __forceinline__ void stage_b_pair(const uint2* in, int j, int l, const AOps<T2, DP_F32>& A,
                                             void* __restrict__ out, int P, int p0) {
  const int q2 = (16 * j + l % 16) / PX, px = (16 * j + l % 16) % PX;
  v4f re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const uint2 b = in[(q2 * 16 + 4 * s + l / 16) * PX + px];
    re = __builtin_amdgcn_mfma_f32_16x16x4f32(A.b[s], __uint_as_float(b.x), re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f32_16x16x4f32(A.b[s], __uint_as_float(b.y), im, 0, 0, 0);
  }
  pair_outputs(re, im, l / 16, 16, [&](int q1, float2 V) {
    const size_t idx = (size_t)(q2 + T2 * q1) * P + p0 + px;
    if constexpr (EPI == EPI_ABS)
      st_once<SSOCT_F4_NT>(reinterpret_cast<float*>(out) + idx, sqrtf(V.x * V.x + V.y * V.y));
    else
      st_once<SSOCT_F4_NT>(reinterpret_cast<float2*>(out) + idx, V);
  });
}

// One workgroup per tile of PX pixels and all T frames: the stage-A
// operands go from HBM to registers, the stage-A products cross LDS once,
// stage B writes the volume.
template <int T2, int PREC, int EPI, int PX>
__global__ __launch_bounds__(F4_THREADS) void k_depth_4step(const uint2* __restrict__ H,
                                                            const float2* __restrict__ wt,
                                                            const uint32_t* __restrict__ ops, void* __restrict__ out,
                                                            int P, float mid_scale, float out_scale, int shift) {
  using S = F4Shape<T2, PX>;
  __shared__ uint2 buf[S::T * PX];   // [q2][t1][pixel]
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lc = l & 31, lh = l >> 5;
  const int p0 = blockIdx.x * PX;    // grid = P / PX
  AOps<T2, PREC> A;
  if constexpr (PrecTraits<PREC>::F32) {
    uint2 e[S::TA16_W][PairSteps<T2>::KA];
#pragma unroll
    for (int jj = 0; jj < S::TA16_W; ++jj) {
      const int j = w + S::NW * jj;
      if (j < S::TA16) load_stage_a_pair<T2, PX>(H, P, p0, j, l, shift, e[jj]);
    }
    A.load(ops + (size_t)l * F4_OPS_DWORDS);
#pragma unroll
    for (int jj = 0; jj < S::TA16_W; ++jj) {
      const int j = w + S::NW * jj;
      if (j >= S::TA16) break;
      stage_a_pair<T2, PX>(e[jj], A, buf, j, l, wt);
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < S::TB16_W; ++jj) {
      const int j = w + S::NW * jj;
      if (j < S::TB16) stage_b_pair<T2, EPI, PX>(buf, j, l, A, out, P, p0);
    }
  } else {
    uint2 e[S::TA_W][8];
#pragma unroll
    for (int jj = 0; jj < S::TA_W; ++jj) {
      const int j = w + S::NW * jj;
      if (j < S::TA) load_stage_a<T2, PREC, PX>(H, P, p0, j, lc, lh, shift, e[jj]);
    }
    A.load(ops + (size_t)l * F4_OPS_DWORDS);
#pragma unroll
    for (int jj = 0; jj < S::TA_W; ++jj) {
      const int j = w + S::NW * jj;
      if (j >= S::TA) break;
      v16f ar, ai;
      stage_a_regs<T2, PREC>(e[jj], A, ar, ai);
      stage_a_store<T2, PREC, PX>(buf, j, lc, lh, ar, ai, wt, mid_scale);
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < S::TB_W; ++jj) {
      const int j = w + S::NW * jj;
      if (j < S::TB) stage_b<T2, PREC, EPI, PX>(buf, j, lc, lh, A, out, P, p0, out_scale);
    }
  }
}

template <int T2, int PREC, int EPI, int PX>
static hipError_t go_4step(int P, const void* H, const float2* wt, const uint32_t* ops, void* out, float mid,
                           float os, int shift, hipStream_t s) {
  hipLaunchKernelGGL((k_depth_4step<T2, PREC, EPI, PX>), dim3(P / PX), dim3(F4_THREADS), 0, s,
                     reinterpret_cast<const uint2*>(H), wt, ops, out, P, mid, os, shift);
  return hipGetLastError();
}

template <int T2, int PREC, int PX>
static hipError_t go_4step_epi(int epi, int P, const void* H, const float2* wt, const uint32_t* ops, void* out,
                               float mid, float os, int shift, hipStream_t s) {
  if (epi == EPI_ABS) return go_4step<T2, PREC, EPI_ABS, PX>(P, H, wt, ops, out, mid, os, shift, s);
  return go_4step<T2, PREC, EPI_STORE, PX>(P, H, wt, ops, out, mid, os, shift, s);
}

template <int T2, int PREC>
static hipError_t go_4step_px(int px, int epi, int P, const void* H, const float2* wt, const uint32_t* ops,
                              void* out, float mid, float os, int shift, hipStream_t s) {
  if (px == 16) return go_4step_epi<T2, PREC, 16>(epi, P, H, wt, ops, out, mid, os, shift, s);
  return go_4step_epi<T2, PREC, 32>(epi, P, H, wt, ops, out, mid, os, shift, s);
}

template <int T2>
static hipError_t go_4step_prec(int prec, int px, int epi, int P, const void* H, const float2* wt,
                                const uint32_t* ops, void* out, float mid, float os, int shift, hipStream_t s) {
  switch (prec) {
    case DP_F32: return go_4step_px<T2, DP_F32>(px, epi, P, H, wt, ops, out, mid, os, shift, s);
    case DP_F16: return go_4step_px<T2, DP_F16>(px, epi, P, H, wt, ops, out, mid, os, shift, s);
    case DP_BF16: return go_4step_px<T2, DP_BF16>(px, epi, P, H, wt, ops, out, mid, os, shift, s);
    case DP_F16_SPLIT: return go_4step_px<T2, DP_F16_SPLIT>(px, epi, P, H, wt, ops, out, mid, os, shift, s);
    case DP_BF16_SPLIT: return go_4step_px<T2, DP_BF16_SPLIT>(px, epi, P, H, wt, ops, out, mid, os, shift, s);
    default: return hipErrorInvalidValue;
  }
}

bool depth_4step_supported(int T) { return T == 32 || T == 64 || T == 128 || T == 256; }

size_t depth_4step_ops_bytes() { return (size_t)64 * F4_OPS_DWORDS * sizeof(uint32_t); }

template <int T2>
static hipError_t ops_prec(int prec, uint32_t* ops, hipStream_t s) {
  switch (prec) {
    case DP_F32: hipLaunchKernelGGL((k_4step_operands<T2, DP_F32>), dim3(1), dim3(64), 0, s, ops); break;
    case DP_F16: hipLaunchKernelGGL((k_4step_operands<T2, DP_F16>), dim3(1), dim3(64), 0, s, ops); break;
    case DP_BF16: hipLaunchKernelGGL((k_4step_operands<T2, DP_BF16>), dim3(1), dim3(64), 0, s, ops); break;
    case DP_F16_SPLIT: hipLaunchKernelGGL((k_4step_operands<T2, DP_F16_SPLIT>), dim3(1), dim3(64), 0, s, ops); break;
    case DP_BF16_SPLIT: hipLaunchKernelGGL((k_4step_operands<T2, DP_BF16_SPLIT>), dim3(1), dim3(64), 0, s, ops); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_4step_operands(int T, int prec, uint32_t* ops, hipStream_t s) {
  switch (T) {
    case 32: return ops_prec<2>(prec, ops, s);
    case 64: return ops_prec<4>(prec, ops, s);
    case 128: return ops_prec<8>(prec, ops, s);
    case 256: return ops_prec<16>(prec, ops, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_depth_4step(int T, int P, int prec, int epi, const void* H, const float2* wt, const uint32_t* ops,
                              void* out, int sigma, hipStream_t s, int shift, int px) {
  if (P <= 0) return hipSuccess;
  if (!ops) return hipErrorInvalidValue;
  if (px == 0) px = F4_PX;
  if ((px != 16 && px != 32) || P % px != 0 || (epi != EPI_STORE && epi != EPI_ABS) || shift < 0 || shift >= T)
    return hipErrorInvalidValue;
  const int T2 = T / 16;
  // FP16 stage-B operands: the stage-A sums grow by up to T2, scaled back by an exact power of two
  const bool f16 = prec == DP_F16 || prec == DP_F16_SPLIT;
  const float mid = f16 ? 1.0f / (float)T2 : 1.0f;
  const float os = ldexpf(f16 ? (float)T2 : 1.0f, sigma);
  switch (T) {
    case 32: return go_4step_prec<2>(prec, px, epi, P, H, wt, ops, out, mid, os, shift, s);
    case 64: return go_4step_prec<4>(prec, px, epi, P, H, wt, ops, out, mid, os, shift, s);
    case 128: return go_4step_prec<8>(prec, px, epi, P, H, wt, ops, out, mid, os, shift, s);
    case 256: return go_4step_prec<16>(prec, px, epi, P, H, wt, ops, out, mid, os, shift, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ssoct
