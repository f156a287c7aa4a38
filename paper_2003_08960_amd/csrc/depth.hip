// Depth transform (Eq. 7 with a rectangular gate over the T frames of a
// sweep) as a dense real GEMM on MFMA.
//
// The complex DFT matrix W[q][t] = exp(-2 pi i q t / T) has W_{T-q} =
// conj(W_q).  With A_q = sum_t Re(W_q[t]) h_t and B_q = sum_t Im(W_q[t]) h_t,
//     V[q]   = A_q + i B_q,     V[T-q] = A_q - i B_q,
// so one T x T real matrix whose rows are the pairs (Re W_q, Im W_q)
// (q = 1 .. T-1-T/2, plus the pair (W_0, W_{T/2})) applied to the complex
// stack viewed as reals gives the whole spectrum with 4 T^2 real flops per
// pixel instead of 8 T^2.  The adjoint (exp(+2 pi i q t / T)) swaps V[q] and
// V[T-q].
//
// Work split: a workgroup owns all M rows (one wave per 32-row block, rows
// kept in registers for the life of the kernel) and walks 32-pixel tiles of
// the stack; each tile of KC frames x 32 pixels is staged in LDS and read by
// every wave.  Row pairs (2k, 2k+1) and the re/im columns of a pixel land in
// the same lane of the 32x32 accumulator, so the epilogue needs no exchange.
//
// Operand precisions: FP32 (v_mfma_f32_32x32x2_f32), FP16/BF16 hi only, and
// FP16/BF16 split hi*hi + hi*lo + lo*hi (v_mfma_f32_32x32x16_{f16,bf16}),
// always with FP32 accumulation.
#include "access.hpp"
#include "internal.hpp"
#include "mfma.hpp"

#ifndef SSOCT_DEPTH_NT
#define SSOCT_DEPTH_NT 0         // non-temporal loads of H and stores of the volume
#endif

namespace ssoct {

constexpr int PT = 32;  // pixels per tile

template <int PREC, int KC, int WAVES, int DIR, int EPI>
__global__ __launch_bounds__(WAVES * 64) void k_depth(const uint2* __restrict__ in, const void* __restrict__ amat,
                                                      void* __restrict__ out, int T, int T_pad, int P, int slabs,
                                                      float out_scale, float gamma_scale,
                                                      double* __restrict__ loss_partials,
                                                      const float2* __restrict__ wt, int shift, int general) {
  using PT_ = PrecTraits<PREC>;
  constexpr int NA = PT_::F32 ? KC / 2 : (PT_::SPLIT ? KC / 2 : KC / 4);  // dwords of A per lane
  constexpr int PER_ROW = PT / 2;                                       // uint4 per tile row
  constexpr int ROWS_PER_PASS = WAVES * 64 / PER_ROW;
  constexpr int NLD = (KC + ROWS_PER_PASS - 1) / ROWS_PER_PASS;         // prefetch registers (uint4)
  __shared__ uint2 btile[KC * PT];
  __shared__ double red[WAVES];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nch = T_pad / KC;
  const int ntp = P / PT;
  const int ntiles = ntp * slabs;
  const int h = T / 2;
  const int npairs = general ? T : T - h;   // general matrix: one row pair per bin
  const int my_tiles = blockIdx.x < ntiles ? (ntiles - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int nitems = my_tiles * nch;                                    // (tile, chunk) work items
  const int cq = threadIdx.x % PER_ROW, r0 = threadIdx.x / PER_ROW;
  uint32_t a[NA];
  uint4 pf[NLD];
  double loss = 0.0;
  int a_slab = -1, a_chunk = -1;
  v16f acc_re, acc_im;

  // global loads of work item `it` (KC frames x 32 pixels) into pf, zero past T
  auto issue = [&](int it) {
    const int tile = blockIdx.x + (it / nch) * gridDim.x;
    const int ch = it % nch;
    const int p0 = (tile % ntp) * PT;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int r = r0 + i * ROWS_PER_PASS;
      const int t = ch * KC + r;
      pf[i] = make_uint4(0u, 0u, 0u, 0u);
      if (r < KC && t < T) pf[i] = ld_once<SSOCT_DEPTH_NT>(reinterpret_cast<const uint4*>(in + (size_t)t * P + p0 + 2 * cq));
    }
  };

  if (nitems > 0) issue(0);
  for (int it = 0; it < nitems; ++it) {
    const int tile = blockIdx.x + (it / nch) * gridDim.x;
    const int ch = it % nch;
    const int slab = tile / ntp;
    const int p0 = (tile % ntp) * PT;
    const int rb = slab * WAVES + w;       // this wave's row block
    if (ch == 0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        acc_re[i] = 0.f;
        acc_im[i] = 0.f;
      }
    }
    // ---- A rows for (slab, chunk): loaded once when there is one slab and one chunk
    if (a_slab != slab || a_chunk != ch) {
      if constexpr (PT_::F32) {
        const float* src = reinterpret_cast<const float*>(amat) + ((size_t)rb * (T_pad / 2) + ch * (KC / 2)) * 64 + l;
#pragma unroll
        for (int s = 0; s < KC / 2; ++s) a[s] = __float_as_uint(src[(size_t)s * 64]);
      } else {
        const uint4* src = reinterpret_cast<const uint4*>(amat) + ((size_t)rb * (T_pad / 16) + ch * (KC / 16)) * 128 + l;
#pragma unroll
        for (int s = 0; s < KC / 16; ++s) {
          const uint4 hi = src[(size_t)s * 128];
          a[(PT_::SPLIT ? 8 : 4) * s + 0] = hi.x;
          a[(PT_::SPLIT ? 8 : 4) * s + 1] = hi.y;
          a[(PT_::SPLIT ? 8 : 4) * s + 2] = hi.z;
          a[(PT_::SPLIT ? 8 : 4) * s + 3] = hi.w;
          if constexpr (PT_::SPLIT) {
            const uint4 lo = src[(size_t)s * 128 + 64];
            a[8 * s + 4] = lo.x;
            a[8 * s + 5] = lo.y;
            a[8 * s + 6] = lo.z;
            a[8 * s + 7] = lo.w;
          }
        }
      }
      a_slab = slab;
      a_chunk = ch;
    }
    // ---- publish the prefetched tile, then start loading the next one
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int r = r0 + i * ROWS_PER_PASS;
      if (r < KC) *reinterpret_cast<uint4*>(&btile[r * PT + 2 * cq]) = pf[i];
    }
    __syncthreads();
    if (it + 1 < nitems) issue(it + 1);
    // ---- MFMA over the chunk
    if constexpr (PT_::F32) {
#pragma unroll
      for (int s = 0; s < KC / 2; ++s) {
        const uint2 b = btile[(2 * s + (l >> 5)) * PT + (l & 31)];
        const float av = __uint_as_float(a[s]);
        acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(av, __uint_as_float(b.x), acc_re, 0, 0, 0);
        acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(av, __uint_as_float(b.y), acc_im, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < KC / 16; ++s) {
        uint2 e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = btile[(16 * s + 8 * (l >> 5) + i) * PT + (l & 31)];
        uint4 re_hi, im_hi, re_lo, im_lo;
        re_hi.x = pack_lo(e[0].x, e[1].x); re_hi.y = pack_lo(e[2].x, e[3].x);
        re_hi.z = pack_lo(e[4].x, e[5].x); re_hi.w = pack_lo(e[6].x, e[7].x);
        im_hi.x = pack_lo(e[0].y, e[1].y); im_hi.y = pack_lo(e[2].y, e[3].y);
        im_hi.z = pack_lo(e[4].y, e[5].y); im_hi.w = pack_lo(e[6].y, e[7].y);
        const int ai = (PT_::SPLIT ? 8 : 4) * s;
        const uint4 ahi = make_uint4(a[ai], a[ai + 1], a[ai + 2], a[ai + 3]);
        if constexpr (PT_::SPLIT) {
          re_lo.x = pack_hi(e[0].x, e[1].x); re_lo.y = pack_hi(e[2].x, e[3].x);
          re_lo.z = pack_hi(e[4].x, e[5].x); re_lo.w = pack_hi(e[6].x, e[7].x);
          im_lo.x = pack_hi(e[0].y, e[1].y); im_lo.y = pack_hi(e[2].y, e[3].y);
          im_lo.z = pack_hi(e[4].y, e[5].y); im_lo.w = pack_hi(e[6].y, e[7].y);
          const uint4 alo = make_uint4(a[ai + 4], a[ai + 5], a[ai + 6], a[ai + 7]);
          acc_re = mfma_x16<PT_::BF>(alo, re_hi, acc_re);
          acc_im = mfma_x16<PT_::BF>(alo, im_hi, acc_im);
          acc_re = mfma_x16<PT_::BF>(ahi, re_lo, acc_re);
          acc_im = mfma_x16<PT_::BF>(ahi, im_lo, acc_im);
        }
        acc_re = mfma_x16<PT_::BF>(ahi, re_hi, acc_re);
        acc_im = mfma_x16<PT_::BF>(ahi, im_hi, acc_im);
      }
    }
    if (ch != nch - 1) continue;
    // ---- epilogue: lane holds rows 8 (r/4) + 4 (l/32) + r%4 of its block, column l%32
    const int p = p0 + (l & 31);
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int row = rb * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
      const int k = row >> 1;
      if (k >= npairs) continue;
      const float Ar = acc_re[r] * out_scale, Ai = acc_im[r] * out_scale;
      const float Br = acc_re[r + 1] * out_scale, Bi = acc_im[r + 1] * out_scale;
      float2 v1, v2;
      int q1, q2;
      if (general) {          // rows (Re W_k, Im W_k) of a general matrix: V[k] = A + i B
        q1 = k; v1 = make_float2(Ar - Bi, Ai + Br);
        q2 = -1; v2 = v1;
      } else if (k == 0) {
        q1 = 0; v1 = make_float2(Ar, Ai);
        q2 = (T % 2 == 0) ? h : -1; v2 = make_float2(Br, Bi);
      } else {
        const float2 vq = make_float2(Ar - Bi, Ai + Br);
        const float2 vm = make_float2(Ar + Bi, Ai - Br);
        q1 = k; q2 = T - k;
        v1 = DIR > 0 ? vq : vm;
        v2 = DIR > 0 ? vm : vq;
      }
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const int q = o == 0 ? q1 : q2;
        if (q < 0) continue;
        float2 V = o == 0 ? v1 : v2;
        const size_t idx = (size_t)q * P + p;
        if constexpr (EPI == EPI_STORE) {
          // window starting `shift` frames into the ring: bin q gains exp(+2 pi i q shift / T)
          if (DIR > 0 && shift != 0) {
            const float2 w = wt[(q * shift) % T];   // V conj(w)
            V = make_float2(V.x * w.x + V.y * w.y, V.y * w.x - V.x * w.y);
          }
          st_once<SSOCT_DEPTH_NT>(reinterpret_cast<float2*>(out) + idx, V);
        } else if constexpr (EPI == EPI_ABS) {
          st_once<SSOCT_DEPTH_NT>(reinterpret_cast<float*>(out) + idx, sqrtf(V.x * V.x + V.y * V.y));
        } else {
          const double a2 = (double)V.x * V.x + (double)V.y * V.y;
          loss += a2 * a2;
          const float sx = V.x * gamma_scale, sy = V.y * gamma_scale;
          const float m2 = 4.0f * (sx * sx + sy * sy);
          reinterpret_cast<float2*>(out)[idx] = make_float2(m2 * sx, m2 * sy);
        }
      }
    }
  }
  if constexpr (EPI == EPI_GAMMA) {
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if (l == 0) red[w] = loss;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int i = 0; i < WAVES; ++i) s += red[i];
      loss_partials[blockIdx.x] = s;
    }
  }
}

template <int PREC, int KC, int WAVES, int DIR, int EPI>
static hipError_t depth_go(int grid, hipStream_t s, const void* in, const void* amat, void* out, int T, int T_pad,
                           int P, int slabs, float out_scale, float gamma_scale, double* partials, const float2* wt,
                           int shift, int general) {
  hipLaunchKernelGGL((k_depth<PREC, KC, WAVES, DIR, EPI>), dim3(grid), dim3(WAVES * 64), 0, s,
                     reinterpret_cast<const uint2*>(in), amat, out, T, T_pad, P, slabs, out_scale, gamma_scale,
                     partials, wt, shift, general);
  return hipGetLastError();
}

template <int PREC, int KC, int WAVES>
static hipError_t depth_dir_epi(int dir, int epi, int grid, hipStream_t s, const void* in, const void* amat,
                                void* out, int T, int T_pad, int P, int slabs, float os, float gs, double* part, const float2* wt, int shift, int general) {
  if (dir > 0) {
    if (epi == EPI_STORE) return depth_go<PREC, KC, WAVES, +1, EPI_STORE>(grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    if (epi == EPI_ABS) return depth_go<PREC, KC, WAVES, +1, EPI_ABS>(grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    if constexpr (PREC == DP_F32)
      return depth_go<PREC, KC, WAVES, +1, EPI_GAMMA>(grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    return hipErrorInvalidValue;
  }
  if constexpr (PREC == DP_F32) {
    if (epi == EPI_STORE) return depth_go<PREC, KC, WAVES, -1, EPI_STORE>(grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
  }
  return hipErrorInvalidValue;
}

template <int PREC, int KC>
static hipError_t depth_waves(int waves, int dir, int epi, int grid, hipStream_t s, const void* in, const void* amat,
                              void* out, int T, int T_pad, int P, int slabs, float os, float gs, double* part, const float2* wt, int shift, int general) {
  switch (waves) {
    case 1: return depth_dir_epi<PREC, KC, 1>(dir, epi, grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    case 2: return depth_dir_epi<PREC, KC, 2>(dir, epi, grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    case 4: return depth_dir_epi<PREC, KC, 4>(dir, epi, grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    case 8: return depth_dir_epi<PREC, KC, 8>(dir, epi, grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    default: return hipErrorInvalidValue;
  }
}

template <int PREC>
static hipError_t depth_kc(int KC, int waves, int dir, int epi, int grid, hipStream_t s, const void* in,
                           const void* amat, void* out, int T, int T_pad, int P, int slabs, float os, float gs,
                           double* part, const float2* wt, int shift, int general) {
  switch (KC) {
    case 32: return depth_waves<PREC, 32>(waves, dir, epi, grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    case 64: return depth_waves<PREC, 64>(waves, dir, epi, grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    case 128: return depth_waves<PREC, 128>(waves, dir, epi, grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    case 256: return depth_waves<PREC, 256>(waves, dir, epi, grid, s, in, amat, out, T, T_pad, P, slabs, os, gs, part, wt, shift, general);
    default: return hipErrorInvalidValue;
  }
}

int depth_grid(int T, int P, int cu_count, bool general) {
  DepthLayout L = depth_layout(T, general);
  const int ntiles = (P / PT) * L.slabs;
  int per_cu = 8 / L.waves;          // waves per CU target ~8
  if (per_cu < 1) per_cu = 1;
  const int g = cu_count * per_cu;
  return ntiles < g ? ntiles : g;
}

hipError_t launch_depth(int T, int P, int prec, int dir, int epi, const void* in, const void* amat, void* out,
                        int sigma, int gamma_exp, double* partials, int grid, hipStream_t s, const float2* wt,
                        int shift, bool general, int kc) {
  if (shift != 0 && !wt) return hipErrorInvalidValue;
  if (general && (dir < 0 || epi == EPI_GAMMA || shift != 0)) return hipErrorInvalidValue;   // forward only
  DepthLayout L = depth_layout(T, general);
  // a smaller K chunk that divides the layout's keeps T_pad and the matrix layout (the K sum runs
  // through the same products in the same order, chunk after chunk)
  if (kc != 0) {
    if (kc < 32 || kc > L.KC || L.KC % kc != 0) return hipErrorInvalidValue;
    L.KC = kc;
  }
  const int gen = general ? 1 : 0;
  const float os = ldexpf(1.0f, sigma);
  const float gs = ldexpf(1.0f, -gamma_exp);
  switch (prec) {
    case DP_F32: return depth_kc<DP_F32>(L.KC, L.waves, dir, epi, grid, s, in, amat, out, T, L.T_pad, P, L.slabs, os, gs, partials, wt, shift, gen);
    case DP_F16: return depth_kc<DP_F16>(L.KC, L.waves, dir, epi, grid, s, in, amat, out, T, L.T_pad, P, L.slabs, os, gs, partials, wt, shift, gen);
    case DP_BF16: return depth_kc<DP_BF16>(L.KC, L.waves, dir, epi, grid, s, in, amat, out, T, L.T_pad, P, L.slabs, os, gs, partials, wt, shift, gen);
    case DP_F16_SPLIT: return depth_kc<DP_F16_SPLIT>(L.KC, L.waves, dir, epi, grid, s, in, amat, out, T, L.T_pad, P, L.slabs, os, gs, partials, wt, shift, gen);
    case DP_BF16_SPLIT: return depth_kc<DP_BF16_SPLIT>(L.KC, L.waves, dir, epi, grid, s, in, amat, out, T, L.T_pad, P, L.slabs, os, gs, partials, wt, shift, gen);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ssoct
