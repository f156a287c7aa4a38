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
#ifndef SSOCT_XCDS
#define SSOCT_XCDS 8             // accelerator complex dies of an MI355X (one L2 each)
#endif
#ifndef SSOCT_DFFT_WGCU
#define SSOCT_DFFT_WGCU 0        // > 0: that many resident workgroups per CU walk the tiles; 0: one per tile
#endif
#ifndef SSOCT_DFFT_NT
#define SSOCT_DFFT_NT 1          // non-temporal loads of H and stores of the volume (both touched once)
#endif

// stage A for the tile of pixels base..base+PX-1: DFT over t2 of h[r + 16 t2],
// times the twiddles, into lds as [q2][t1][px].  With shift > 0 the stack is
// a ring whose window starts `shift` slots in: h[t] is ring slot (t + shift) mod T.
template <int T2, int DIR, int PX>
__device__ __forceinline__ void fft_stage_a_regs(const float2* __restrict__ H, float2 (&a)[T2], int P, int base,
                                                 int px, int r, bool live, int shift) {
  constexpr int T = 16 * T2;
#pragma unroll
  for (int t2 = 0; t2 < T2; ++t2) {
    const int slot = (r + 16 * t2 + shift) & (T - 1);
    a[t2] = live ? ld_once<SSOCT_DFFT_NT>(H + (size_t)slot * P + base + px) : make_float2(0.f, 0.f);
  }
  if constexpr (T2 > 1) dft_small<T2, -DIR>(a);   // engine sign: forward depth DFT has exponent -2 pi i q t / T
}

// bins q2 = q0 .. q0 + NQ - 1 of stage A, times the twiddles, into lds as [q2 - q0][t1][px]
template <int T2, int DIR, int PX, int NQ>
__device__ __forceinline__ void fft_stage_a_publish(const float2 (&a)[T2], const float2* __restrict__ wt,
                                                    float2* lds, int q0, int px, int r) {
  constexpr int T = 16 * T2;
#pragma unroll
  for (int ql = 0; ql < NQ; ++ql) {
    const int q2 = q0 + ql;
    float2 w = wt[(q2 * r) % T];     // exp(-2 pi i q2 t1 / T), FP64-derived
    if constexpr (DIR < 0) w = cconj(w);
    lds[(ql * 16 + r) * PX + px] = q2 == 0 ? a[q2] : cmul(a[q2], w);
  }
}

template <int T2, int DIR, int PX>
__device__ __forceinline__ void fft_stage_a(const float2* __restrict__ H, const float2* __restrict__ wt, float2* lds,
                                            int P, int base, int px, int r, bool live, int shift = 0) {
  float2 a[T2];
  fft_stage_a_regs<T2, DIR, PX>(H, a, P, base, px, r, live, shift);
  fft_stage_a_publish<T2, DIR, PX, T2>(a, wt, lds, 0, px, r);
}

// stage B for bin column q2 = r: 16-point DFT over t1 of the LDS tile
template <int T2, int DIR, int PX>
__device__ __forceinline__ void fft_stage_b(const float2* lds, int px, int r, float2 (&b)[16]) {
#pragma unroll
  for (int t1 = 0; t1 < 16; ++t1) b[t1] = lds[(r * 16 + t1) * PX + px];
  dft16<-DIR>(b);
}

// EPI_STORE / EPI_ABS: workgroups walk the PX-pixel tiles with stride
// gridDim.x (one tile each when the grid covers them all).
template <int T2, int DIR, int EPI, int PX>
__global__ __launch_bounds__(16 * PX) void k_depth_fft(const float2* __restrict__ H, const float2* __restrict__ wt,
                                                        void* __restrict__ out, int P_, int shift) {
  constexpr int T = 16 * T2;
  __shared__ float2 lds[T * PX];     // [q2][t1][px]
  const int px = threadIdx.x % PX, r_ = threadIdx.x / PX;   // r = t1 in stage A, q2 in stage B
  const int ntiles = (P_ + PX - 1) / PX;
#pragma unroll 1
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int P = P_, r = r_;
    if (SSOCT_DFFT_WGCU > 0) {
      if (tile != (int)blockIdx.x) __syncthreads();   // the previous tile's stage-B reads are done
      // P and r opaque per tile: their offset and twiddle products are recomputed,
      // not held in registers across the loop
      asm volatile("" : "+s"(P));
      asm volatile("" : "+v"(r));
    }
    const int base = tile * PX;
    const bool live = base + px < P;
    fft_stage_a<T2, DIR, PX>(H, wt, lds, P, base, px, r, live, shift);
    __syncthreads();
    if (r < T2) {   // stage B for bin column q2 = r
      float2 b[16];
      fft_stage_b<T2, DIR, PX>(lds, px, r, b);
      if (live) {
#pragma unroll
        for (int q1 = 0; q1 < 16; ++q1) {
          const size_t idx = (size_t)(r + T2 * q1) * P + base + px;
          if constexpr (EPI == EPI_ABS)
            st_once<SSOCT_DFFT_NT>(reinterpret_cast<float*>(out) + idx, sqrtf(b[q1].x * b[q1].x + b[q1].y * b[q1].y));
          else
            st_once<SSOCT_DFFT_NT>(reinterpret_cast<float2*>(out) + idx, b[q1]);
        }
      }
    }
    if (SSOCT_DFFT_WGCU == 0) break;   // one tile per workgroup
  }
}

// EPI_GAMMA (forward): Gamma = 4 |V~|^2 V~ with V~ = V 2^-e and one FP64
// partial of sum |V|^4 per workgroup, one tile per workgroup.
template <int T2, int PX>
__global__ __launch_bounds__(16 * PX) void k_depth_fft_gamma(const float2* __restrict__ H,
                                                              const float2* __restrict__ wt, float2* __restrict__ out,
                                                              int P, float gamma_scale,
                                                              double* __restrict__ loss_partials) {
  constexpr int T = 16 * T2;
  __shared__ float2 lds[T * PX];
  __shared__ double red[16 * PX / 64];
  const int px = threadIdx.x % PX, r = threadIdx.x / PX;
  const int base = blockIdx.x * PX;
  const bool live = base + px < P;
  fft_stage_a<T2, +1, PX>(H, wt, lds, P, base, px, r, live);
  __syncthreads();
  double loss = 0.0;   // every thread stays for the workgroup's loss reduction
  if (r < T2 && live) {
    float2 b[16];
    fft_stage_b<T2, +1, PX>(lds, px, r, b);
#pragma unroll
    for (int q1 = 0; q1 < 16; ++q1) {
      const size_t idx = (size_t)(r + T2 * q1) * P + base + px;
      const double a2 = (double)b[q1].x * b[q1].x + (double)b[q1].y * b[q1].y;
      loss += a2 * a2;
      const float sx = b[q1].x * gamma_scale, sy = b[q1].y * gamma_scale;
      const float m2 = 4.0f * (sx * sx + sy * sy);
      out[idx] = make_float2(m2 * sx, m2 * sy);
    }
  }
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = loss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int i = 0; i < 16 * PX / 64; ++i) sum += red[i];
    loss_partials[blockIdx.x] = sum;
  }
}

// Depth-first order, stage 1: the depth DFT of the rescaled frames J_t (Eq. 5)
// before any spatial transform.  J_t is real, so G_q = sum_t J_t wT^(q t) is
// Hermitian in q and only bins q = 0..T/2 are written: G [T/2 + 1][N][N],
// pixels at FFT positions (m, n) of the Fresnel passes (row and column tables
// of frame t give the source position and weight of each position).
template <int T2, int PX>
__global__ __launch_bounds__(16 * PX) void k_rescale_dft(const uint16_t* __restrict__ frames,
                                                          const AxisTab* __restrict__ rows,
                                                          const AxisTab* __restrict__ cols,
                                                          const float2* __restrict__ wt, float2* __restrict__ G,
                                                          int N, int logN) {
  constexpr int T = 16 * T2;
  __shared__ float2 lds[T * PX];
  const int px = threadIdx.x % PX, r = threadIdx.x / PX;
  const size_t P = (size_t)N * N;
  const int pix = blockIdx.x * PX + px;               // P is a multiple of PX (N >= 16, PX <= 256)
  const int m = pix >> logN, n = pix & (N - 1);

  float2 a[T2];
#pragma unroll
  for (int t2 = 0; t2 < T2; ++t2) {
    const int t = r + 16 * t2;
    const AxisTab rt = rows[(size_t)t * N + m];
    const AxisTab ct = cols[(size_t)t * N + n];
    const uint16_t* I = frames + (size_t)t * P;
    const int y1 = rt.i0 + 1 < N ? rt.i0 + 1 : N - 1;
    const int x1 = ct.i0 + 1 < N ? ct.i0 + 1 : N - 1;
    const float a00 = I[(size_t)rt.i0 * N + ct.i0], a01 = I[(size_t)rt.i0 * N + x1];
    const float a10 = I[(size_t)y1 * N + ct.i0], a11 = I[(size_t)y1 * N + x1];
    const float ya = a00 + rt.f * (a10 - a00);        // lerp along y, then along x
    const float yb = a01 + rt.f * (a11 - a01);
    a[t2] = make_float2(ya + ct.f * (yb - ya), 0.f);
  }
  if constexpr (T2 > 1) dft_small<T2, -1>(a);
#pragma unroll
  for (int q2 = 0; q2 < T2; ++q2) lds[(q2 * 16 + r) * PX + px] = q2 == 0 ? a[q2] : cmul(a[q2], wt[(q2 * r) % T]);
  __syncthreads();
  if (r >= T2) return;
  float2 b[16];
#pragma unroll
  for (int t1 = 0; t1 < 16; ++t1) b[t1] = lds[(r * 16 + t1) * PX + px];
  dft16<-1>(b);
#pragma unroll
  for (int q1 = 0; q1 < 16; ++q1) {
    const int q = r + T2 * q1;
    if (2 * q <= T) st_once<SSOCT_DFFT_NT>(G + (size_t)q * P + pix, b[q1]);
  }
}

// Source position of FFT position i at frame scale s, exactly as the axis
// tables compute it: N/2 + c s in FP64 without contraction, floor, clamp.
__device__ __forceinline__ void src_pos(int i, int N, double s, int& i0, float& f) {
  const int half = N >> 1;
  const int c = ((i + half) & (N - 1)) - half;
  const double P = __dadd_rn(__dmul_rn((double)c, s), (double)half);
  const double p0 = floor(P);
  int k = (int)p0;
  k = k < 0 ? 0 : (k > N - 1 ? N - 1 : k);
  i0 = k;
  f = (float)(P - p0);
}

// The same transform for N >= 64, where a tile of PX = 32 FFT positions lies
// inside one row and one half of the centred order, so its source columns at
// frame t form a window.  The two source rows of every frame's window are
// interpolated along y once while they are staged (16-byte loads of 8
// samples, FP32 rows in LDS), so that each sample then takes two LDS reads
// and one interpolation along x; twiddles are staged in LDS.  The window of
// a 32-position tile at frame t starts at the first position's source
// column rounded down to 8 samples and spans 40 samples: the last position's
// right tap lies at most 7 + 31 + 1 samples past the start (s_t <= 1).
//
// The frames are real, so the transform is Hermitian in q and only bins
// 0..T/2 are kept; the same holds inside the split.  Stage A of thread t1 is
// a real T2-point DFT whose bins T2 - q2 are the conjugates of bins q2, so
// only rows q2 = 0..T2/2 are twiddled and cross LDS, and stage B runs the
// 16-point DFT of those T2/2 + 1 rows only.  Row q2 (0 < q2 < T2/2) yields
// bins q2 + T2 q1 directly for q1 <= 7 and, through
//   V[T - q] = conj V[q],  T - (q2 + T2 q1) = (T2 - q2) + T2 (15 - q1),
// bins (T2 - q2) + T2 (15 - q1) for q1 >= 8; row 0 yields bins T2 q1 for
// q1 <= 8 and row T2/2 bins T2/2 + T2 q1 for q1 <= 7.
template <int T2>
__global__ __launch_bounds__(512) void k_rescale_dft_win(const uint16_t* __restrict__ frames,
                                                         const double* __restrict__ params,
                                                         const float2* __restrict__ wt, float2* __restrict__ G,
                                                         int N, int logN) {
  constexpr int PX = 32;
  constexpr int T = 16 * T2;
  constexpr int NT = 16 * PX;                 // threads
  constexpr int WS = 40;                      // staged samples per frame (five chunks of 8)
  constexpr int NCH = WS / 8;
  constexpr int NITEM = T * NCH;              // (frame, chunk) staging items
  constexpr int NI = (NITEM + NT - 1) / NT;
  constexpr int STRIDE = ParamLayout::PER_FRAME;   // doubles per frame in the parameter block (s_t first)
  constexpr int NROW = T2 / 2 + 1;            // rows of stage A that cross LDS
  constexpr int LDSN = (T * WS / 2 > NROW * 16 * PX) ? T * WS / 2 : NROW * 16 * PX;
  // one block in declaration order: the per-frame values first, so that
  // their addresses fit the 16-bit offset field of the LDS instructions
  struct Lds {
    double fs[T];             // per frame: s_t
    double fp[T];             // per frame: position of the tile's first column, relative to the window start
    int frow[T];              // per frame: source row y0
    int fxs[T];               // per frame: window start (first column rounded down to 8 samples)
    float ffy[T];             // per frame: y weight
    float2 tws[T];            // exp(-2 pi i k / T)
    float2 lds[LDSN];         // transposition [q2][t1][px], rows q2 = 0..T2/2; the staged rows alias it
  };
  __shared__ Lds sm;
  float* ya = reinterpret_cast<float*>(sm.lds);  // [T][WS]
  const int tid = threadIdx.x;
  const int px = tid % PX, r = tid / PX;
  // element offsets fit 32 bits (T N^2 <= 2^30 for the T this form takes)
  const uint32_t P = (uint32_t)N * (uint32_t)N;
  // contiguous runs of tiles per XCD (workgroups are dispatched round-robin
  // over the XCDs), so that neighbouring rows, which share source rows, meet in one L2
  const int tile = (gridDim.x % SSOCT_XCDS == 0)
                       ? (blockIdx.x % SSOCT_XCDS) * (gridDim.x / SSOCT_XCDS) + blockIdx.x / SSOCT_XCDS
                       : blockIdx.x;
  const int pix0 = tile * PX;
  const int m = pix0 >> logN, n0 = pix0 & (N - 1);
  const int half = N >> 1;
  const int c0 = ((n0 + half) & (N - 1)) - half;   // centred index of the first column (same half as the tile)
  for (int t = tid; t < T; t += NT) {
    const double st = params[(size_t)STRIDE * t];
    int y0, x0;
    float fy, fx;
    src_pos(m, N, st, y0, fy);
    src_pos(n0, N, st, x0, fx);
    // the window start xs is an integer within 8 samples of N/2 + c0 s_t: the
    // difference is exact in FP64, so positions are taken relative to it
    const int xs = x0 & ~7;
    sm.fs[t] = st;
    sm.fp[t] = __dadd_rn(__dmul_rn((double)c0, st), (double)half) - (double)xs;
    sm.frow[t] = y0;
    sm.ffy[t] = fy;
    sm.fxs[t] = xs;
    sm.tws[t] = wt[t];
  }
  __syncthreads();
  // every staging load is in flight before the first interpolation.  A chunk
  // starting at or past column N (x and N are multiples of 8) only feeds the
  // right tap of the last column, whose weight is exactly 0: it is read from
  // the frame's last chunk instead, any finite value giving the same sample.
  uint4 ra[NI], rb[NI];
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    const int i = tid + k * NT;
    if (i < NITEM) {
      const int t = i / NCH, c = i - (i / NCH) * NCH;
      int x = sm.fxs[t] + 8 * c;
      x = x < N ? x : N - 8;
      const int y0 = sm.frow[t];
      const int y1 = y0 + 1 < N ? y0 + 1 : N - 1;
      const uint32_t row0 = ((uint32_t)t * (uint32_t)N + (uint32_t)y0) * (uint32_t)N + (uint32_t)x;
      const uint32_t row1 = row0 + (uint32_t)(y1 - y0) * (uint32_t)N;
      ra[k] = *reinterpret_cast<const uint4*>(frames + row0);
      rb[k] = *reinterpret_cast<const uint4*>(frames + row1);
    }
  }
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    const int i = tid + k * NT;
    if (i < NITEM) {
      const int t = i / NCH, c = i - (i / NCH) * NCH;
      const float fy = sm.ffy[t];
      const uint32_t wa[4] = {ra[k].x, ra[k].y, ra[k].z, ra[k].w};
      const uint32_t wb[4] = {rb[k].x, rb[k].y, rb[k].z, rb[k].w};
      float o[8];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const float a0 = (float)(wa[h] & 0xffffu), a1 = (float)(wa[h] >> 16);
        const float b0 = (float)(wb[h] & 0xffffu), b1 = (float)(wb[h] >> 16);
        o[2 * h] = a0 + fy * (b0 - a0);            // lerp along y (then along x below)
        o[2 * h + 1] = a1 + fy * (b1 - a1);
      }
      float4* dst = reinterpret_cast<float4*>(ya + t * WS + 8 * c);
      dst[0] = make_float4(o[0], o[1], o[2], o[3]);
      dst[1] = make_float4(o[4], o[5], o[6], o[7]);
    }
  }
  __syncthreads();
  float2 a[T2];
  const double dpx = (double)px;
#pragma unroll
  for (int t2 = 0; t2 < T2; ++t2) {
    const int t = r + 16 * t2;
    // N/2 + (c0 + px) s_t - xs = fp[t] + px s_t up to FP64 rounding; column and weight as in the tables
    const double Pd = fma(dpx, sm.fs[t], sm.fp[t]);
    const double p0 = floor(Pd);
    const float fx = (float)(Pd - p0);
    const float* w = ya + t * WS + (int)p0;
    const float y0 = w[0], y1 = w[1];
    a[t2] = make_float2(y0 + fx * (y1 - y0), 0.f);
  }
  __syncthreads();   // staged rows read before the transposition buffer is written
  if constexpr (T2 > 1) dft_small<T2, -1>(a);
  float2* tr = sm.lds + r * PX + px;
#pragma unroll
  for (int q2 = 0; q2 < NROW; ++q2)
    tr[q2 * 16 * PX] = q2 == 0 ? make_float2(a[0].x, 0.f) : cmul(a[q2], sm.tws[(q2 * r) & (T - 1)]);
  __syncthreads();
  if (r >= NROW) return;
  float2 b[16];
  const float2* tb = sm.lds + r * 16 * PX + px;
#pragma unroll
  for (int t1 = 0; t1 < 16; ++t1) b[t1] = tb[t1 * PX];
  dft16<-1>(b);
  // row r: bins r + T2 q1 (q1 <= 7, and q1 = 8 on row 0); rows strictly
  // between 0 and T2/2 also give the conjugate bins (T2 - r) + T2 (15 - q1)
  const bool mirror = r > 0 && 2 * r < T2;
  float2* gdir = G + ((uint32_t)r * P + (uint32_t)(pix0 + px));
  float2* gmir = G + ((uint32_t)(T2 - r) * P + (uint32_t)(pix0 + px));
#pragma unroll
  for (int q1 = 0; q1 < 16; ++q1) {
    if (q1 < 8) {
      st_once<SSOCT_DFFT_NT>(gdir + (uint32_t)(T2 * q1) * P, b[q1]);
    } else {
      if (q1 == 8 && r == 0) st_once<SSOCT_DFFT_NT>(gdir + (uint32_t)(T2 * 8) * P, b[8]);
      if (mirror) st_once<SSOCT_DFFT_NT>(gmir + (uint32_t)(T2 * (15 - q1)) * P, cconj(b[q1]));
    }
  }
}

template <int T2>
static hipError_t rescale_dft_t(int N, const uint16_t* frames, const AxisTab* rows, const AxisTab* cols,
                                const double* params, const float2* wt, float2* G, hipStream_t s) {
  int logN = 0;
  while ((1 << logN) < N) ++logN;
  const size_t P = (size_t)N * N;
  if (N >= 64) {
    hipLaunchKernelGGL((k_rescale_dft_win<T2>), dim3((unsigned)(P / 32)), dim3(512), 0, s, frames, params, wt, G, N,
                       logN);
  } else {
    constexpr int PX = SSOCT_DFFT_PX;
    hipLaunchKernelGGL((k_rescale_dft<T2, PX>), dim3((unsigned)(P / PX)), dim3(16 * PX), 0, s, frames, rows, cols,
                       wt, G, N, logN);
  }
  return hipGetLastError();
}

hipError_t launch_rescale_dft(int T, int N, const uint16_t* frames, const AxisTab* rows, const AxisTab* cols,
                              const double* params, const float2* wt, float2* G, hipStream_t s) {
  if ((size_t)N * N % SSOCT_DFFT_PX != 0) return hipErrorInvalidValue;
  switch (T) {
    case 16: return rescale_dft_t<1>(N, frames, rows, cols, params, wt, G, s);
    case 32: return rescale_dft_t<2>(N, frames, rows, cols, params, wt, G, s);
    case 64: return rescale_dft_t<4>(N, frames, rows, cols, params, wt, G, s);
    case 128: return rescale_dft_t<8>(N, frames, rows, cols, params, wt, G, s);
    case 256: return rescale_dft_t<16>(N, frames, rows, cols, params, wt, G, s);
    default: return hipErrorInvalidValue;
  }
}

template <int T2, int DIR, int EPI, int PX>
static hipError_t depth_fft_px(int P, const float2* H, const float2* wt, void* out, int shift, int grid,
                               hipStream_t s) {
  const int ntiles = (P + PX - 1) / PX;
  const int g = grid > 0 && grid < ntiles ? grid : ntiles;
  hipLaunchKernelGGL((k_depth_fft<T2, DIR, EPI, PX>), dim3(g), dim3(16 * PX), 0, s, H, wt, out, P, shift);
  return hipGetLastError();
}

// px: pixels per workgroup of the forward store/|V| transform (16, 32 or 64,
// a tuning choice; anything else takes SSOCT_DFFT_PX)
template <int T2, int DIR, int EPI>
static hipError_t depth_fft_t(int P, const float2* H, const float2* wt, void* out, int shift, float gs,
                              double* partials, int grid, int px, hipStream_t s) {
  constexpr int PX = SSOCT_DFFT_PX;
  if constexpr (EPI == EPI_GAMMA) {
    const int ntiles = (P + PX - 1) / PX;
    hipLaunchKernelGGL((k_depth_fft_gamma<T2, PX>), dim3(ntiles), dim3(16 * PX), 0, s, H, wt,
                       static_cast<float2*>(out), P, gs, partials);
    return hipGetLastError();
  } else if constexpr (DIR > 0) {
    if (px == 16 && PX != 16) return depth_fft_px<T2, DIR, EPI, 16>(P, H, wt, out, shift, grid, s);
    if (px == 64 && PX != 64) return depth_fft_px<T2, DIR, EPI, 64>(P, H, wt, out, shift, grid, s);
    if (px == 32 && PX != 32) return depth_fft_px<T2, DIR, EPI, 32>(P, H, wt, out, shift, grid, s);
  }
  return depth_fft_px<T2, DIR, EPI, PX>(P, H, wt, out, shift, grid, s);
}

template <int DIR, int EPI>
static hipError_t depth_fft_d(int T, int P, const float2* H, const float2* wt, void* out, int shift, float gs,
                              double* partials, int grid, int px, hipStream_t s) {
  switch (T) {
    case 16: return depth_fft_t<1, DIR, EPI>(P, H, wt, out, shift, gs, partials, grid, px, s);
    case 32: return depth_fft_t<2, DIR, EPI>(P, H, wt, out, shift, gs, partials, grid, px, s);
    case 64: return depth_fft_t<4, DIR, EPI>(P, H, wt, out, shift, gs, partials, grid, px, s);
    case 128: return depth_fft_t<8, DIR, EPI>(P, H, wt, out, shift, gs, partials, grid, px, s);
    case 256: return depth_fft_t<16, DIR, EPI>(P, H, wt, out, shift, gs, partials, grid, px, s);
    default: return hipErrorInvalidValue;
  }
}

bool depth_fft_supported(int T) { return T == 16 || T == 32 || T == 64 || T == 128 || T == 256; }

int depth_fft_blocks(int P) { return (P + SSOCT_DFFT_PX - 1) / SSOCT_DFFT_PX; }

int depth_fft_grid(int cu_count) { return SSOCT_DFFT_WGCU > 0 ? SSOCT_DFFT_WGCU * cu_count : 0; }

hipError_t launch_depth_fft(int T, int P, int dir, int epi, const float2* H, const float2* wt, void* out,
                            hipStream_t s, int shift, int gamma_exp, double* partials, int grid, int px) {
  if (P <= 0) return hipSuccess;
  if (shift < 0 || shift >= T) return hipErrorInvalidValue;
  if (dir > 0) {
    if (epi == EPI_ABS) return depth_fft_d<+1, EPI_ABS>(T, P, H, wt, out, shift, 1.f, nullptr, grid, px, s);
    if (epi == EPI_GAMMA) {
      if (!partials || shift != 0) return hipErrorInvalidValue;
      return depth_fft_d<+1, EPI_GAMMA>(T, P, H, wt, out, 0, ldexpf(1.0f, -gamma_exp), partials, 0, 0, s);
    }
    return depth_fft_d<+1, EPI_STORE>(T, P, H, wt, out, shift, 1.f, nullptr, grid, px, s);
  }
  if (epi != EPI_STORE || shift != 0) return hipErrorInvalidValue;
  return depth_fft_d<-1, EPI_STORE>(T, P, H, wt, out, 0, 1.f, nullptr, grid, 0, s);
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
