// Register/LDS Stockham FFT engine for gfx950 (wave64).
//
// One FFT of size N (power of two, 16..2048) is computed by a group of
// G = N/16 threads; every thread holds 16 complex values in registers.
// Passes are radix-16 while 16 divides the remaining length, then one pass of
// radix 2, 4 or 8.  Between passes the data moves through LDS in the
// self-sorting (Stockham) order, so input and output are both in natural
// order and no bit reversal is needed.
//
// Direction DIR = +1 computes X[k] = sum_n x[n] exp(+2 pi i n k / N), the
// kernel of the Fresnel transform (Eq. 6 expanded, positive exponent);
// DIR = -1 is its adjoint.
//
// Register convention shared by every kernel that uses the engine:
//   input : v[k] = x[j + k G]                      (k = 0..15)
//   output: v[e] = X[j + out_offset<N, PL>(e)]     (e = 0..15)
// so for every register slot the G threads of a group touch G consecutive
// elements (coalesced global loads and stores).
//
// Radix order PL: 0 runs the radix-16 passes first and the small radix
// (2, 4 or 8) last (16 16 4 at N = 1024); 1 runs the small radix first
// (4 16 16), which puts the output in the input's order (out_offset = e G)
// at the price of twiddles on every radix-16 pass.  Both are Stockham
// passes of the same DFT; they differ in rounding only.  Sizes that are a
// power of 16 have one order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssoct {

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// multiply by DIR * i
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
  return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by exp(DIR * i * theta) with cos = c, sin = s (compile-time constants)
template <int DIR>
__device__ __forceinline__ float2 rot(float2 a, float c, float s) {
  const float sd = DIR > 0 ? s : -s;
  return make_float2(a.x * c - a.y * sd, a.y * c + a.x * sd);
}
// exp(DIR i pi/4) and exp(DIR i 3pi/4)
template <int DIR>
__device__ __forceinline__ float2 rot8_1(float2 a) {
  const float h = 0.70710678118654752440f;
  return DIR > 0 ? make_float2((a.x - a.y) * h, (a.y + a.x) * h) : make_float2((a.x + a.y) * h, (a.y - a.x) * h);
}
template <int DIR>
__device__ __forceinline__ float2 rot8_3(float2 a) {
  const float h = 0.70710678118654752440f;
  return DIR > 0 ? make_float2((-a.x - a.y) * h, (a.x - a.y) * h) : make_float2((a.y - a.x) * h, (-a.y - a.x) * h);
}

// ---------------------------------------------------------------- small DFTs (natural order out)
template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
  float2 a2 = cadd(x1, x3), a3 = mul_i<DIR>(csub(x1, x3));
  x0 = cadd(a0, a2);
  x2 = csub(a0, a2);
  x1 = cadd(a1, a3);
  x3 = csub(a1, a3);
}

// 8 = 2 x 4: n = n2 + 2 n1, k = k1 + 4 k2
template <int DIR>
__device__ __forceinline__ void dft8(float2* v) {
  dft4<DIR>(v[0], v[2], v[4], v[6]);
  dft4<DIR>(v[1], v[3], v[5], v[7]);
  v[3] = rot8_1<DIR>(v[3]);
  v[5] = mul_i<DIR>(v[5]);
  v[7] = rot8_3<DIR>(v[7]);
  float2 X[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    X[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
    X[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = X[k];
}

// 16 = 4 x 4: n = n2 + 4 n1, k = k1 + 4 k2
template <int DIR>
__device__ __forceinline__ void dft16(float2* v) {
  const float c1 = 0.92387953251128675613f;  // cos(pi/8)
  const float s1 = 0.38268343236508977173f;  // sin(pi/8)
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<DIR>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
  // Y[n2][k1] sits in v[n2 + 4 k1]; twiddle exp(DIR 2 pi i n2 k1 / 16)
  v[1 + 4] = rot<DIR>(v[1 + 4], c1, s1);       // e = 1
  v[1 + 8] = rot8_1<DIR>(v[1 + 8]);            // e = 2
  v[1 + 12] = rot<DIR>(v[1 + 12], s1, c1);     // e = 3
  v[2 + 4] = rot8_1<DIR>(v[2 + 4]);            // e = 2
  v[2 + 8] = mul_i<DIR>(v[2 + 8]);             // e = 4
  v[2 + 12] = rot8_3<DIR>(v[2 + 12]);          // e = 6
  v[3 + 4] = rot<DIR>(v[3 + 4], s1, c1);       // e = 3
  v[3 + 8] = rot8_3<DIR>(v[3 + 8]);            // e = 6
  v[3 + 12] = rot<DIR>(v[3 + 12], -c1, -s1);   // e = 9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<DIR>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // X[k1 + 4 k2] sits in v[4 k1 + k2]
  float2 X[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) X[k] = v[4 * (k & 3) + (k >> 2)];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = X[k];
}

template <int R, int DIR>
__device__ __forceinline__ void dft_small(float2* v) {
  if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
  else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<DIR>(v);
  else dft16<DIR>(v);
}

// ---------------------------------------------------------------- plan (compile time)
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

template <int N>
struct FFTShape {
  static_assert(N >= 16 && N <= 2048 && (N & (N - 1)) == 0, "N must be a power of two in [16, 2048]");
  static constexpr int G = N / 16;                         // threads per FFT
  static constexpr int LOG = ilog2(N);
  static constexpr int P16 = LOG / 4;                      // radix-16 passes
  static constexpr int L = N >> (4 * P16);                 // last radix (1 = none)
  static constexpr int LDS = N + (N >> 4);                 // padded complex slots per FFT
};

// LDS slot of element i (one pad slot every 16 keeps stride-16 writes conflict-free)
__device__ __forceinline__ constexpr int lds_slot(int i) { return i + (i >> 4); }
// slot(a + b) = slot(a) + slot(b) whenever (a mod 16) + (b mod 16) < 16.  Every
// exchange index below is split that way into a per-thread part and a
// compile-time part, so that the LDS accesses of a thread share one base
// address and take immediate offsets (the condition is noted at each use).

// output register e of thread j holds element j + out_offset<N, PL>(e)
template <int N, int PL = 0>
__device__ __forceinline__ constexpr int out_offset(int e) {
  using S = FFTShape<N>;
  if constexpr (S::L == 1 || PL == 1) {
    return e * S::G;
  } else {
    return S::G * (e / S::L) + (e % S::L) * (N / S::L);
  }
}

// Per-thread twiddle table.  For every pass that needs twiddles, thread j of
// a group reads E consecutive entries (one base address, immediate offsets):
//   radix-16 pass p >= 1 (Ns = 16^p): entry r-1 = exp(+2 pi i s r / N),
//       s = (j mod Ns) N / (16 Ns), r = 1..15
//   final radix-L pass (Ns = N/L):   entry i (L-1) + k-1 = exp(+2 pi i b k / N),
//       b = j + G i, i = 0..16/L-1, k = 1..L-1
// With the small radix first (PL = 1) every radix-16 pass p = 0..P16-1 has
// twiddles (Ns = L 16^p), entry r-1 of thread j at off16(p) + 15 j, and
// there is no radix-L table.
// The table is built in FP64 on the GPU (tables.hip) from this same layout.
template <int N, int PL = 0>
struct TwPlan {
  using S = FFTShape<N>;
  static constexpr bool SMALL_FIRST = PL == 1 && S::L > 1;
  static constexpr int G = S::G;
  static constexpr int E16 = 15;
  static constexpr int NB = S::L > 1 ? 16 / S::L : 0;
  static constexpr int EL = S::L > 1 && !SMALL_FIRST ? NB * (S::L - 1) : 0;
  static constexpr int OFF_L = (SMALL_FIRST ? S::P16 : S::P16 - 1) * G * E16;
  static constexpr int SIZE = OFF_L + G * EL;
  static constexpr int off16(int p) { return (SMALL_FIRST ? p : p - 1) * G * E16; }
};

template <int DIR>
__device__ __forceinline__ float2 tw_dir(float2 w) {
  return DIR > 0 ? w : cconj(w);
}

// Barrier between LDS writes and reads of one exchange.  A group that lives
// inside one wavefront (G <= 64) only needs its own LDS accesses ordered:
// the LDS unit executes the instructions of a wave in order, so a compiler
// fence at wavefront scope is enough.  Larger groups use the workgroup
// barrier.
template <bool WAVE>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Twiddle sources of fft_group.  TwMem reads the table of TwPlan for thread
// j at every use; TwRegs holds the same entries in registers, loaded once by
// a kernel that runs many transforms per thread, so that its loads can be
// completed before the transform loop starts.
template <int N, int PL = 0>
struct TwMem {
  static constexpr int PLAN = PL;
  const float2* __restrict__ tw;
  int j;
  __device__ __forceinline__ float2 w16(int p, int r) const {
    return tw[TwPlan<N, PL>::off16(p) + j * TwPlan<N, PL>::E16 + r - 1];
  }
  __device__ __forceinline__ float2 wl(int i) const {
    return tw[TwPlan<N, PL>::OFF_L + j * TwPlan<N, PL>::EL + i];
  }
};

template <int N>
struct TwRegs {
  static constexpr int PLAN = 0;
  using S = FFTShape<N>;
  static constexpr int P = S::P16 > 1 ? S::P16 - 1 : 1;
  static constexpr int E = TwPlan<N>::EL > 0 ? TwPlan<N>::EL : 1;
  float2 a[P][15];
  float2 b[E];
  __device__ __forceinline__ float2 w16(int p, int r) const { return a[p - 1][r - 1]; }
  __device__ __forceinline__ float2 wl(int i) const { return b[i]; }
};

template <int N>
__device__ __forceinline__ TwRegs<N> load_tw_regs(const float2* __restrict__ tw, int j) {
  using S = FFTShape<N>;
  TwRegs<N> t;
  const TwMem<N> m{tw, j};
#pragma unroll
  for (int p = 1; p < S::P16; ++p) {
#pragma unroll
    for (int r = 1; r < 16; ++r) t.a[p - 1][r - 1] = m.w16(p, r);
  }
  if constexpr (S::L > 1 && S::P16 > 0) {
#pragma unroll
    for (int i = 0; i < TwPlan<N>::EL; ++i) t.b[i] = m.wl(i);
  }
  return t;
}

// Full N-point FFT of one group.  `lds` points to this group's LDS region of
// FFTShape<N>::LDS complex slots with element stride LS (1 for row FFTs, C
// for a C-column tile; a compile-time constant so that every LDS address is a
// base plus an immediate offset).  With WAVE = false every thread of the
// workgroup must call this the same number of times (workgroup barriers).
// `tws` is a twiddle source (TwMem or TwRegs) for this thread.
//
// The twiddle source's PLAN picks the radix order; with the small radix
// first, butterfly b = j + G i (i < 16/L) of the first pass takes elements
// b + k N/L, which thread j holds in registers i + k 16/L.
template <int N, int DIR, int LS, bool WAVE, class TW>
__device__ __forceinline__ void fft_group_tw(float2 (&v)[16], int j, float2* lds, const TW& tws) {
  constexpr int ls = LS;
  using S = FFTShape<N>;
  constexpr int G = S::G;
  // Exchange addresses (see lds_slot).  write_slots: base = (j / Ns) 16 Ns +
  // j mod Ns has base mod 16 = j mod Ns < Ns when Ns < 16 (Ns divides 16, so
  // k Ns mod 16 <= 16 - Ns), and k Ns mod 16 = 0 otherwise.  read_slots:
  // j + k G (and the last pass's j + G (i + k 16/L)) with j < G: G >= 16
  // gives k G mod 16 = 0, and G < 16 (a divisor of 16) gives j < G and
  // k G mod 16 <= 16 - G.
  const int sj = lds_slot(j);
  if constexpr (TwPlan<N, TW::PLAN>::SMALL_FIRST) {
    constexpr int L = S::L;
    constexpr int NB = 16 / L;
    // Ns = 1: output k of butterfly b goes to b L + k.  Its address
    // (j + G i) L + k = L j + (L G i + k): L j mod 16 is a multiple of L, at
    // most L (G - 1) when L G < 16 (else 16 - L), and L G i mod 16 + k at
    // most 16 - L G + L - 1 (else L - 1), so the sums stay below 16.
    exchange_sync<WAVE>();  // previous reads of this region are complete
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      float2 u[L];
#pragma unroll
      for (int k = 0; k < L; ++k) u[k] = v[i + k * NB];
      dft_small<L, DIR>(u);
#pragma unroll
      for (int k = 0; k < L; ++k) lds[(lds_slot(L * j) + lds_slot(L * G * i + k)) * ls] = u[k];
    }
    exchange_sync<WAVE>();
    int Ns = L;
#pragma unroll
    for (int p = 0; p < S::P16; ++p) {
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = lds[(sj + lds_slot(k * G)) * ls];   // see read_slots
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tw_dir<DIR>(tws.w16(p, r)));
      dft16<DIR>(v);
      if (p < S::P16 - 1) {
        const int sb = lds_slot((j / Ns) * Ns * 16 + (j % Ns));
        exchange_sync<WAVE>();
#pragma unroll
        for (int k = 0; k < 16; ++k) lds[(sb + lds_slot(k * Ns)) * ls] = v[k];   // see write_slots
        exchange_sync<WAVE>();
        Ns *= 16;
      }
    }
    // the last pass has Ns = G: output k of thread j is element j + k G
    return;
  }
  int Ns = 1;
#pragma unroll
  for (int p = 0; p < S::P16; ++p) {
    if (p > 0) {
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tw_dir<DIR>(tws.w16(p, r)));
    }
    dft16<DIR>(v);
    const bool last = (p == S::P16 - 1) && (S::L == 1);
    if (!last) {
      const int sb = lds_slot((j / Ns) * Ns * 16 + (j % Ns));
      exchange_sync<WAVE>();  // previous reads of this region are complete
#pragma unroll
      for (int k = 0; k < 16; ++k) lds[(sb + lds_slot(k * Ns)) * ls] = v[k];
      exchange_sync<WAVE>();
      Ns *= 16;
      if constexpr (S::L == 1) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = lds[(sj + lds_slot(k * G)) * ls];
      } else {
        if (p < S::P16 - 1) {
#pragma unroll
          for (int k = 0; k < 16; ++k) v[k] = lds[(sj + lds_slot(k * G)) * ls];
        }
      }
    }
  }
  if constexpr (S::L > 1) {
    constexpr int L = S::L;
    constexpr int NB = 16 / L;  // butterflies per thread
    // Ns == N / L here; butterfly b = j + G i reads x[b + k N/L]
#pragma unroll
    for (int i = 0; i < NB; ++i) {
#pragma unroll
      for (int k = 0; k < L; ++k) v[i * L + k] = lds[(sj + lds_slot(G * i + k * (N / L))) * ls];
    }
    if constexpr (S::P16 > 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
#pragma unroll
        for (int k = 1; k < L; ++k) v[i * L + k] = cmul(v[i * L + k], tw_dir<DIR>(tws.wl(i * (L - 1) + k - 1)));
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) dft_small<L, DIR>(&v[i * L]);
  }
}

// The same with the twiddles read from the table at every use
template <int N, int DIR, int LS, bool WAVE = false>
__device__ __forceinline__ void fft_group(float2 (&v)[16], int j, float2* lds, const float2* __restrict__ tw) {
  fft_group_tw<N, DIR, LS, WAVE>(v, j, lds, TwMem<N>{tw, j});
}

}  // namespace ssoct
