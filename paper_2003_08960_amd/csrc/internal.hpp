// Internal interfaces between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ssoct {

// Per (frame, FFT position) entry of the rescale/chirp tables.  FFT position i
// holds the original sample i' = (i + N/2) mod N (the input half-swap that,
// with the (-1)^i' sign folded into `fac`, turns the centred DFT of Eq. 6 into
// a plain DFT).  `i0`, `f`: bilinear source index and weight of Eq. 5;
// `fac`: (-1)^i' exp(-i alpha_t c^2) (times exp(i phi_t) and the Eq. 6
// prefactor for the row table).
struct __align__(16) AxisTab {
  int i0;
  float f;
  float2 fac;
};

// Storage of the hologram stack H[t][pixel] between the Fresnel stage and the
// depth transform.  All formats use 8 bytes per complex pixel.
enum HFormat : int {
  HF_F32 = 0,   // float2 (re, im)
  HF_F16 = 1,   // 4 x fp16: re_hi, re_lo, im_hi, im_lo, scaled by 2^-sigma
  HF_BF16 = 2,  // 4 x bf16: re_hi, re_lo, im_hi, im_lo
};

// Depth-transform operand precision.
enum DepthPrec : int {
  DP_F32 = 0,
  DP_F16 = 1,
  DP_BF16 = 2,
  DP_F16_SPLIT = 3,
  DP_BF16_SPLIT = 4,
};

// Epilogue of the depth transform.
enum DepthEpi : int {
  EPI_STORE = 0,      // complex volume V[q][pixel]
  EPI_ABS = 1,        // |V| as float
  EPI_GAMMA = 2,      // Gamma^ = 4 |V^|^2 V^ with V^ = 2^-e V, plus FP64 partials of sum |V|^4
};

// Per-frame scalar parameters in device memory (FP64), 4 doubles per frame
// followed by globals; filled on the host, consumed by the table kernels.
struct ParamLayout {
  static constexpr int PER_FRAME = 4;  // s_t, kappa_t (cycles per c^2), row phase (cycles), row amplitude
  __host__ __device__ static size_t globals(int T) { return (size_t)PER_FRAME * T; }
  // globals: [0] kappa_out (cycles per c^2, Eq. 6 output phase), [1..15] aberration polynomial
  //          coefficients (rad) in monomial order, [16] aberration flag
  static constexpr int G_KAPPA_OUT = 0;
  static constexpr int G_POLY = 1;
  static constexpr int G_HAS_ABERR = 16;
  static constexpr int N_GLOBALS = 17;
  __host__ __device__ static size_t count(int T) { return globals(T) + N_GLOBALS; }
};

// Monomial order used for aberration phases and gradient moments: x^a y^b with
// (a, b) = (0,0) (1,0) (0,1) (2,0) (1,1) (0,2) (3,0) (2,1) (1,2) (0,3)
//          (4,0) (3,1) (2,2) (1,3) (0,4)
constexpr int N_MONO = 15;

struct DepthLayout {
  int T;        // frames
  int KC;       // frames per K chunk (32, 64, 128 or 256)
  int T_pad;    // T rounded up to KC
  int rows;     // real rows of the depth matrix (T, or T + 1 for odd T)
  int M_pad;    // rows rounded up to 32
  int nrb;      // row blocks of 32
  int waves;    // waves per workgroup (row blocks per slab, <= 8)
  int slabs;    // ceil(nrb / waves)
};
DepthLayout depth_layout(int T, bool general = false);   // general: 2T rows (sweeps not linear in k)

// ---------------------------------------------------------------- launchers
hipError_t launch_axis_tables(const double* params, int T, int N, AxisTab* rows, AxisTab* cols,
                              hipStream_t s);
// Aberration screen as per-row polynomials: row m (FFT position) holds, at
// apoly[m * APOLY_STRIDE + a], the FP32 coefficient (cycles) of x^a, a = 0..4,
// of the phase sum_k c_k Z_k at x = centred original column * sqrt 2 / N.
constexpr int APOLY_STRIDE = 8;
hipError_t launch_misc_tables(const double* params, int T, int N, float2* outfac, float* apoly, hipStream_t s);
// The same screen as N x N complex factors (FP64 phases), for the adjoint row pass
hipError_t launch_aberr_screen(const double* params, int T, int N, float2* screen, hipStream_t s);
// FFT engine twiddles (per-thread layout of radix order pl: 0 = radix-16
// passes first, 1 = the small radix first), FP64 -> FP32; size in float2 entries
hipError_t launch_twiddles(int N, float2* tw, hipStream_t s, int pl = 0);
size_t twiddle_table_size(int N, int pl = 0);
// N has a second radix order (N is not a power of 16)
inline bool has_radix_orders(int N) { return N != 16 && N != 256; }
// kappa == nullptr: DFT matrix (paired real form); else the general matrix exp(-2 pi i q kappa_t / T)
hipError_t launch_depth_tables(int T, const double* kappa, float* a_f32, uint4* a_f16, uint4* a_bf16,
                               hipStream_t s);

// Forward Fresnel stage on frames [t0, t0 + F): rescale + chirp + row DFT into
// `inter` ([F][N][N] complex64), then column DFT into H (format `fmt`).
hipError_t launch_row_pass(int N, int F, int t0, const uint16_t* frames, const AxisTab* rows,
                           const AxisTab* cols, const float2* tw, const float* apoly,
                           const float2* outfac, float2* inter, hipStream_t s);
// ctile: column tile width (0 = default; col_tiles lists the choices; the
// Eq. 6 output phase takes the default); radix: radix order of the column
// transforms (0 or 1, tw the table of that order)
hipError_t launch_col_pass(int N, int F, int t0, const float2* inter, const float2* tw,
                           const float2* outfac, void* H, int fmt, int sigma, int grid, hipStream_t s,
                           int ctile = 0, int radix = 0);
// Default persistent grid of the column passes (forward, adjoint, volume
// output) on a device with `cu` compute units, for column tile width ct (0 = default)
int col_default_grid(int N, int cu, int ct = 0);
// Column tile widths of the Fresnel column passes: out[0] the default, out[1]
// and out[2] the narrower alternatives (0 where N has none)
void col_tiles(int N, int* out);
// Default persistent grid of the angular-spectrum column pass (a host query
// of the kernel's residency: call it outside stream capture)
int as_col_default_grid(int N, int cu);

// Angular-spectrum propagation of frames [t0, t0 + F) into H (format fmt):
// row DFT^-, column DFT^- x transfer function x DFT^+, row DFT^+ (uncentred,
// natural pixel order).  asp: per frame {1/lambda^2, phase offset (cycles),
// amplitude (gate / N^2)}; inv_nd = 1 / (N pitch).
hipError_t launch_as_stage(int N, int F, int t0, const uint16_t* frames, const float2* tw, const double* asp,
                           double inv_nd, double z, float2* inter, void* H, int fmt, int sigma, int grid,
                           hipStream_t s);

// Depth-first order (frame-independent chirp, no per-frame phase):
// G [T/2 + 1][N][N] = depth DFT of the rescaled frames (stage 1); then per
// chunk of nb bins from qa: row DFTs of fac G_q and fac conj(G_q) into
// inter[f] and inter[Fh + f], and column DFTs of a chunk into the volume,
// frame f of the chunk at V + f fstride N^2.
hipError_t launch_rescale_dft(int T, int N, const uint16_t* frames, const AxisTab* rows, const AxisTab* cols,
                              const double* params, const float2* wt, float2* G, hipStream_t s);
// rpg: rows per row group (8, 4 or 2; anything else picks by the launch size on `cu` CUs)
hipError_t launch_row_pass_g(int N, int nb, int qa, int T, const float2* G, const AxisTab* rows0,
                             const AxisTab* cols0, const float2* tw, const float* apoly, const float2* outfac,
                             float2* inter, int Fh, int rpg, int cu, hipStream_t s);
// F2 > 0 adds a second run of F2 transforms in the same launch: from inter2
// (consecutive frames) to V2 + i fstride2 N^2
hipError_t launch_col_pass_v(int N, int F, const float2* inter, const float2* tw, const float2* outfac, float2* V,
                             int fstride, int grid, int ctile, hipStream_t s, int F2 = 0,
                             const float2* inter2 = nullptr, float2* V2 = nullptr, int fstride2 = 0,
                             int radix = 0);

// Adjoint Fresnel stage: column DFT^- of B[t0 .. t0+F) ([T][N][N] complex64)
// into `inter`, then row DFT^- fused with the recomputed row input and the
// per-frame FP64 moments of Im(conj(g) z) (partials [T][nblk][N_MONO]).
hipError_t launch_col_pass_adj(int N, int F, int t0, const float2* B, const float2* tw,
                               float2* inter, int grid, hipStream_t s);
hipError_t launch_row_pass_adj(int N, int F, int t0, const uint16_t* frames, const AxisTab* rows,
                               const AxisTab* cols, const float2* tw, const float2* screen,
                               const float2* inter, double* partials, hipStream_t s);
int row_adj_blocks(int N);

// Depth transform over the whole stack: out[q][p] = sum_t W[q][t] in[t][p]
// (dir = +1) or sum_t conj(W[q][t]) in[t][p] (dir = -1).
// shift > 0 (forward, EPI_STORE): the stack is a ring whose window starts at
// slot `shift`; bin q is multiplied by exp(+2 pi i q shift / T) = conj(wt[q shift mod T]).
// kc: frames per K chunk (0 = the layout's; else a divisor of it, at least 32)
hipError_t launch_depth(int T, int P, int prec, int dir, int epi, const void* in, const void* amat,
                        void* out, int sigma, int gamma_exp, double* partials, int grid,
                        hipStream_t s, const float2* wt = nullptr, int shift = 0, bool general = false, int kc = 0);
int depth_grid(int T, int P, int cu_count, bool general = false);

// Depth transform as a radix FFT along the sweep (FP32; dir -1: adjoint).
// shift (forward): the stack is a ring whose window starts at slot `shift`;
// frame t of the window is read from slot (t + shift) mod T.
// epi: EPI_STORE (complex64), EPI_ABS or EPI_GAMMA (forward only; the latter
// writes Gamma = 4 |V 2^-gamma_exp|^2 V 2^-gamma_exp and one FP64 partial of
// sum |V|^4 per workgroup, depth_fft_blocks(P) of them).  wt: exp(-2 pi i k/T).
// grid: workgroups of the EPI_STORE / EPI_ABS kernels walking the tiles
// (0 = one per tile; depth_fft_grid(cu) gives the tuned value); px: pixels per
// workgroup of the forward EPI_STORE / EPI_ABS kernels (16, 32 or 64; 0 = default).
bool depth_fft_supported(int T);
int depth_fft_blocks(int P);
int depth_fft_grid(int cu_count);
hipError_t launch_depth_fft(int T, int P, int dir, int epi, const float2* H, const float2* wt, void* out,
                            hipStream_t s, int shift = 0, int gamma_exp = 0, double* partials = nullptr,
                            int grid = 0, int px = 0);
hipError_t launch_depth_twiddles(int T, float2* wt, hipStream_t s);

// Depth transform as a two-factor (16 x T/16) DFT on MFMA, forward only, in
// any operand precision (H in the format of that precision, scaled by
// 2^-sigma for FP16); epi EPI_STORE (with the ring shift) or EPI_ABS.
// ops: the per-lane DFT-matrix operands of the plan's (T, precision),
// depth_4step_ops_bytes() of device memory filled by launch_4step_operands.
bool depth_4step_supported(int T);
size_t depth_4step_ops_bytes();
hipError_t launch_4step_operands(int T, int prec, uint32_t* ops, hipStream_t s);
// px: pixels per workgroup tile, 16 or 32 (0 = 32)
hipError_t launch_depth_4step(int T, int P, int prec, int epi, const void* H, const float2* wt, const uint32_t* ops,
                              void* out, int sigma, hipStream_t s, int shift = 0, int px = 0);

hipError_t launch_cuts(int T, int N, const float2* vol, int x0, int y0, int q0, int power,
                       float* cut_xy, float* cut_xz, float* cut_yz, hipStream_t s);

// Final reduction of the gradient: out[0] = L (or 0), out[1] = dL/dz,
// out[2..16] = dL/dc, out[17..17+T) = dL/dphi.
hipError_t launch_grad_finish(int T, int N, int nblk, const double* mono_partials,
                              const double* loss_partials, int n_loss, const double* alpha_over_z,
                              const double* zmat, double grad_scale, double* out, hipStream_t s);

}  // namespace ssoct
