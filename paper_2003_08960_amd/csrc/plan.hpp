// Host-side plan object shared by the C ABI (abi.cpp) and the streaming
// engine (stream.cpp).
#pragma once
#include <string>
#include <vector>

#include "../../include/ssoct.h"
#include "internal.hpp"

namespace ssoct {

// Workspace layout: H stack, one chunk of row-transformed frames, and with
// SSOCT_BACKWARD a second stack plus the FP64 reduction partials.
struct WsLayout {
  size_t H, inter, B2, mono, loss, total;
};
WsLayout ws_layout(int T, int N, uint32_t flags, int F);
int frames_per_chunk(int T, int N, int mib);
int chunk_capacity(int T, int N, uint32_t flags);

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* where);

#define SSOCT_HIP(call)                                \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return ssoct::hip_fail(e_, #call); \
  } while (0)

}  // namespace ssoct

struct ssoct_plan {
  int T = 0, N = 0, device = 0, cu = 0;
  int F = 0;                   // frames per chunk the workspace is sized for
  int F_frame = 0;             // default frames per chunk of the frame order
  int F_df = 0;                // default frames per chunk of the depth-first order (two per bin)
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  ssoct::DepthLayout dl{};
  // launch shapes (ssoct_plan_tune / ssoct_plan_set_tuning)
  int F_run = 0;               // frames per chunk set by the tuning (1 .. F; 0 = the order's default)
  int col_grid = 0;            // persistent column workgroups (0 = default)
  int as_col_grid0 = 0;        // default of the angular-spectrum column pass (set at creation)
  int depth_grid = 0;          // persistent depth workgroups (0 = default)
  int rpg_g = 0;               // rows per row group of the bin-pair row pass (0 = by launch size; 2, 4, 8)
  int col_tile = 0;            // column tile width of the Fresnel column passes (0 = default)
  int depth_kc = 0;            // frames per K chunk of the dense depth product (0 = default; half of it)
  int col_radix = 0;           // radix order of the forward column transforms (0: 16..16 L, 1: L 16..16)
  int dfft_px = 0;             // pixels per workgroup of the forward FFT (16, 32, 64) or factored (16, 32)
                               // depth transform (0 = default 32)
  // device tables
  ssoct::AxisTab* rows = nullptr;
  ssoct::AxisTab* cols = nullptr;
  float2* tw = nullptr;
  float2* tw1 = nullptr;        // twiddles of the second radix order (N not a power of 16)
  float2* outfac = nullptr;
  float* apoly = nullptr;       // aberration screen, per-row polynomials [N][APOLY_STRIDE]
  float2* screen = nullptr;     // the same screen as N x N factors, built for the gradient entry points
  uint32_t* f4ops = nullptr;    // DFT-matrix operands of the factored depth form
  bool screen_ok = false;       // screen matches the current tables
  double* params = nullptr;    // ParamLayout + alpha/z [T] + zmat [15 x 15]
  float* a_f32 = nullptr;
  uint4* a_f16 = nullptr;
  uint4* a_bf16 = nullptr;
  float2* dtw = nullptr;       // exp(-2 pi i k / T): FFT depth twiddles, dense window phase
  bool general = false;        // SSOCT_NONUNIFORM_K: general depth matrix from kappa_t
  double* kappa = nullptr;     // device kappa_t (general matrix)
  std::vector<double> gate;    // apodising gate g_t (empty: rectangular)
  double* as_params = nullptr; // SSOCT_ANGULAR_SPECTRUM: per frame {1/lambda^2, phase cycles, amplitude}
  double as_pitch = 0.0, as_z = 0.0;
  double zmat[15][ssoct::N_MONO];
  std::vector<double> cache;   // parameter set the tables were last built from
  bool have_aberr = false;
  int sigma = 0;               // FP16 operand scale exponent for the current tables
  // profiling record (SSOCT_PROFILE): per render, events at start, after the
  // tables, after the Fresnel stage and after the depth transform, plus one
  // after every row-pass and column-pass launch (kev, up to KMAX chunks)
  static constexpr int MAXREC = 64;
  static constexpr int KMAX = 64;
  std::vector<hipEvent_t> ev;   // [MAXREC][4]
  std::vector<hipEvent_t> kev;  // [MAXREC][2 KMAX], created on first use
  std::vector<int> rec_nch;     // chunks of each record (0: no per-kernel events)
  std::vector<int> rec_df;      // record made in the depth-first order
  int rec = 0;
  bool streaming = false;      // a stream object uses the plan's tables
  bool df_allowed = false;     // current tables allow the depth-first order (SSOCT_DEPTH_FFT)
  int order = 1;               // tuning: 1 = depth-first order where allowed (default, measured faster), 0 = frame order
  bool depth_first() const { return df_allowed && order == 1; }
  // frames per chunk of the evaluation order in use, and of the frame order
  // (the sliding windows and the adjoint always transform frames)
  int frames_run() const { return F_run > 0 ? F_run : (depth_first() ? F_df : F_frame); }
  int frames_run_frame() const { return F_run > 0 ? F_run : F_frame; }
};

namespace ssoct {

int check_plan(const ssoct_plan* p);
int update_tables(ssoct_plan* p, const double* lambda, double pitch, double z, const double* disp,
                  const double* zern, bool for_backward);
int depth_prec(uint32_t flags);
// Enqueue one forward render on `stream` (tables must be current): Fresnel
// stage into the workspace, depth transform into vol.  `ev` (4 events or
// null) brackets the stages for the profiling record; `kev` (2 events per
// chunk, or null) is recorded after each row-pass and column-pass launch.
int render_core(ssoct_plan* p, hipStream_t stream, const uint16_t* frames, char* ws, const WsLayout& L, void* vol,
                hipEvent_t* ev, hipEvent_t* kev = nullptr);
// The two halves of render_core: the Fresnel stage of frames [t0, t0 + Fc)
// (Fc <= the plan's frames per chunk), and the depth transform of the whole
// H stack into vol.
int render_chunk(ssoct_plan* p, hipStream_t stream, const uint16_t* frames, char* ws, const WsLayout& L, int t0,
                 int Fc);
// shift: the stack is a ring of frames by sweep position and the window
// starts at slot `shift` (read in rotated order, or bin q multiplied by
// exp(+2 pi i q shift / T) for the dense product); 0 otherwise
int render_depth(ssoct_plan* p, hipStream_t stream, char* ws, const WsLayout& L, void* vol, int shift = 0);
// Fresnel-stage launches per render (chunks of frames, or of bins in the depth-first order)
int fresnel_chunks(const ssoct_plan* p);

}  // namespace ssoct
