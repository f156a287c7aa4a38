// C ABI: plans, argument checks, table caching, launch shapes (tuning) and
// the order of kernel launches for render, cuts and the gradient entry points.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "plan.hpp"

#include <array>
#include <map>

using namespace ssoct;

// Fresnel-stage chunking: the row pass of a chunk of frames writes a buffer
// of SSOCT_CHUNK_MIB that the column pass reads right after.  (Overlapping
// the two passes on two streams with a ring of buffers was measured slower:
// the per-chunk cross-stream waits cost more than the overlap.)  The
// depth-first order of the FFT form runs best with twice that buffer (its
// 2-D passes per chunk of bins then stay within the 256 MB MALL with half as
// many launches), so FFT-form plans size the buffer for SSOCT_CHUNK_DF_MIB.
#ifndef SSOCT_CHUNK_MIB
#define SSOCT_CHUNK_MIB 128
#endif
#ifndef SSOCT_CHUNK_DF_MIB
#define SSOCT_CHUNK_DF_MIB 256
#endif

namespace ssoct {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return SSOCT_EHIP;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static bool pow2_in_range(int N) { return N >= 16 && N <= 2048 && (N & (N - 1)) == 0; }

int frames_per_chunk(int T, int N, int mib) {
  // one chunk of row-transformed frames (8 bytes per pixel) near `mib` MiB
  const size_t per = (size_t)N * N * 8;
  size_t f = ((size_t)mib << 20) / per;
  if (f < 1) f = 1;
  if (f > (size_t)T) f = (size_t)T;
  return (int)f;
}

int chunk_capacity(int T, int N, uint32_t flags) {
  const int fr = frames_per_chunk(T, N, SSOCT_CHUNK_MIB);
  const int df = (flags & SSOCT_DEPTH_FFT) ? frames_per_chunk(T, N, SSOCT_CHUNK_DF_MIB) : fr;
  return fr > df ? fr : df;
}

// FP64 loss partials of the sharpness epilogue: one per dense depth
// workgroup (at most 4096) or one per FFT depth workgroup
static size_t loss_partial_capacity(int N) {
  const size_t nfft = (size_t)depth_fft_blocks(N * N);
  return nfft > 4096 ? nfft : 4096;
}

WsLayout ws_layout(int T, int N, uint32_t flags, int F) {
  WsLayout w{};
  const size_t stack = (size_t)T * N * N * 8;
  size_t off = 0;
  w.H = off;
  off += align256(stack);
  w.inter = off;
  off += align256((size_t)F * N * N * 8);
  if (flags & SSOCT_BACKWARD) {
    w.B2 = off;
    off += align256(stack);
    w.mono = off;
    off += align256((size_t)T * row_adj_blocks(N) * N_MONO * sizeof(double));
    w.loss = off;
    off += align256((size_t)loss_partial_capacity(N) * sizeof(double));
  }
  w.total = off;
  return w;
}

// Zernike j (ANSI/OSA, orthonormal) expanded in the monomials x^a y^b of the
// fixed order (a + b <= 4): Z_j = norm * R_n^|m|(rho) * {cos, sin}(|m| theta),
// with rho^|m| cos(|m| theta) = Re (x + i y)^|m|, rho^|m| sin = Im, and the
// remaining even power of rho as (x^2 + y^2)^k.
static void zernike_monomials(double zmat[15][N_MONO]) {
  static const int A[N_MONO] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
  static const int B[N_MONO] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4};
  auto fact = [](int n) {
    double r = 1;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
  };
  auto binom = [&](int n, int k) { return fact(n) / (fact(k) * fact(n - k)); };
  for (int j = 0; j < 15; ++j) {
    const int n = (int)std::ceil((-3.0 + std::sqrt(9.0 + 8.0 * j)) / 2.0);
    const int m = 2 * j - n * (n + 2);
    const int am = m < 0 ? -m : m;
    double poly[5][5] = {};  // poly[a][b]: coefficient of x^a y^b
    double ang[5][5] = {};   // Re (m >= 0) or Im (m < 0) of (x + i y)^|m|
    for (int r = 0; r <= am; ++r) {
      const double c = binom(am, r);  // c x^(am-r) (i y)^r
      if (m >= 0 && r % 2 == 0) ang[am - r][r] += c * ((r / 2) % 2 ? -1.0 : 1.0);
      if (m < 0 && r % 2 == 1) ang[am - r][r] += c * (((r - 1) / 2) % 2 ? -1.0 : 1.0);
    }
    const int p = (n - am) / 2;
    for (int k = 0; k <= p; ++k) {
      const double rc =
          ((k % 2) ? -1.0 : 1.0) * fact(n - k) / (fact(k) * fact((n + am) / 2 - k) * fact((n - am) / 2 - k));
      const int e = p - k;  // times (x^2 + y^2)^e
      for (int r = 0; r <= e; ++r) {
        const double bc = binom(e, r);
        for (int a = 0; a + 2 * (e - r) <= 4; ++a)
          for (int b = 0; b + 2 * r <= 4; ++b)
            if (ang[a][b] != 0.0) poly[a + 2 * (e - r)][b + 2 * r] += rc * bc * ang[a][b];
      }
    }
    const double norm = std::sqrt((m == 0 ? 1.0 : 2.0) * (n + 1));
    for (int k = 0; k < N_MONO; ++k) zmat[j][k] = norm * poly[A[k]][B[k]];
  }
}

static void plan_free(ssoct_plan* p) {
  if (!p) return;
  (void)hipFree(p->rows);
  (void)hipFree(p->cols);
  (void)hipFree(p->tw);
  (void)hipFree(p->tw1);
  (void)hipFree(p->outfac);
  (void)hipFree(p->apoly);
  (void)hipFree(p->screen);
  (void)hipFree(p->f4ops);
  (void)hipFree(p->params);
  (void)hipFree(p->a_f32);
  (void)hipFree(p->a_f16);
  (void)hipFree(p->a_bf16);
  (void)hipFree(p->dtw);
  (void)hipFree(p->kappa);
  (void)hipFree(p->as_params);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->kev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

static bool finite_all(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

int depth_prec(uint32_t flags) {
  const uint32_t pr = flags & SSOCT_PREC_MASK;
  const bool split = (flags & SSOCT_SPLIT) != 0;
  if (pr == SSOCT_PREC_FP16) return split ? DP_F16_SPLIT : DP_F16;
  if (pr == SSOCT_PREC_BF16) return split ? DP_BF16_SPLIT : DP_BF16;
  return DP_F32;
}

static int h_format(int prec) {
  if (prec == DP_F16 || prec == DP_F16_SPLIT) return HF_F16;
  if (prec == DP_BF16 || prec == DP_BF16_SPLIT) return HF_BF16;
  return HF_F32;
}

static const void* amat_for(const ssoct_plan* p, int prec) {
  if (prec == DP_F32) return p->a_f32;
  if (prec == DP_F16 || prec == DP_F16_SPLIT) return p->a_f16;
  return p->a_bf16;
}

int check_plan(const ssoct_plan* p) {
  if (!p) return fail(SSOCT_EINVAL, "plan is NULL");
  return SSOCT_OK;
}

// Validate the per-call physical parameters and (re)build the tables when
// they changed.  Returns SSOCT_OK, SSOCT_WARN_UNDERSAMPLED or an error.
int update_tables(ssoct_plan* p, const double* lambda, double pitch, double z, const double* disp,
                  const double* zern, bool for_backward) {
  const int T = p->T, N = p->N;
  if (!lambda) return fail(SSOCT_EINVAL, "lambda is NULL");
  if (!finite_all(lambda, T)) return fail(SSOCT_EINVAL, "lambda has a non-finite entry");
  for (int t = 0; t < T; ++t)
    if (!(lambda[t] > 0)) return fail(SSOCT_EINVAL, "lambda must be > 0");
  if (!(pitch > 0) || !std::isfinite(pitch)) return fail(SSOCT_EINVAL, "pitch must be finite and > 0");
  if (!(z != 0) || !std::isfinite(z)) return fail(SSOCT_EINVAL, "z must be finite and non-zero");
  if (disp && !finite_all(disp, T)) return fail(SSOCT_EINVAL, "disp_phase has a non-finite entry");
  if (zern && !finite_all(zern, 15)) return fail(SSOCT_EINVAL, "zernike has a non-finite entry");
  if (for_backward && (p->flags & SSOCT_EQ6_PHASE))
    return fail(SSOCT_EUNSUPPORTED, "gradients are not available with SSOCT_EQ6_PHASE");
  if (for_backward && (p->general || !p->gate.empty() || (p->flags & SSOCT_ANGULAR_SPECTRUM)))
    return fail(SSOCT_EUNSUPPORTED,
                "gradients are not available with a gate, SSOCT_NONUNIFORM_K or SSOCT_ANGULAR_SPECTRUM");
  if ((p->flags & SSOCT_ANGULAR_SPECTRUM) && zern)
    return fail(SSOCT_EUNSUPPORTED, "the aberration screen belongs to the Fresnel path");

  double lam1 = lambda[0];
  for (int t = 1; t < T; ++t) lam1 = lambda[t] > lam1 ? lambda[t] : lam1;
  const bool as = (p->flags & SSOCT_ANGULAR_SPECTRUM) != 0;
  // the validity bound after Eq. 6 concerns the Fresnel transform only
  const int status = (!as && std::fabs(z) < (double)N * pitch * pitch / lam1) ? SSOCT_WARN_UNDERSAMPLED : SSOCT_OK;

  std::vector<double> key;
  key.reserve(3 * T + 20);
  key.insert(key.end(), lambda, lambda + T);
  key.push_back(pitch);
  key.push_back(z);
  key.push_back(disp ? 1.0 : 0.0);
  if (disp) key.insert(key.end(), disp, disp + T);
  key.push_back(zern ? 1.0 : 0.0);
  if (zern) key.insert(key.end(), zern, zern + 15);
  key.push_back((double)p->gate.size());
  key.insert(key.end(), p->gate.begin(), p->gate.end());
  if (key == p->cache) return status;
  if (p->streaming) return fail(SSOCT_EINVAL, "the plan's parameters are fixed while a stream uses it");

  const bool exact = (p->flags & SSOCT_CHIRP_EXACT) != 0;
  const bool eq6 = (p->flags & SSOCT_EQ6_PHASE) != 0;
  std::vector<double> h(ParamLayout::count(T) + T + 15 * N_MONO, 0.0);
  const double two_pi = 6.283185307179586476925;
  const double eq6_cyc = eq6 ? 0.25 - (z / lam1 - std::floor(z / lam1)) : 0.0;
  for (int t = 0; t < T; ++t) {
    const double s = lambda[t] / lam1;
    const double kappa = pitch * pitch * (exact ? s : 1.0) / (2.0 * lam1 * z);  // alpha_t / (2 pi)
    double* pf = &h[(size_t)ParamLayout::PER_FRAME * t];
    pf[0] = s;
    pf[1] = kappa;
    pf[2] = (disp ? disp[t] / two_pi : 0.0) + eq6_cyc;
    pf[3] = (eq6 ? pitch * pitch / (lam1 * z) : 1.0) * (p->gate.empty() ? 1.0 : p->gate[t]);   // gate g_t
    h[ParamLayout::count(T) + t] = two_pi * kappa / z;  // alpha_t / z
  }
  double* g = &h[ParamLayout::globals(T)];
  g[ParamLayout::G_KAPPA_OUT] = lam1 * z / (2.0 * (double)N * N * pitch * pitch);
  // all-zero coefficients give A = 1 exactly: no screen is built or read
  bool zern_on = false;
  for (int j = 0; zern && j < 15; ++j) zern_on = zern_on || zern[j] != 0.0;
  if (zern_on) {
    for (int k = 0; k < N_MONO; ++k) {
      double c = 0.0;
      for (int j = 0; j < 15; ++j) c += zern[j] * p->zmat[j][k];
      g[ParamLayout::G_POLY + k] = c;
    }
    g[ParamLayout::G_HAS_ABERR] = 1.0;
  }
  std::memcpy(&h[ParamLayout::count(T) + T], &p->zmat[0][0], sizeof(double) * 15 * N_MONO);
  SSOCT_HIP(hipMemcpyAsync(p->params, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
  SSOCT_HIP(launch_axis_tables(p->params, T, N, p->rows, p->cols, p->stream));
  if (as) {
    // per frame: 1/lambda_t^2, dispersion phase in cycles, gate / N^2 (inverse DFT normalisation)
    std::vector<double> a(3 * (size_t)T);
    for (int t = 0; t < T; ++t) {
      a[3 * t] = 1.0 / (lambda[t] * lambda[t]);
      a[3 * t + 1] = disp ? disp[t] / two_pi : 0.0;
      a[3 * t + 2] = (p->gate.empty() ? 1.0 : p->gate[t]) / ((double)N * N);
    }
    SSOCT_HIP(hipMemcpyAsync(p->as_params, a.data(), a.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
    p->as_pitch = pitch;
    p->as_z = z;
  }
  if (p->general) {
    // kappa_t = (k_t - k_0) / dk, dk = (k_{T-1} - k_0) / (T - 1): sweep position in mean wavenumber steps
    std::vector<double> kap(T, 0.0);
    if (T > 1) {
      const double two_pi_ = 6.283185307179586476925;
      const double k0 = two_pi_ / lambda[0], dk = (two_pi_ / lambda[T - 1] - k0) / (double)(T - 1);
      if (!(dk != 0.0) || !std::isfinite(dk)) return fail(SSOCT_EINVAL, "SSOCT_NONUNIFORM_K needs lambda_0 != lambda_{T-1}");
      for (int t = 0; t < T; ++t) kap[t] = (two_pi_ / lambda[t] - k0) / dk;
    }
    SSOCT_HIP(hipMemcpyAsync(p->kappa, kap.data(), (size_t)T * sizeof(double), hipMemcpyHostToDevice, p->stream));
    SSOCT_HIP(launch_depth_tables(T, p->kappa, p->a_f32, p->a_f16, p->a_bf16, p->stream));
  }
  SSOCT_HIP(launch_misc_tables(p->params, T, N, p->outfac, zern_on ? p->apoly : nullptr, p->stream));
  p->have_aberr = zern_on;
  p->screen_ok = false;
  // depth-first order: the chirp and the per-frame row factor must not depend on the frame
  bool no_disp = true;
  for (int t = 0; disp && t < T; ++t) no_disp = no_disp && disp[t] == 0.0;
  p->df_allowed = (p->flags & SSOCT_DEPTH_FFT) && !exact && !(p->flags & SSOCT_WRITE_ABS) && no_disp &&
                  p->gate.empty() && !as;
  // FP16 operands: |H| <= N^2 * 65535 * amplitude, kept below 2^15 by an exact power-of-two scale
  p->sigma = 0;
  if (h_format(depth_prec(p->flags)) == HF_F16) {
    const double amp = eq6 ? std::fabs(pitch * pitch / (lam1 * z)) : 1.0;
    p->sigma = (int)std::ceil(std::log2((double)N * N * 65535.0 * amp / 32768.0));
  }
  p->cache.swap(key);
  return status;
}

// Persistent column workgroups: the tuned count, else the default for N and
// the column tile width in use (ct; 0 = the default tile)
// twiddle table of the forward column transforms' radix order
static const float2* col_tw(const ssoct_plan* p) { return p->col_radix ? p->tw1 : p->tw; }

static int col_grid_of(const ssoct_plan* p, int ct = 0) {
  return p->col_grid > 0 ? p->col_grid : col_default_grid(p->N, p->cu, ct);
}

// Fresnel stage over all frames, chunk by chunk: row pass (rescale + chirp +
// row DFT) into the chunk buffer, then column DFT into H.
static int depth_grid_for(const ssoct_plan* p) {
  return p->depth_grid > 0 ? p->depth_grid : depth_grid(p->T, p->N * p->N, p->cu, p->general);
}

int render_chunk(ssoct_plan* p, hipStream_t s, const uint16_t* frames, char* ws, const WsLayout& L, int t0, int Fc) {
  const int N = p->N;
  const int fmt = h_format(depth_prec(p->flags));
  if (p->flags & SSOCT_ANGULAR_SPECTRUM) {
    SSOCT_HIP(launch_as_stage(N, Fc, t0, frames, p->tw, p->as_params, 1.0 / ((double)N * p->as_pitch), p->as_z,
                              reinterpret_cast<float2*>(ws + L.inter), ws + L.H, fmt, p->sigma,
                              p->col_grid > 0 ? p->col_grid : p->as_col_grid0, s));
    return SSOCT_OK;
  }
  float2* inter = reinterpret_cast<float2*>(ws + L.inter);
  const float* ab = p->have_aberr ? p->apoly : nullptr;
  SSOCT_HIP(launch_row_pass(N, Fc, t0, frames, p->rows, p->cols, p->tw, ab, p->outfac, inter, s));
  SSOCT_HIP(launch_col_pass(N, Fc, t0, inter, col_tw(p), p->outfac, ws + L.H, fmt, p->sigma,
                            col_grid_of(p, p->col_tile), s, p->col_tile, p->col_radix));
  return SSOCT_OK;
}

int render_depth(ssoct_plan* p, hipStream_t s, char* ws, const WsLayout& L, void* vol, int shift) {
  const int prec = depth_prec(p->flags);
  const int epi = (p->flags & SSOCT_WRITE_ABS) ? EPI_ABS : EPI_STORE;
  if (p->flags & SSOCT_DEPTH_FFT) {
    SSOCT_HIP(launch_depth_fft(p->T, p->N * p->N, +1, epi, reinterpret_cast<const float2*>(ws + L.H), p->dtw, vol, s,
                               shift, 0, nullptr, depth_fft_grid(p->cu), p->dfft_px));
    return SSOCT_OK;
  }
  if (p->flags & SSOCT_DEPTH_4STEP) {
    SSOCT_HIP(launch_depth_4step(p->T, p->N * p->N, prec, epi, ws + L.H, p->dtw, p->f4ops, vol, p->sigma, s, shift,
                                 p->dfft_px));
    return SSOCT_OK;
  }
  SSOCT_HIP(launch_depth(p->T, p->N * p->N, prec, +1, epi, ws + L.H, amat_for(p, prec), vol, p->sigma, 0, nullptr,
                         depth_grid_for(p), s, p->dtw, shift, p->general, p->depth_kc));
  return SSOCT_OK;
}

int fresnel_chunks(const ssoct_plan* p) {
  const int F = p->frames_run();
  if (p->depth_first()) {
    const int fh = F / 2 > 0 ? F / 2 : 1;
    return (p->T / 2 + fh) / fh;   // ceil((T/2 + 1) / fh)
  }
  return (p->T + F - 1) / F;
}

// Depth-first order (frame-independent chirp and row factor): the depth
// DFT of the rescaled real frames, G_q for q = 0..T/2 (stage 1), then the
// Fresnel transforms of the bins, chunk by chunk: V[q] = DFT2(fac G_q) and
// V[T - q] = DFT2(fac conj(G_q)) for 0 < q < T/2.  Events: ev[1] start,
// ev[2] after stage 1, ev[3] at the end; kev after each row and column step.
static int render_depth_first(ssoct_plan* p, hipStream_t s, const uint16_t* frames, char* ws, const WsLayout& L,
                              void* vol, hipEvent_t* ev, hipEvent_t* kev) {
  const int T = p->T, N = p->N;
  const size_t P = (size_t)N * N;
  float2* G = reinterpret_cast<float2*>(ws + L.H);
  float2* inter = reinterpret_cast<float2*>(ws + L.inter);
  float2* V = static_cast<float2*>(vol);
  const float* ab = p->have_aberr ? p->apoly : nullptr;
  const int nb = T / 2 + 1;                     // bins of G
  const int nconj = (T + 1) / 2;                // bins q < nconj have a partner T - q (q >= 1)
  const int F = p->frames_run();
  const int fh = F / 2 > 0 ? F / 2 : 1;   // bins per chunk: 2 fh transforms fit the chunk buffer
  if (2 * fh > p->F) return fail(SSOCT_EUNSUPPORTED, "chunk buffer too small for the depth-first order");
  if (ev) SSOCT_HIP(hipEventRecord(ev[1], s));
  SSOCT_HIP(launch_rescale_dft(T, N, frames, p->rows, p->cols, p->params, p->dtw, G, s));
  if (ev) SSOCT_HIP(hipEventRecord(ev[2], s));
  for (int qa = 0, c = 0; qa < nb; qa += fh, ++c) {
    const int n = nb - qa < fh ? nb - qa : fh;
    SSOCT_HIP(launch_row_pass_g(N, n, qa, T, G, p->rows, p->cols, p->tw, ab, p->outfac, inter, fh, p->rpg_g, p->cu, s));
    if (kev) SSOCT_HIP(hipEventRecord(kev[2 * c], s));
    // one launch: V[q] for the chunk's bins, then V[T - q] for those with a partner
    const int cg = col_grid_of(p, p->col_tile);
    const int ca = qa > 1 ? qa : 1;
    const int cb = qa + n < nconj ? qa + n : nconj;
    const int nm = cb > ca ? cb - ca : 0;
    SSOCT_HIP(launch_col_pass_v(N, n, inter, col_tw(p), p->outfac, V + (size_t)qa * P, +1, cg, p->col_tile, s, nm,
                                inter + (size_t)(fh + ca - qa) * P, V + (size_t)(T - ca) * P, -1, p->col_radix));
    if (kev) SSOCT_HIP(hipEventRecord(kev[2 * c + 1], s));
  }
  if (ev) SSOCT_HIP(hipEventRecord(ev[3], s));
  return SSOCT_OK;
}

int render_core(ssoct_plan* p, hipStream_t s, const uint16_t* frames, char* ws, const WsLayout& L, void* vol,
                hipEvent_t* ev, hipEvent_t* kev) {
  if (p->depth_first()) return render_depth_first(p, s, frames, ws, L, vol, ev, kev);
  const int T = p->T, N = p->N, F = p->frames_run();
  if (ev) SSOCT_HIP(hipEventRecord(ev[1], s));
  if (kev) {  // the two passes launched one by one with an event after each
    const int fmt = h_format(depth_prec(p->flags));
    float2* inter = reinterpret_cast<float2*>(ws + L.inter);
    const float* ab = p->have_aberr ? p->apoly : nullptr;
    for (int t0 = 0, c = 0; t0 < T; t0 += F, ++c) {
      const int Fc = T - t0 < F ? T - t0 : F;
      SSOCT_HIP(launch_row_pass(N, Fc, t0, frames, p->rows, p->cols, p->tw, ab, p->outfac, inter, s));
      SSOCT_HIP(hipEventRecord(kev[2 * c], s));
      SSOCT_HIP(launch_col_pass(N, Fc, t0, inter, col_tw(p), p->outfac, ws + L.H, fmt, p->sigma,
                                col_grid_of(p, p->col_tile), s, p->col_tile, p->col_radix));
      SSOCT_HIP(hipEventRecord(kev[2 * c + 1], s));
    }
  } else {
    for (int t0 = 0; t0 < T; t0 += F) {
      if (int rc = render_chunk(p, s, frames, ws, L, t0, T - t0 < F ? T - t0 : F)) return rc;
    }
  }
  if (ev) SSOCT_HIP(hipEventRecord(ev[2], s));
  if (int rc = render_depth(p, s, ws, L, vol)) return rc;
  if (ev) SSOCT_HIP(hipEventRecord(ev[3], s));
  return SSOCT_OK;
}

// The gradient runs in FP32 whatever the plan's depth form: as radix FFTs
// along the sweep when T allows, else as the dense FP32 product.
static bool adjoint_by_fft(const ssoct_plan* p) { return depth_fft_supported(p->T) && !p->general; }

static int adjoint_chain(ssoct_plan* p, const uint16_t* frames, const void* G, char* ws, const WsLayout& L,
                         const double* loss_partials, int n_loss, double grad_scale, double* out) {
  const int T = p->T, N = p->N, F = p->frames_run_frame();
  if (p->have_aberr && !p->screen_ok) {   // the adjoint row pass reads the screen as N x N factors
    if (!p->screen) SSOCT_HIP(hipMalloc(&p->screen, (size_t)N * N * sizeof(float2)));
    SSOCT_HIP(launch_aberr_screen(p->params, T, N, p->screen, p->stream));
    p->screen_ok = true;
  }
  float2* beta = reinterpret_cast<float2*>(ws + L.H);
  float2* inter = reinterpret_cast<float2*>(ws + L.inter);
  double* mono = reinterpret_cast<double*>(ws + L.mono);
  if (adjoint_by_fft(p))
    SSOCT_HIP(launch_depth_fft(T, N * N, -1, EPI_STORE, static_cast<const float2*>(G), p->dtw, beta, p->stream, 0, 0,
                               nullptr, depth_fft_grid(p->cu)));
  else
    SSOCT_HIP(launch_depth(T, N * N, DP_F32, -1, EPI_STORE, G, p->a_f32, beta, 0, 0, nullptr, depth_grid_for(p),
                           p->stream));
  for (int t0 = 0; t0 < T; t0 += F) {
    const int Fc = T - t0 < F ? T - t0 : F;
    SSOCT_HIP(launch_col_pass_adj(N, Fc, t0, beta, p->tw, inter, col_grid_of(p), p->stream));
    SSOCT_HIP(launch_row_pass_adj(N, Fc, t0, frames, p->rows, p->cols, p->tw, p->have_aberr ? p->screen : nullptr,
                                  inter, mono, p->stream));
  }
  const double* aoz = p->params + ParamLayout::count(T);
  const double* zm = aoz + T;
  SSOCT_HIP(launch_grad_finish(T, N, row_adj_blocks(N), mono, loss_partials, n_loss, aoz, zm, grad_scale, out,
                               p->stream));
  return SSOCT_OK;
}

// argument checks shared by render and tune
static int check_render_args(ssoct_plan* p, const uint16_t* frames, void* workspace, size_t workspace_bytes,
                             void* vol, WsLayout* L) {
  if (int rc = check_plan(p)) return rc;
  if (!frames || !workspace || !vol) return fail(SSOCT_EINVAL, "frames, workspace and vol must be non-NULL");
  const int T = p->T, N = p->N;
  *L = ws_layout(T, N, p->flags & ~SSOCT_BACKWARD, p->F);
  if (workspace_bytes < L->total) return fail(SSOCT_ENOMEM, "workspace smaller than ssoct_workspace_size()");
  const size_t vol_bytes = (size_t)T * N * N * ((p->flags & SSOCT_WRITE_ABS) ? 4 : 8);
  if (overlap(vol, vol_bytes, frames, (size_t)T * N * N * 2) || overlap(vol, vol_bytes, workspace, workspace_bytes))
    return fail(SSOCT_EALIAS, "vol overlaps frames or workspace");
  return SSOCT_OK;
}

}  // namespace ssoct

extern "C" {

int ssoct_version(void) { return SSOCT_VERSION; }

const char* ssoct_last_error(void) { return g_err.c_str(); }

size_t ssoct_workspace_size(int T, int N, uint32_t flags) {
  if (T < 1 || T > 1024 || !pow2_in_range(N)) return 0;
  return ws_layout(T, N, flags, chunk_capacity(T, N, flags)).total;
}

int ssoct_plan_create(ssoct_plan** plan, int T, int N, uint32_t flags, hipStream_t stream) {
  if (!plan) return fail(SSOCT_EINVAL, "plan pointer is NULL");
  *plan = nullptr;
  if (T < 1 || T > 1024) return fail(SSOCT_EUNSUPPORTED, "T must be in [1, 1024]");
  if (!pow2_in_range(N)) return fail(SSOCT_EUNSUPPORTED, "N must be a power of two in [16, 2048]");
  if ((flags & SSOCT_PREC_MASK) == 3u) return fail(SSOCT_EINVAL, "unknown precision");
  if ((flags & SSOCT_SPLIT) && (flags & SSOCT_PREC_MASK) == SSOCT_PREC_FP32)
    return fail(SSOCT_EINVAL, "SSOCT_SPLIT needs SSOCT_PREC_FP16 or SSOCT_PREC_BF16");
  if ((flags & SSOCT_DEPTH_FFT) && (flags & (SSOCT_PREC_MASK | SSOCT_SPLIT)))
    return fail(SSOCT_EINVAL, "SSOCT_DEPTH_FFT is an FP32 form");
  if ((flags & SSOCT_ANGULAR_SPECTRUM) && (flags & (SSOCT_CHIRP_EXACT | SSOCT_EQ6_PHASE)))
    return fail(SSOCT_EINVAL, "SSOCT_CHIRP_EXACT and SSOCT_EQ6_PHASE belong to the Fresnel transform");
  if ((flags & SSOCT_DEPTH_FFT) && (flags & SSOCT_NONUNIFORM_K))
    return fail(SSOCT_EINVAL, "SSOCT_NONUNIFORM_K needs the dense depth transform (no SSOCT_DEPTH_FFT)");
  if ((flags & SSOCT_DEPTH_FFT) && !depth_fft_supported(T))
    return fail(SSOCT_EUNSUPPORTED, "SSOCT_DEPTH_FFT needs T in {16, 32, 64, 128, 256}");
  if ((flags & SSOCT_DEPTH_4STEP) && (flags & (SSOCT_DEPTH_FFT | SSOCT_NONUNIFORM_K)))
    return fail(SSOCT_EINVAL, "SSOCT_DEPTH_4STEP excludes SSOCT_DEPTH_FFT and SSOCT_NONUNIFORM_K");
  if ((flags & SSOCT_DEPTH_4STEP) && !depth_4step_supported(T))
    return fail(SSOCT_EUNSUPPORTED, "SSOCT_DEPTH_4STEP needs T in {32, 64, 128, 256}");
  ssoct_plan* p = new (std::nothrow) ssoct_plan();
  if (!p) return fail(SSOCT_ENOMEM, "host allocation failed");
  p->T = T;
  p->N = N;
  p->flags = flags;
  p->stream = stream;
  p->F_frame = frames_per_chunk(T, N, SSOCT_CHUNK_MIB);
  p->F_df = (flags & SSOCT_DEPTH_FFT) ? frames_per_chunk(T, N, SSOCT_CHUNK_DF_MIB) : p->F_frame;
  p->F = chunk_capacity(T, N, flags);
  p->F_run = 0;
  p->general = (flags & SSOCT_NONUNIFORM_K) != 0;
  p->dl = depth_layout(T, p->general);
  zernike_monomials(p->zmat);
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cu, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e == hipSuccess && (flags & SSOCT_ANGULAR_SPECTRUM)) p->as_col_grid0 = as_col_default_grid(N, p->cu);
  const size_t axis = (size_t)T * N * sizeof(AxisTab);
  const size_t nparams = ParamLayout::count(T) + T + 15 * N_MONO;
  const size_t na32 = (size_t)p->dl.nrb * (p->dl.T_pad / 2) * 64;
  const size_t na16 = (size_t)p->dl.nrb * (p->dl.T_pad / 16) * 128;
  const size_t ntw = twiddle_table_size(N);
  if (e == hipSuccess) e = hipMalloc(&p->rows, axis);
  if (e == hipSuccess) e = hipMalloc(&p->cols, axis);
  if (e == hipSuccess) e = hipMalloc(&p->tw, (ntw > 0 ? ntw : 1) * sizeof(float2));
  if (e == hipSuccess && has_radix_orders(N)) e = hipMalloc(&p->tw1, twiddle_table_size(N, 1) * sizeof(float2));
  if (e == hipSuccess && (flags & SSOCT_EQ6_PHASE)) e = hipMalloc(&p->outfac, (size_t)N * sizeof(float2));
  // the aberration screen's row polynomials (N x 8 floats): allocated here, so that a render never allocates
  if (e == hipSuccess) e = hipMalloc(&p->apoly, (size_t)N * APOLY_STRIDE * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->params, nparams * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->a_f32, na32 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->a_f16, na16 * sizeof(uint4));
  if (e == hipSuccess) e = hipMalloc(&p->a_bf16, na16 * sizeof(uint4));
  if (e == hipSuccess && (flags & SSOCT_PROFILE)) {
    p->ev.assign((size_t)ssoct_plan::MAXREC * 4, nullptr);
    p->rec_nch.assign(ssoct_plan::MAXREC, 0);
    p->rec_df.assign(ssoct_plan::MAXREC, 0);
    for (auto& ev : p->ev)
      if (e == hipSuccess) e = hipEventCreate(&ev);
  }
  // the general matrix depends on lambda: built with the other tables on the first render
  if (e == hipSuccess && p->general) e = hipMalloc(&p->kappa, (size_t)T * sizeof(double));
  if (e == hipSuccess && (flags & SSOCT_ANGULAR_SPECTRUM)) e = hipMalloc(&p->as_params, (size_t)3 * T * sizeof(double));
  if (e == hipSuccess && !p->general) e = launch_depth_tables(T, nullptr, p->a_f32, p->a_f16, p->a_bf16, stream);
  if (e == hipSuccess) e = launch_twiddles(N, p->tw, stream);
  if (e == hipSuccess && p->tw1) e = launch_twiddles(N, p->tw1, stream, 1);
  if (e == hipSuccess) e = hipMalloc(&p->dtw, (size_t)T * sizeof(float2));
  if (e == hipSuccess) e = launch_depth_twiddles(T, p->dtw, stream);
  if (e == hipSuccess && (flags & SSOCT_DEPTH_4STEP)) e = hipMalloc(&p->f4ops, depth_4step_ops_bytes());
  if (e == hipSuccess && (flags & SSOCT_DEPTH_4STEP)) e = launch_4step_operands(T, depth_prec(flags), p->f4ops, stream);
  if (e != hipSuccess) {
    const int rc = (e == hipErrorOutOfMemory) ? fail(SSOCT_ENOMEM, "device allocation failed")
                                              : hip_fail(e, "ssoct_plan_create");
    plan_free(p);
    return rc;
  }
  *plan = p;
  return SSOCT_OK;
}

int ssoct_plan_set_stream(ssoct_plan* plan, hipStream_t stream) {
  if (int rc = check_plan(plan)) return rc;
  plan->stream = stream;
  return SSOCT_OK;
}

int ssoct_plan_destroy(ssoct_plan* plan) {
  if (!plan) return SSOCT_OK;
  if (plan->streaming) return fail(SSOCT_EINVAL, "a stream or sliding-window object still uses the plan");
  (void)hipStreamSynchronize(plan->stream);
  plan_free(plan);
  return SSOCT_OK;
}

int ssoct_plan_render(ssoct_plan* p, const uint16_t* frames, const double* lambda, double pitch, double z,
                      const double* disp_phase, const double* zernike, void* workspace, size_t workspace_bytes,
                      void* vol) {
  WsLayout L;
  if (int rc = check_render_args(p, frames, workspace, workspace_bytes, vol, &L)) return rc;
  SSOCT_HIP(hipSetDevice(p->device));
  const bool prof = (p->flags & SSOCT_PROFILE) != 0;
  const int slot = p->rec % ssoct_plan::MAXREC;
  hipEvent_t* ev = prof ? &p->ev[(size_t)slot * 4] : nullptr;
  hipEvent_t* kev = nullptr;
  if (prof) SSOCT_HIP(hipEventRecord(ev[0], p->stream));
  const int status = update_tables(p, lambda, pitch, z, disp_phase, zernike, false);
  if (status < 0) return status;
  if (prof) {
    const int nch = fresnel_chunks(p);
    if ((p->flags & SSOCT_PROFILE_KERNELS) && nch <= ssoct_plan::KMAX) {
      if (p->kev.empty()) {
        p->kev.assign((size_t)ssoct_plan::MAXREC * 2 * ssoct_plan::KMAX, nullptr);
        for (auto& e : p->kev) SSOCT_HIP(hipEventCreate(&e));
      }
      kev = &p->kev[(size_t)slot * 2 * ssoct_plan::KMAX];
    }
    p->rec_nch[slot] = kev ? nch : 0;
    p->rec_df[slot] = p->depth_first() ? 1 : 0;
  }
  if (int rc = render_core(p, p->stream, frames, static_cast<char*>(workspace), L, vol, ev, kev)) return rc;
  if (prof) ++p->rec;
  return status;
}

// Default plans of the five-argument render: one plan and workspace per
// (device, stream, T, N), created on first use and kept until
// ssoct_render_release.  Calls on one stream are ordered on the GPU, so they
// can share a workspace; the lock orders the table updates of concurrent
// host threads.
namespace {
struct DefaultPlan {
  int device;
  hipStream_t stream;
  int T, N;
  ssoct_plan* plan;
  void* ws;
  size_t bytes;
};
std::mutex g_default_mu;
std::vector<DefaultPlan> g_default;

// Launch shapes chosen by ssoct_plan_tune, per device architecture, CU count,
// T, N, plan flags (profiling aside) and whether the depth-first order and the
// aberration factor apply: a later tune of the same kind takes them unmeasured.
std::mutex g_tune_mu;
std::map<std::string, std::array<int, SSOCT_TUNING_LEN>> g_tune_cache;

int tune_key(const ssoct_plan* p, std::string* key) {
  hipDeviceProp_t prop;
  SSOCT_HIP(hipGetDeviceProperties(&prop, p->device));
  const unsigned flags = p->flags & ~(unsigned)(SSOCT_PROFILE | SSOCT_PROFILE_KERNELS);
  *key = std::string(prop.gcnArchName) + "/" + std::to_string(p->cu) + "/" + std::to_string(p->T) + "/" +
         std::to_string(p->N) + "/" + std::to_string(flags) + "/" + std::to_string((int)p->df_allowed) + "/" +
         std::to_string((int)p->have_aberr);
  return SSOCT_OK;
}
}  // namespace

int ssoct_render(const uint16_t* frames, int T, int N, const double* lambda, double pitch, double z, void* vol,
                 hipStream_t stream) {
  if (!frames || !lambda || !vol) return fail(SSOCT_EINVAL, "frames, lambda and vol must be non-NULL");
  if (T < 1 || T > 1024) return fail(SSOCT_EUNSUPPORTED, "T must be in [1, 1024]");
  if (!pow2_in_range(N)) return fail(SSOCT_EUNSUPPORTED, "N must be a power of two in [16, 2048]");
  int dev = 0;
  SSOCT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_default_mu);
  DefaultPlan* d = nullptr;
  for (auto& e : g_default)
    if (e.device == dev && e.stream == stream && e.T == T && e.N == N) d = &e;
  if (!d) {
    // FP32 throughout: the depth transform as a radix FFT where T allows it, else the dense product
    const uint32_t flags = depth_fft_supported(T) ? SSOCT_DEPTH_FFT : SSOCT_PREC_FP32;
    DefaultPlan e{dev, stream, T, N, nullptr, nullptr, ssoct_workspace_size(T, N, flags)};
    if (int rc = ssoct_plan_create(&e.plan, T, N, flags, stream)) return rc;
    const hipError_t he = hipMalloc(&e.ws, e.bytes);
    if (he != hipSuccess) {
      plan_free(e.plan);
      return he == hipErrorOutOfMemory ? fail(SSOCT_ENOMEM, "workspace allocation failed")
                                       : hip_fail(he, "ssoct_render workspace");
    }
    g_default.push_back(e);
    d = &g_default.back();
  }
  return ssoct_plan_render(d->plan, frames, lambda, pitch, z, nullptr, nullptr, d->ws, d->bytes, vol);
}

int ssoct_render_release(void) {
  std::lock_guard<std::mutex> lock(g_default_mu);
  int rc = SSOCT_OK;
  for (auto& e : g_default) {
    // the streams the renders ran on may be gone: wait for the whole device
    hipError_t he = hipSetDevice(e.device);
    if (he == hipSuccess) he = hipDeviceSynchronize();
    if (he != hipSuccess && rc == SSOCT_OK) rc = hip_fail(he, "ssoct_render_release");
    plan_free(e.plan);
    (void)hipFree(e.ws);
  }
  g_default.clear();
  return rc;
}

int ssoct_cuts(ssoct_plan* p, const void* vol, int x0, int y0, int q0, float* cut_xy, float* cut_xz, float* cut_yz) {
  if (int rc = check_plan(p)) return rc;
  if (!vol || !cut_xy || !cut_xz || !cut_yz) return fail(SSOCT_EINVAL, "vol and cut pointers must be non-NULL");
  if (p->flags & SSOCT_WRITE_ABS) return fail(SSOCT_EUNSUPPORTED, "cuts need a complex64 volume");
  if (x0 < 0 || x0 >= p->N || y0 < 0 || y0 >= p->N || q0 < 0 || q0 >= p->T)
    return fail(SSOCT_EINVAL, "cut position out of range");
  const size_t vb = (size_t)p->T * p->N * p->N * 8;
  const size_t nxy = (size_t)p->N * p->N * 4, nz = (size_t)p->T * p->N * 4;
  if (overlap(vol, vb, cut_xy, nxy) || overlap(vol, vb, cut_xz, nz) || overlap(vol, vb, cut_yz, nz))
    return fail(SSOCT_EALIAS, "a cut overlaps the volume");
  SSOCT_HIP(hipSetDevice(p->device));
  SSOCT_HIP(launch_cuts(p->T, p->N, static_cast<const float2*>(vol), x0, y0, q0,
                        (p->flags & SSOCT_CUT_POWER) ? 1 : 0, cut_xy, cut_xz, cut_yz, p->stream));
  return SSOCT_OK;
}

int ssoct_backward(ssoct_plan* p, const uint16_t* frames, const double* lambda, double pitch, double z,
                   const double* disp_phase, const double* zernike, const void* grad_vol, void* workspace,
                   size_t workspace_bytes, double* grad_out) {
  if (int rc = check_plan(p)) return rc;
  if (!frames || !grad_vol || !workspace || !grad_out)
    return fail(SSOCT_EINVAL, "frames, grad_vol, workspace and grad_out must be non-NULL");
  const int T = p->T, N = p->N;
  const WsLayout L = ws_layout(T, N, p->flags | SSOCT_BACKWARD, p->F);
  if (workspace_bytes < L.total)
    return fail(SSOCT_ENOMEM, "workspace smaller than ssoct_workspace_size(SSOCT_BACKWARD)");
  if (overlap(grad_out, (size_t)(17 + T) * 8, workspace, workspace_bytes) ||
      overlap(grad_vol, (size_t)T * N * N * 8, workspace, workspace_bytes))
    return fail(SSOCT_EALIAS, "grad_vol or grad_out overlaps the workspace");
  SSOCT_HIP(hipSetDevice(p->device));
  const int status = update_tables(p, lambda, pitch, z, disp_phase, zernike, true);
  if (status < 0) return status;
  if (int rc = adjoint_chain(p, frames, grad_vol, static_cast<char*>(workspace), L, nullptr, 0, 1.0, grad_out))
    return rc;
  return status;
}

int ssoct_backward_sharpness(ssoct_plan* p, const uint16_t* frames, const double* lambda, double pitch, double z,
                             const double* disp_phase, const double* zernike, void* workspace,
                             size_t workspace_bytes, double* grad_out) {
  if (int rc = check_plan(p)) return rc;
  if (!frames || !workspace || !grad_out) return fail(SSOCT_EINVAL, "frames, workspace and grad_out must be non-NULL");
  const int T = p->T, N = p->N;
  const WsLayout L = ws_layout(T, N, p->flags | SSOCT_BACKWARD, p->F);
  if (workspace_bytes < L.total)
    return fail(SSOCT_ENOMEM, "workspace smaller than ssoct_workspace_size(SSOCT_BACKWARD)");
  if (overlap(grad_out, (size_t)(17 + T) * 8, workspace, workspace_bytes))
    return fail(SSOCT_EALIAS, "grad_out overlaps the workspace");
  SSOCT_HIP(hipSetDevice(p->device));
  const int status = update_tables(p, lambda, pitch, z, disp_phase, zernike, true);
  if (status < 0) return status;
  char* ws = static_cast<char*>(workspace);
  void* H = ws + L.H;
  float2* gam = reinterpret_cast<float2*>(ws + L.B2);
  double* loss = reinterpret_cast<double*>(ws + L.loss);
  // Fresnel stage in FP32 whatever the plan's depth precision: the loss and its adjoint run in FP32
  float2* inter = reinterpret_cast<float2*>(ws + L.inter);
  const float* ab = p->have_aberr ? p->apoly : nullptr;
  const int F = p->frames_run_frame();
  for (int t0 = 0; t0 < T; t0 += F) {
    const int Fc = T - t0 < F ? T - t0 : F;
    SSOCT_HIP(launch_row_pass(N, Fc, t0, frames, p->rows, p->cols, p->tw, ab, p->outfac, inter, p->stream));
    SSOCT_HIP(launch_col_pass(N, Fc, t0, inter, p->tw, p->outfac, H, HF_F32, 0, col_grid_of(p), p->stream));
  }
  // |V| <= T N^2 65535: scale by 2^-e so that 4 |V^|^3 stays finite in FP32
  const double bound = (double)T * N * N * 65535.0;
  int e = (int)std::ceil(std::log2(bound)) - 40;
  if (e < 0) e = 0;
  int n_loss;
  if (adjoint_by_fft(p)) {
    n_loss = depth_fft_blocks(N * N);
    SSOCT_HIP(launch_depth_fft(T, N * N, +1, EPI_GAMMA, static_cast<const float2*>(H), p->dtw, gam, p->stream, 0, e,
                               loss));
  } else {
    n_loss = depth_grid_for(p);
    if (n_loss > 4096) return fail(SSOCT_EINVAL, "depth grid larger than the loss-partial buffer");
    SSOCT_HIP(launch_depth(T, N * N, DP_F32, +1, EPI_GAMMA, H, p->a_f32, gam, 0, e, loss, n_loss, p->stream));
  }
  if (int rc = adjoint_chain(p, frames, gam, ws, L, loss, n_loss, std::ldexp(1.0, 3 * e), grad_out)) return rc;
  return status;
}

int ssoct_plan_set_gate(ssoct_plan* p, const double* gate) {
  if (int rc = check_plan(p)) return rc;
  if (p->streaming) return fail(SSOCT_EINVAL, "the plan's parameters are fixed while a stream uses it");
  if (gate && !finite_all(gate, p->T)) return fail(SSOCT_EINVAL, "gate has a non-finite entry");
  if (gate) p->gate.assign(gate, gate + p->T);
  else p->gate.clear();
  p->cache.clear();   // tables rebuilt on the next call
  return SSOCT_OK;
}

int ssoct_profile_read(ssoct_plan* p, float* ms) {
  if (int rc = check_plan(p)) return rc;
  if (!ms) return fail(SSOCT_EINVAL, "ms is NULL");
  if (!(p->flags & SSOCT_PROFILE) || p->rec == 0) return fail(SSOCT_EINVAL, "no profiled render recorded");
  const int n = p->rec < ssoct_plan::MAXREC ? p->rec : ssoct_plan::MAXREC;
  const int last = (p->rec - 1) % ssoct_plan::MAXREC;
  SSOCT_HIP(hipEventSynchronize(p->ev[(size_t)last * 4 + 3]));
  double sum[5] = {0, 0, 0, 0, 0};
  int nk = 0;
  for (int r = 0; r < n; ++r) {
    const int slot = (p->rec - 1 - r) % ssoct_plan::MAXREC;
    hipEvent_t* e = &p->ev[(size_t)slot * 4];
    const bool df = p->rec_df[slot] != 0;   // depth-first order: depth stage between e[1] and e[2]
    for (int i = 0; i < 3; ++i) {
      float t = 0.f;
      SSOCT_HIP(hipEventElapsedTime(&t, e[i], e[i + 1]));
      sum[(df && i > 0) ? 3 - i : i] += t;
    }
    const int nch = p->rec_nch[slot];
    if (nch > 0) {
      hipEvent_t* k = &p->kev[(size_t)slot * 2 * ssoct_plan::KMAX];
      hipEvent_t start = df ? e[2] : e[1];
      for (int c = 0; c < nch; ++c) {
        float tr = 0.f, tc = 0.f;
        SSOCT_HIP(hipEventElapsedTime(&tr, c == 0 ? start : k[2 * c - 1], k[2 * c]));
        SSOCT_HIP(hipEventElapsedTime(&tc, k[2 * c], k[2 * c + 1]));
        sum[3] += tr;
        sum[4] += tc;
      }
      ++nk;
    }
  }
  for (int i = 0; i < 3; ++i) ms[i] = (float)(sum[i] / n);
  ms[3] = (float)n;
  ms[4] = nk == n ? (float)(sum[3] / n) : -1.0f;
  ms[5] = nk == n ? (float)(sum[4] / n) : -1.0f;
  p->rec = 0;
  return SSOCT_OK;
}

int ssoct_plan_get_tuning(const ssoct_plan* p, int* tuning) {
  if (int rc = check_plan(p)) return rc;
  if (!tuning) return fail(SSOCT_EINVAL, "tuning is NULL");
  tuning[0] = p->F_run;
  tuning[1] = p->col_grid;
  tuning[2] = p->depth_grid;
  tuning[3] = p->order;
  tuning[4] = p->rpg_g;
  tuning[5] = p->col_tile;
  tuning[6] = p->dfft_px;
  tuning[7] = p->depth_kc;
  tuning[8] = p->col_radix;
  return SSOCT_OK;
}

int ssoct_plan_set_tuning(ssoct_plan* p, const int* tuning) {
  if (int rc = check_plan(p)) return rc;
  if (!tuning) return fail(SSOCT_EINVAL, "tuning is NULL");
  if (tuning[0] < 0 || tuning[0] > p->F) return fail(SSOCT_EINVAL, "frames per chunk out of range");
  if (tuning[1] < 0 || tuning[1] > 65536 || tuning[2] < 0 || tuning[2] > 4096)
    return fail(SSOCT_EINVAL, "workgroup count out of range");
  if (tuning[3] != 0 && tuning[3] != 1) return fail(SSOCT_EINVAL, "order must be 0 or 1");
  if (tuning[4] != 0 && tuning[4] != 2 && tuning[4] != 4 && tuning[4] != 8)
    return fail(SSOCT_EINVAL, "rows per row group must be 0, 2, 4 or 8");
  int ct[3];
  col_tiles(p->N, ct);
  if (tuning[5] != 0 && tuning[5] != ct[0] && (tuning[5] != ct[1] || !ct[1]) && (tuning[5] != ct[2] || !ct[2]))
    return fail(SSOCT_EINVAL, "column tile width not available for this N");
  if (tuning[6] != 0 && tuning[6] != 16 && tuning[6] != 32 && tuning[6] != 64)
    return fail(SSOCT_EINVAL, "depth pixels per workgroup must be 0, 16, 32 or 64");
  if ((p->flags & SSOCT_DEPTH_4STEP) && tuning[6] == 64)
    return fail(SSOCT_EINVAL, "the factored depth form takes 16 or 32 pixels per workgroup");
  if (tuning[7] != 0 && (tuning[7] != p->dl.KC / 2 || tuning[7] < 32))
    return fail(SSOCT_EINVAL, "dense depth K chunk must be 0 or half the default chunk (at least 32 frames)");
  if (tuning[8] != 0 &&
      (tuning[8] != 1 || !has_radix_orders(p->N) || (p->flags & SSOCT_ANGULAR_SPECTRUM)))
    return fail(SSOCT_EINVAL, "radix order must be 0, or 1 for a Fresnel plan whose N is not a power of 16");
  if (p->streaming && tuning[3] != p->order) return fail(SSOCT_EINVAL, "the order is fixed while a stream uses the plan");
  p->F_run = tuning[0];
  p->col_grid = tuning[1];
  p->depth_grid = tuning[2];
  p->order = tuning[3];
  p->rpg_g = tuning[4];
  p->col_tile = tuning[5] == ct[0] ? 0 : tuning[5];
  p->dfft_px = tuning[6];
  p->depth_kc = tuning[7];
  p->col_radix = tuning[8];
  return SSOCT_OK;
}

int ssoct_plan_tune(ssoct_plan* p, const uint16_t* frames, const double* lambda, double pitch, double z,
                    const double* disp_phase, const double* zernike, void* workspace, size_t workspace_bytes,
                    void* vol, int* tuning) {
  WsLayout L;
  if (int rc = check_render_args(p, frames, workspace, workspace_bytes, vol, &L)) return rc;
  SSOCT_HIP(hipSetDevice(p->device));
  const int status = update_tables(p, lambda, pitch, z, disp_phase, zernike, false);
  if (status < 0) return status;
  std::string key;
  if (int rc = tune_key(p, &key)) return rc;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {   // shapes already timed for this device, size and form
      if (int rc = ssoct_plan_set_tuning(p, it->second.data())) return rc;
      if (tuning) ssoct_plan_get_tuning(p, tuning);
      return status;
    }
  }
  hipEvent_t ev[4];
  for (auto& e : ev) SSOCT_HIP(hipEventCreate(&e));
  auto measure = [&](float* stage_a, float* stage_b) -> int {
    float best_a = 1e30f, best_b = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      if (int rc = render_core(p, p->stream, frames, static_cast<char*>(workspace), L, vol, ev)) return rc;
      SSOCT_HIP(hipEventSynchronize(ev[3]));
      float a = 0, b = 0;
      SSOCT_HIP(hipEventElapsedTime(&a, ev[1], ev[2]));
      SSOCT_HIP(hipEventElapsedTime(&b, ev[2], ev[3]));
      if (p->depth_first()) std::swap(a, b);   // that order runs the depth stage first
      if (rep > 0) {  // first run warms caches and code
        best_a = a < best_a ? a : best_a;
        best_b = b < best_b ? b : best_b;
      }
    }
    *stage_a = best_a;
    *stage_b = best_b;
    return SSOCT_OK;
  };
  // Each search keeps the fastest candidate of its own stage (the Fresnel
  // stage, or the depth transform) before the next search starts; the first
  // candidate (the default) gives way only to one faster by more than 1 %,
  // so that run-to-run noise does not pick an alternative of equal speed.
  int rc = SSOCT_OK;
  float a, b;
  auto search = [&](int* knob, const int* cand, int n, bool stage_b) {
    int best_v = *knob;
    float best = 1e30f;
    for (int i = 0; i < n && rc == SSOCT_OK; ++i) {
      *knob = cand[i];
      rc = measure(&a, &b);
      const float t = stage_b ? b : a;
      if (rc == SSOCT_OK && (i == 0 ? t < best : t < 0.99f * best)) best = t, best_v = cand[i];
    }
    *knob = best_v;
  };
  // evaluation order (FFT form without frame-dependent factors) first: the whole render, both orders
  if (p->df_allowed) {
    float tot[2] = {1e30f, 1e30f};
    for (int o = 0; o < 2 && rc == SSOCT_OK; ++o) {
      p->order = o;
      rc = measure(&a, &b);
      tot[o] = a + b;
    }
    p->order = tot[0] < 0.99f * tot[1] ? 0 : 1;   // the default (depth first) unless the frame order is faster
  }
  const bool df = p->depth_first();   // the Fresnel-stage timings below are of that order's 2-D transforms
  // Fresnel stage: frames per chunk x column tile width x persistent column workgroups
  int ct[3];
  col_tiles(p->N, ct);
  // frames per chunk: the order's default (0) first, then F, F/2, F/4 where they differ from it
  const int Fs[3] = {p->F, p->F / 2, p->F / 4};
  p->F_run = 0;
  const int Fdef = p->frames_run();
  int nF = 1, Fc[4] = {0, 0, 0, 0};
  for (int i = 0; i < 3; ++i)
    if (Fs[i] >= 1 && Fs[i] != Fdef && Fs[i] != Fc[nF - 1] && (!df || Fs[i] >= 2)) Fc[nF++] = Fs[i];
  search(&p->F_run, Fc, nF, false);
  if (!(p->flags & SSOCT_ANGULAR_SPECTRUM)) {
    int tiles[3] = {0, ct[1], ct[2]}, nt = 1;
    if (ct[1]) ++nt;
    if (ct[2]) ++nt;
    search(&p->col_tile, tiles, nt, false);
    if (has_radix_orders(p->N)) {   // radix order of the column transforms
      const int Rx[2] = {0, 1};
      search(&p->col_radix, Rx, 2, false);
    }
  }
  {
    const int c0 = (p->flags & SSOCT_ANGULAR_SPECTRUM) ? p->as_col_grid0 : col_default_grid(p->N, p->cu, p->col_tile);
    const int Cs[3] = {0, 2 * c0, 4 * c0};
    search(&p->col_grid, Cs, 3, false);
  }
  if (df) {
    const int Rs[4] = {0, 8, 4, 2};
    search(&p->rpg_g, Rs, 4, false);
  }
  // depth transform: pixels per workgroup of the FFT form (frame order), or
  // the persistent grid of the dense product
  if ((p->flags & SSOCT_DEPTH_FFT) && !df) {
    const int Ps[3] = {0, 16, 64};
    search(&p->dfft_px, Ps, 3, true);
  } else if (p->flags & SSOCT_DEPTH_4STEP) {
    const int Ps[2] = {0, 16};
    search(&p->dfft_px, Ps, 2, true);
  } else if (!(p->flags & (SSOCT_DEPTH_FFT | SSOCT_DEPTH_4STEP))) {
    const int d0 = depth_grid(p->T, p->N * p->N, p->cu, p->general);
    const int Ds[2] = {0, 2 * d0 <= 4096 ? 2 * d0 : d0};
    search(&p->depth_grid, Ds, 2, true);
    if (p->dl.KC / 2 >= 32) {
      const int Ks[2] = {0, p->dl.KC / 2};
      search(&p->depth_kc, Ks, 2, true);
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc != SSOCT_OK) return rc;
  {
    std::array<int, SSOCT_TUNING_LEN> t{};
    ssoct_plan_get_tuning(p, t.data());
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = t;
  }
  if (tuning) ssoct_plan_get_tuning(p, tuning);
  return status;
}

int ssoct_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache.clear();
  return SSOCT_OK;
}

}  // extern "C"
