/*
 * ssoct.h -- C ABI of the MI355X (gfx950) renderer for swept-source optical
 * coherence tomography by off-axis Fresnel-transform digital holography
 * (Charpentier et al., arXiv 2003.08960).
 *
 * Pipeline of one render (ssoct_render, ssoct_plan_render; flowchart of Fig. 3):
 *   1. chromatic rescale of each 16-bit interferogram by linear interpolation,
 *      I'(x, y, t) = I(x lambda_t / lambda_1, y lambda_t / lambda_1, t)
 *      about the frame centre (Eq. 5; makes the Fresnel pixel of Eq. 4
 *      wavelength independent)
 *   2. discrete Fresnel transform with lambda_1 for every frame (Eq. 6):
 *      chirp exp(-i pi d^2 c^2 / (lambda_1 z)) on the sensor grid, then the
 *      centred, positive-exponent, unnormalised 2-D DFT
 *   3. DFT along the sweep over one rectangular gate of all T frames
 *      (Eq. 7): V[q] = sum_t h_t exp(-2 pi i q t / T), natural bin order
 *   4. envelope |V| and three orthogonal cuts (text after Eq. 7)
 *
 * lambda_1 is the longest wavelength of the sweep (the start wavelength of
 * the paper's sweep).  Optional extensions: a per-frame dispersion phase
 * exp(i phi_t) on h_t, an aberration screen exp(i sum_j c_j Z_j) (ANSI/OSA
 * Zernike j = 0..14, orthonormal, rho = r / (N d / sqrt 2)) on the rescaled
 * frame, and the gradient of the sharpness loss sum |V|^4 with respect to z,
 * c and phi.
 *
 * Conventions for every entry point:
 *   - Arrays named frames, vol, grad_vol, cut_*, workspace and grad_out are
 *     DEVICE pointers on the plan's device, owned by the caller; lambda,
 *     disp_phase and zernike are HOST arrays read before the call returns.
 *   - frames: uint16 [T][N][N], row-major (t, y, x).
 *   - vol: complex64 [T][N][N] = interleaved float (re, im), index (q, u, v)
 *     with u = row (y), v = column (x); or float [T][N][N] = |V| when the plan
 *     has SSOCT_WRITE_ABS.
 *   - All work is enqueued asynchronously on the plan's stream; nothing is
 *     synchronised.  A plan is not thread safe: use one plan per thread.
 *   - Return value: SSOCT_OK (0), a warning (> 0, the result is computed) or
 *     an error (< 0, nothing was enqueued).  ssoct_last_error() gives the
 *     text of the last error of the calling thread.  No C++ exception
 *     crosses this interface.
 */
#ifndef SSOCT_H
#define SSOCT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSOCT_VERSION 1

/* status codes */
#define SSOCT_OK 0
#define SSOCT_WARN_UNDERSAMPLED 1 /* |z| < z_b = N d^2 / lambda_1 (validity bound after Eq. 6) */
#define SSOCT_EINVAL (-1)         /* null pointer, bad size, lambda <= 0, z == 0, non-finite value */
#define SSOCT_EUNSUPPORTED (-2)   /* N not a power of two in [16, 2048], T not in [1, 1024], option not available */
#define SSOCT_EHIP (-3)           /* HIP runtime error (text in ssoct_last_error) */
#define SSOCT_ENOMEM (-4)         /* device allocation failed, or workspace too small */
#define SSOCT_EALIAS (-5)         /* output overlaps an input or the workspace */
#define SSOCT_EDROPPED (-6)       /* streaming: a frame-sequence gap or a full ring; the incomplete sweep was discarded */
#define SSOCT_EAGAIN (-7)         /* streaming: no finished volume yet (non-blocking pop) or no free slot */

/* plan flags */
#define SSOCT_PREC_FP32 0u        /* depth transform on FP32 MFMA */
#define SSOCT_PREC_FP16 1u        /* depth transform on FP16 MFMA, FP32 accumulation */
#define SSOCT_PREC_BF16 2u        /* depth transform on BF16 MFMA, FP32 accumulation */
#define SSOCT_PREC_MASK 3u
#define SSOCT_SPLIT 4u            /* FP16/BF16 operands split hi + lo (3 products) */
#define SSOCT_CHIRP_EXACT 8u      /* chirp rate pi d^2 (lambda_t/lambda_1) / (lambda_1 z) instead of lambda_1 only */
#define SSOCT_EQ6_PHASE 16u       /* apply the Eq. 6 prefactor (i d^2/(lambda_1 z)) e^{-i k_1 z} and output phase */
#define SSOCT_WRITE_ABS 32u       /* ssoct_plan_render writes |V| (float) instead of V (complex64) */
#define SSOCT_CUT_POWER 64u       /* ssoct_cuts returns |V|^2 instead of |V| */
#define SSOCT_BACKWARD 128u       /* workspace also sized for the gradient entry points */
#define SSOCT_PROFILE 256u        /* record per-stage HIP events (ssoct_profile_read) */
#define SSOCT_PROFILE_KERNELS 512u /* with SSOCT_PROFILE: an event after every Fresnel-stage launch too
                                      (each adds a few microseconds to the render) */
#define SSOCT_ANGULAR_SPECTRUM 4096u /* propagate each frame by the angular spectrum at its own wavelength
                                      (no rescale, sensor pitch, valid for any z) instead of Eq. 6:
                                      F^-1{F{I_t} exp(-2 pi i z sqrt(lambda_t^-2 - f^2))}, the sign of
                                      Eq. 6 (fields carry exp(+i omega t)), so one z names the same plane
                                      for both propagators; not with SSOCT_CHIRP_EXACT, SSOCT_EQ6_PHASE,
                                      aberration or gradients */
#define SSOCT_NONUNIFORM_K 2048u  /* depth transform exp(-2 pi i q kappa_t / T), kappa_t = (k_t - k_0)/dk from lambda:
                                      the uniform depth grid of a sweep not linear in k (dense forms only) */
#define SSOCT_DEPTH_FFT 1024u     /* FP32 depth transform as a radix FFT along the sweep (T in {16..256},
                                      powers of two) instead of the dense DFT-matrix product */
#define SSOCT_DEPTH_4STEP 8192u   /* depth transform of Eq. 7 factored as T = 16 (T/16): two small DFT-matrix
                                      products on MFMA with a twiddle between them, in the precision the
                                      other flags select (T in {32, 64, 128, 256}; not with SSOCT_DEPTH_FFT
                                      or SSOCT_NONUNIFORM_K) */

typedef struct ssoct_plan ssoct_plan;

/* Library version (SSOCT_VERSION). */
int ssoct_version(void);

/* Text of the last error returned to the calling thread ("" if none). */
const char* ssoct_last_error(void);

/* Bytes of device workspace ssoct_plan_render (and, with SSOCT_BACKWARD, the
 * gradient entry points) need for T frames of N x N; 0 for unsupported
 * sizes.  The workspace holds the hologram stack H (T N^2 x 8 bytes), one
 * chunk of row-transformed frames, and with SSOCT_BACKWARD a second stack and
 * the FP64 reduction partials. */
size_t ssoct_workspace_size(int T, int N, uint32_t flags);

/* Create a plan for T frames of N x N on the current HIP device, enqueuing
 * its work on `stream` (0 = null stream).  Allocates the small FP64-derived
 * tables (twiddles, depth DFT matrix in MFMA register order; O(T N + T^2)).
 * On error *plan is NULL. */
int ssoct_plan_create(ssoct_plan** plan, int T, int N, uint32_t flags, hipStream_t stream);

/* Change the stream of a plan. */
int ssoct_plan_set_stream(ssoct_plan* plan, hipStream_t stream);

/* Release a plan (waits for its stream). NULL is accepted.  SSOCT_EINVAL (and
 * nothing released) while a stream or sliding-window object uses the plan:
 * destroy those first. */
int ssoct_plan_destroy(ssoct_plan* plan);

/* The paper's problem statement as one call (Eq. 5-7): the interferograms of
 * one sweep, their wavelengths, the pixel pitch and the reconstruction
 * distance in; the complex volume out (steps 1-3).
 *   frames  device uint16 [T][N][N]
 *   T, N    frames per sweep (1 .. 1024) and frame size (power of two, 16 .. 2048)
 *   lambda  host double [T], metres, > 0 (any order; lambda_1 = max)
 *   pitch   sensor pixel pitch d, metres, > 0
 *   z       reconstruction distance, metres, != 0
 *   vol     device complex64 [T][N][N] (q, u, v), must not overlap frames
 *   stream  HIP stream the work is enqueued on (0 = null stream)
 * FP32 throughout (the depth transform as a radix FFT for T in {16, 32, 64,
 * 128, 256}, else the dense DFT-matrix product on FP32 MFMA), no dispersion
 * or aberration, rectangular gate.  The plan and its workspace (about
 * T N^2 8 bytes plus one chunk of at most 128 MiB) are created on the first
 * call for a (device, stream, T, N) and reused by later calls with the same
 * four; they are released by ssoct_render_release.  Returns as
 * ssoct_plan_render (SSOCT_WARN_UNDERSAMPLED when |z| < N d^2 / lambda_1).
 * Safe to call from several threads (the cache is locked); calls on one stream
 * share a workspace and run in stream order. */
int ssoct_render(const uint16_t* frames, int T, int N, const double* lambda, double pitch, double z, void* vol,
                 hipStream_t stream);

/* Release every plan and workspace ssoct_render has cached (waits for each
 * device they were made on).  No ssoct_render call may be in flight on
 * another thread. */
int ssoct_render_release(void);

/* Render one sweep with an explicit plan: frames [T][N][N] uint16 -> vol
 * [T][N][N] (steps 1-3), in the plan's precision and depth form.
 *   lambda     host double [T], metres, > 0 (any order; lambda_1 = max)
 *   pitch      sensor pixel pitch d, metres, > 0
 *   z          reconstruction distance, metres, != 0
 *   disp_phase host double [T] radians, or NULL (zero)
 *   zernike    host double [15] radians, or NULL (no aberration)
 *   workspace  device, at least ssoct_workspace_size(T, N, flags) bytes
 * Rescale/chirp tables are rebuilt (FP64 on the GPU) only when lambda, pitch,
 * z, disp_phase or zernike change between calls. */
int ssoct_plan_render(ssoct_plan* plan, const uint16_t* frames, const double* lambda, double pitch, double z,
                      const double* disp_phase, const double* zernike, void* workspace, size_t workspace_bytes,
                      void* vol);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * render as ssoct_plan_render, with the workspace taken from a device array
 * of SSOCT_NOALLOC_SCRATCH_BYTES inside the library instead of an argument.
 * It calls no allocating routine (the plan's tables exist since
 * ssoct_plan_create).  The plan's frames per chunk are lowered as far as
 * needed to fit the array (the result does not change); SSOCT_EUNSUPPORTED
 * when even one frame per chunk does not fit (T N^2 8 bytes plus N^2 8 bytes
 * beyond the array, e.g. T = 256, N = 1024).  Each GPU the call runs on holds
 * the array until the process ends, and every call on that GPU shares it:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * on it; calls on one stream are ordered.  Nothing in it needs clearing (a
 * render writes every workspace byte it reads).  No profiling events. */
#define SSOCT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int ssoct_plan_render_noalloc(ssoct_plan* plan, const uint16_t* frames, const double* lambda, double pitch, double z,
                              const double* disp_phase, const double* zernike, void* vol);

/* Three orthogonal cuts of the envelope (step 4) of a complex64 volume:
 *   cut_xy[u][v] = M[q0][u][v]   float [N][N]
 *   cut_xz[q][v] = M[q][y0][v]   float [T][N]
 *   cut_yz[q][u] = M[q][u][x0]   float [T][N]
 * with M = |V| (|V|^2 with SSOCT_CUT_POWER); 0 <= x0, y0 < N, 0 <= q0 < T. */
int ssoct_cuts(ssoct_plan* plan, const void* vol, int x0, int y0, int q0, float* cut_xy, float* cut_xz,
               float* cut_yz);

/* Vector-Jacobian product of ssoct_plan_render for a real loss L with
 * dL = Re sum conj(G) dV, G = grad_vol (complex64 [T][N][N], PyTorch's
 * convention G = 2 dL/d conj(V)).  Writes device double grad_out[2 + 15 + T]:
 * [0] = 0, [1] = dL/dz, [2..16] = dL/dc_j, [17..17+T) = dL/dphi_t.
 * The forward transform is not needed: the rescaled, chirped frames are
 * recomputed inside the adjoint.  Any precision and depth form (the adjoint
 * always runs in FP32: its depth transforms are radix FFTs for T in {16, 32,
 * 64, 128, 256}, else dense FP32 products); a workspace sized with
 * SSOCT_BACKWARD; SSOCT_EQ6_PHASE is not supported (SSOCT_EUNSUPPORTED). */
int ssoct_backward(ssoct_plan* plan, const uint16_t* frames, const double* lambda, double pitch, double z,
                   const double* disp_phase, const double* zernike, const void* grad_vol, void* workspace,
                   size_t workspace_bytes, double* grad_out);

/* Sharpness loss L = sum |V|^4 and its gradient in one call: recomputes the
 * FP32 forward, forms G = 4 |V|^2 V with a power-of-two rescaling that keeps
 * it finite in FP32, and runs the adjoint; the volume is never stored.
 * grad_out as for ssoct_backward with grad_out[0] = L (FP64 accumulation). */
int ssoct_backward_sharpness(ssoct_plan* plan, const uint16_t* frames, const double* lambda, double pitch,
                             double z, const double* disp_phase, const double* zernike, void* workspace,
                             size_t workspace_bytes, double* grad_out);

/* Apodising gate g_t (host [T] real weights, or NULL for the rectangular gate
 * of Eq. 7): h_t is multiplied by g_t before the depth transform.  Kept in
 * the plan until changed; fails while a stream or sliding window uses the
 * plan.  Not available for the gradient entry points or sliding windows. */
int ssoct_plan_set_gate(ssoct_plan* plan, const double* gate);

/* With SSOCT_PROFILE every ssoct_plan_render records HIP events on the plan's
 * stream around its stages (and, with SSOCT_PROFILE_KERNELS, after every
 * kernel launch of the Fresnel stage).  This call waits for the last recorded render and fills ms[6] with
 * the mean elapsed milliseconds per render over the renders recorded since
 * the previous call (at most the last 64): ms[0] tables, ms[1] Fresnel stage
 * (rescale + chirp + 2-D DFT, all frame chunks), ms[2] depth transform (one
 * launch), ms[3] the number of renders averaged, ms[4] all row-pass launches,
 * ms[5] all column-pass launches (ms[4] and ms[5] are -1 without
 * SSOCT_PROFILE_KERNELS or when a render had more than 64 frame chunks).
 * Resets the record. */
int ssoct_profile_read(ssoct_plan* plan, float* ms);

/* ---------------------------------------------------------------- tuning
 * Launch-shape parameters of a plan, int tuning[SSOCT_TUNING_LEN]:
 *   [0] frames per chunk of the Fresnel stage (1 .. the chunk the workspace
 *       was sized for; in the depth-first order two transforms per bin, so
 *       half as many bins per chunk).  0 = default of the evaluation order in
 *       use: min(T, 128 MiB / (8 N^2)) frames in the frame order (16 at
 *       N = 1024), min(T, 256 MiB / (8 N^2)) in the depth-first order (32,
 *       i.e. 16 bins); SSOCT_DEPTH_FFT plans size the workspace for the
 *       larger, other plans for the first.
 *   [1] persistent column-pass workgroups (0 = default: as many as are
 *       resident at once on the device wherever the column pass prefetches
 *       its next tile, which is the angular-spectrum column pass at every N
 *       and the Fresnel column pass up to N = 1024; 512 for the Fresnel
 *       column pass at N = 2048)
 *   [2] persistent workgroups of the dense depth transform (0 = default; the
 *       SSOCT_DEPTH_FFT and SSOCT_DEPTH_4STEP forms launch one workgroup per
 *       pixel tile and ignore it)
 *   [3] evaluation order of the SSOCT_DEPTH_FFT form (0 = Fresnel transform
 *       of every frame, then the depth transform; 1 = default: depth
 *       transform of the rescaled real frames first, then one Fresnel
 *       transform per bin, which by linearity is the same map when the chirp
 *       and the per-frame factor do not depend on the frame: no
 *       SSOCT_CHIRP_EXACT, no dispersion, no SSOCT_WRITE_ABS, no gate;
 *       otherwise the frame order is used)
 *   [4] rows per row group of the depth-first order's row pass (0 = 4 where
 *       that gives at least two workgroups per CU, else 2; 2, 4 or 8)
 *   [5] column tile width of the Fresnel column passes (0 = default, 16
 *       adjacent columns up to N = 1024; N >= 512 also takes 1/2 and 1/4 of
 *       the default; the adjoint keeps the default)
 *   [6] pixels per workgroup of the FFT-form depth transform (0 = default 32;
 *       16, 32 or 64) or of the factored MFMA form (SSOCT_DEPTH_4STEP;
 *       0 = default 32; 16 or 32)
 *   [7] frames per K chunk of the dense depth product (0 = default, the
 *       smallest of 32, 64, 128, 256 that covers T; or half of it, at least
 *       32: the same products in the same order, with half the matrix
 *       operands held per lane)
 *   [8] radix order of the forward Fresnel column transforms (0 = default:
 *       the radix-16 passes first and the radix-2, 4 or 8 pass last, 16 16 4
 *       at N = 1024; 1 = the small radix first, 4 16 16, which leaves the
 *       output in natural order in registers at the price of twiddles on
 *       every radix-16 pass).  Only N that is not a power of 16 (32, 64, 128,
 *       512, 1024, 2048) has the second order; angular-spectrum plans and the
 *       adjoint keep the default.
 * [3] and [8] change the rounding only (the same transforms, within the
 * same error bars); every other entry changes speed only, never results. */
#define SSOCT_TUNING_LEN 9

/* Time candidate launch shapes (the evaluation order where allowed, then the
 * Fresnel stage's frames per chunk, column tile width, radix order of the
 * column transforms, column workgroups and,
 * in the depth-first order, rows per row group; then the depth transform's
 * pixels per workgroup (FFT and factored forms) or workgroups and K chunk
 * (dense form)) on the given
 * inputs with HIP events on the plan's stream (synchronises the stream),
 * keep the fastest of each in the plan (the default, tried first, gives way
 * only to a value faster by more than 1 %) and write them to tuning.  Arguments
 * as for ssoct_plan_render; vol is overwritten.
 * The choice is kept in a process-wide cache keyed by the device's
 * architecture and CU count, T, N, the plan flags (the profiling flags
 * aside) and whether the depth-first order and the aberration factor apply
 * to these inputs; a later call with the same key applies the cached shapes
 * without timing anything (vol is then left untouched). */
int ssoct_plan_tune(ssoct_plan* plan, const uint16_t* frames, const double* lambda, double pitch, double z,
                    const double* disp_phase, const double* zernike, void* workspace, size_t workspace_bytes,
                    void* vol, int* tuning);

/* Empty the tuning cache of ssoct_plan_tune: the next call times again.
 * Always SSOCT_OK. */
int ssoct_tune_cache_clear(void);

/* Read or set the launch-shape parameters (e.g. from a tuning cache);
 * SSOCT_TUNING_LEN entries. */
int ssoct_plan_get_tuning(const ssoct_plan* plan, int* tuning);
int ssoct_plan_set_tuning(ssoct_plan* plan, const int* tuning);

/* ---------------------------------------------------------------- streaming
 * Continuous rendering of consecutive sweeps (one volume per T frames) with
 * a ring of `slots` volume slots.  Each slot owns device memory for one
 * sweep of frames, a workspace, the complex volume and the three cuts, a HIP
 * stream, and HIP graphs captured once at creation with the plan's launch
 * shapes at that time: the whole volume (render + cuts + copy of the cuts to
 * pinned host memory), the Fresnel stage of each chunk of frames, and the
 * depth transform + cuts + copy.  Successive volumes overlap (the depth
 * transform of one with the Fresnel stage of the next).  Host-fed frames
 * start each chunk's Fresnel stage as soon as the chunk has landed, so a
 * volume's latency after its last frame is about one chunk plus the depth
 * transform; a device-filled slot is one graph launch.  The model is the
 * buffered camera acquisition of the real-time system described after Eq. 7,
 * which keeps every sweep whole for the depth transform.  Physical parameters (lambda, pitch, z, disp_phase,
 * zernike) and cut positions are fixed for the stream; the plan must not be
 * used concurrently by other calls while the stream exists.  A stream object
 * is safe to use from two threads (a producer pushing, a consumer popping). */
typedef struct ssoct_stream ssoct_stream;

int ssoct_stream_create(ssoct_stream** stream, ssoct_plan* plan, const double* lambda, double pitch, double z,
                        const double* disp_phase, const double* zernike, int slots, int x0, int y0, int q0);

/* Host-fed input: frames [nframes][N][N] in host memory (pinned memory gives
 * asynchronous DMA; pageable memory is staged), with sequence numbers
 * first_seq, first_seq + 1, ...  Frame seq belongs to sweep seq / T at
 * position seq % T.  A sweep is rendered when its T frames have arrived in
 * order.  A gap in the sequence, or a sweep that starts while every slot is
 * in flight, discards the incomplete sweep and skips frames up to the next
 * sweep start (seq % T == 0): the call then returns SSOCT_EDROPPED (after
 * having accepted every other frame).  The host buffer must stay unchanged
 * until the volume that contains its frames has been popped. */
int ssoct_stream_push_frames(ssoct_stream* stream, const uint16_t* host_frames, int nframes, uint64_t first_seq);

/* Device-resident input: take a free slot (SSOCT_EAGAIN if none) and get its
 * device frame buffer [T][N][N]; fill it (any stream, synchronised before
 * submit), then submit it as sweep `volume_seq`. */
int ssoct_stream_acquire(ssoct_stream* stream, int* slot, uint16_t** device_frames);
int ssoct_stream_submit(ssoct_stream* stream, int slot, uint64_t volume_seq);

/* Oldest rendered volume, in submission order.  wait != 0 blocks until it is
 * finished, wait == 0 returns SSOCT_EAGAIN if it is not.  Copies the cuts
 * (host float [N][N], [T][N], [T][N]; any may be NULL) and returns the sweep
 * number, the slot that rendered it, and the latency from submission (last
 * frame pushed) to the end of its graph on the GPU, in ms.  Every output
 * pointer may be NULL.  SSOCT_EAGAIN when nothing is in flight. */
int ssoct_stream_pop(ssoct_stream* stream, int wait, uint64_t* volume_seq, int* slot, float* cut_xy,
                     float* cut_xz, float* cut_yz, double* latency_ms);

/* Device complex volume of a slot (valid between its pop and the slot's reuse). */
int ssoct_stream_slot_volume(ssoct_stream* stream, int slot, const void** device_volume);

/* counters[0] volumes completed, [1] frames dropped, [2] sweeps dropped, [3] volumes in flight */
int ssoct_stream_stats(ssoct_stream* stream, uint64_t* counters);

/* Wait for every volume in flight and release the stream. NULL is accepted. */
int ssoct_stream_destroy(ssoct_stream* stream);

/* ---------------------------------------------------------------- sliding windows
 * The short-time Fourier transform of Eq. 7 over a continuous frame stream:
 * a rectangular gate of T consecutive holograms advanced by `hop` frames
 * (the paper's real-time mode: hop ~13 turns 512 frames/s into ~38 volumes
 * per second).  Every frame is rescaled and Fresnel-transformed once into
 * slot seq % T of a ring of holograms (sweep position seq % T selects
 * lambda, disp_phase and the tables); the window starting at frame j is the
 * DFT of frames j .. j + T - 1 in time order, read from the ring in rotated
 * order (or, for the dense depth product, transformed in slot order with bin
 * q multiplied by exp(+2 pi i q (j % T) / T), the same thing for a circular
 * DFT).  A window is emitted every `hop` frames once T consecutive frames
 * have arrived: depth transform, cuts and copy of the cuts to pinned host
 * memory, into one of `slots` output volumes.  Frames and kernels run in
 * order on one stream owned by the object, the copies of the cuts on a
 * second one.  Windows never span a gap in the frame sequence: a gap
 * restarts the run (the call returns SSOCT_EDROPPED), and a window that finds
 * every output volume still held is dropped and counted.  The plan's
 * parameters are fixed while the object exists; the SSOCT_DEPTH_FFT form
 * always uses the frame order here. */
typedef struct ssoct_slide ssoct_slide;

int ssoct_slide_create(ssoct_slide** slide, ssoct_plan* plan, const double* lambda, double pitch, double z,
                       const double* disp_phase, const double* zernike, int hop, int slots, int x0, int y0, int q0);

/* Host-fed frames [nframes][N][N] (pinned memory is copied asynchronously;
 * keep the buffer unchanged until a later call has returned a window that
 * contains them, or until ssoct_slide_destroy), sequence numbers first_seq,
 * first_seq + 1, ... (non-decreasing across calls). */
int ssoct_slide_push(ssoct_slide* slide, const uint16_t* host_frames, int nframes, uint64_t first_seq);

/* Device-resident input: the frame ring [T][N][N] (frame seq at slot
 * seq % T).  The caller writes frames there and then calls
 * ssoct_slide_advance, ordering its writes before that call; a slot must not
 * be rewritten while an earlier frame in it may still be unprocessed
 * (synchronise with the windows it belongs to). */
int ssoct_slide_ring(ssoct_slide* slide, uint16_t** device_ring);
int ssoct_slide_advance(ssoct_slide* slide, int nframes, uint64_t first_seq);

/* Oldest finished window: its first frame, output slot, cuts (host, N*N and
 * 2 T*N floats, or NULL) and latency from the arrival of its last frame to
 * completion.  wait = 0 returns SSOCT_EAGAIN when it is not finished; also
 * SSOCT_EAGAIN when no window is in flight.  The slot's volume stays valid
 * until a later window reuses it. */
int ssoct_slide_pop(ssoct_slide* slide, int wait, uint64_t* window_start, int* slot, float* cut_xy, float* cut_xz,
                    float* cut_yz, double* latency_ms);
int ssoct_slide_volume(ssoct_slide* slide, int slot, const void** device_volume);

/* counters[5]: windows done, windows dropped (no free output volume), frames
 * transformed, run restarts (sequence gaps), windows in flight. */
int ssoct_slide_stats(ssoct_slide* slide, uint64_t* counters);
int ssoct_slide_destroy(ssoct_slide* slide);

#ifdef __cplusplus
}
#endif

#endif /* SSOCT_H */
