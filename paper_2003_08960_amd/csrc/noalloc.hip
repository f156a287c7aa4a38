// Render entry point that allocates nothing: the workspace of the render
// (hologram stack and one chunk of row-transformed frames) lives in a
// file-scope device array instead of a caller-provided buffer.  For callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).
#include <mutex>

#include "plan.hpp"

namespace ssoct {

// Every GPU on which the entry point runs holds this array (256 MiB) until
// the process ends; its address there is queried once per device.
constexpr size_t STATIC_SCRATCH_BYTES = SSOCT_NOALLOC_SCRATCH_BYTES;
static_assert(STATIC_SCRATCH_BYTES % 256 == 0, "the scratch array holds 256-byte aligned workspace regions");
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device `dev`, which must be current.  The
// array's name is a host-side stand-in; only this address may reach a kernel.
int scratch_on(int dev, char** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(SSOCT_EUNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(SSOCT_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return SSOCT_OK;
}

bool spans_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

}  // namespace
}  // namespace ssoct

using namespace ssoct;

extern "C" int ssoct_plan_render_noalloc(ssoct_plan* p, const uint16_t* frames, const double* lambda, double pitch,
                                         double z, const double* disp_phase, const double* zernike, void* vol) {
  if (int rc = check_plan(p)) return rc;
  if (!frames || !vol) return fail(SSOCT_EINVAL, "frames and vol must be non-NULL");
  const int T = p->T, N = p->N;
  // the plan's frames per chunk, reduced until the workspace fits the array
  // (the chunking changes the speed only, never the result)
  int F = p->frames_run();
  WsLayout L = ws_layout(T, N, p->flags & ~SSOCT_BACKWARD, F);
  while (F > 1 && L.total > STATIC_SCRATCH_BYTES) L = ws_layout(T, N, p->flags & ~SSOCT_BACKWARD, --F);
  if (L.total > STATIC_SCRATCH_BYTES)
    return fail(SSOCT_EUNSUPPORTED, "the render workspace of T x N x N exceeds the 256 MiB static scratch array");
  const size_t vol_bytes = (size_t)T * N * N * ((p->flags & SSOCT_WRITE_ABS) ? 4 : 8);
  if (spans_overlap(vol, vol_bytes, frames, (size_t)T * N * N * 2)) return fail(SSOCT_EALIAS, "vol overlaps frames");
  SSOCT_HIP(hipSetDevice(p->device));
  char* ws = nullptr;
  if (int rc = scratch_on(p->device, &ws)) return rc;
  const int status = update_tables(p, lambda, pitch, z, disp_phase, zernike, false);
  if (status < 0) return status;
  // nothing in the workspace has to start at zero: every byte a kernel reads
  // was written earlier in the same render
  const int saved = p->F_run;
  p->F_run = F;
  const int rc = render_core(p, p->stream, frames, ws, L, vol, nullptr, nullptr);
  p->F_run = saved;
  return rc ? rc : status;
}
