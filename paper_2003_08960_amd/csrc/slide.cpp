// Sliding-window depth transform over a continuous frame stream
// (ssoct_slide_*): the short-time Fourier transform of Eq. 7 with a
// rectangular gate of T consecutive holograms advanced by `hop` frames.
//
// Every frame is rescaled and Fresnel-transformed once, into slot
// seq mod T of a ring of holograms (the tables are indexed by sweep
// position, so slot p always holds a frame recorded at lambda_p).  A window
// starting at frame j holds slots j mod T .. j mod T - 1 in time order: the
// FFT and factored depth kernels read slot (t + j) mod T as frame t; the
// dense product transforms the ring in slot order and multiplies bin q by
// exp(+2 pi i q (j mod T) / T) (the same for a circular DFT).  A depth
// transform and the cuts are launched every `hop` frames into one of `slots`
// output volumes; the cuts' copy to pinned host memory runs on a second
// stream after an event, overlapping the next window.  Frames and kernels
// run in order on the first stream, so a ring slot is never overwritten
// before the transforms that read it.
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>

#include "plan.hpp"

using namespace ssoct;

namespace {

int64_t slide_now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct OutSlot {
  float2* vol = nullptr;     // device volume of one window
  float* cuts = nullptr;     // device cuts xy | xz | yz
  float* hcuts = nullptr;    // pinned host copy of the cuts
  hipEvent_t ready = nullptr;  // volume and device cuts complete (compute stream)
  hipEvent_t done = nullptr;   // host cuts complete too (copy stream)
  bool busy = false;
  uint64_t start = 0;        // first frame of the window
  int64_t t_submit = 0;
  std::atomic<int64_t> t_done{0};
};

void slide_stamp(void* arg) { static_cast<OutSlot*>(arg)->t_done.store(slide_now_ns()); }

}  // namespace

struct ssoct_slide {
  ssoct_plan* plan = nullptr;
  int hop = 1, nslot = 0, x0 = 0, y0 = 0, q0 = 0;
  hipStream_t s = nullptr;    // transfers of frames and all kernels
  hipStream_t cs = nullptr;   // copies of the cuts to the host, overlapping the next window
  uint16_t* ring = nullptr;  // raw frames [T][N][N] by sweep position
  char* ws = nullptr;        // workspace: hologram ring (H) and chunk buffer
  WsLayout L{};
  std::unique_ptr<OutSlot[]> out;
  std::mutex m;
  bool have = false;         // a run of consecutive frames is in progress
  uint64_t expect = 0;       // next frame of the run
  uint64_t run_start = 0;    // first frame of the run
  std::deque<int> inflight;
  uint64_t n_done = 0, n_drop = 0, n_frames = 0, n_restart = 0;
};

namespace {

void slide_free(ssoct_slide* sl) {
  if (!sl) return;
  if (sl->s) (void)hipStreamSynchronize(sl->s);
  if (sl->cs) (void)hipStreamSynchronize(sl->cs);
  if (sl->out) {
    for (int k = 0; k < sl->nslot; ++k) {
      OutSlot& o = sl->out[k];
      if (o.ready) (void)hipEventDestroy(o.ready);
      if (o.done) (void)hipEventDestroy(o.done);
      (void)hipFree(o.vol);
      (void)hipFree(o.cuts);
      if (o.hcuts) (void)hipHostFree(o.hcuts);
    }
  }
  (void)hipFree(sl->ring);
  (void)hipFree(sl->ws);
  if (sl->s) (void)hipStreamDestroy(sl->s);
  if (sl->cs) (void)hipStreamDestroy(sl->cs);
  if (sl->plan) sl->plan->streaming = false;
  delete sl;
}

// depth transform of the ring for the window starting at frame j, cuts, copy
int emit(ssoct_slide* sl, uint64_t j) {
  ssoct_plan* p = sl->plan;
  const int T = p->T, N = p->N;
  int k = -1;
  for (int i = 0; i < sl->nslot; ++i)
    if (!sl->out[i].busy) {
      k = i;
      break;
    }
  if (k < 0) {  // every output volume is still held: this window is lost
    sl->n_drop += 1;
    return SSOCT_OK;
  }
  OutSlot& o = sl->out[k];
  o.busy = true;
  o.start = j;
  o.t_done.store(0);
  o.t_submit = slide_now_ns();
  if (int rc = render_depth(p, sl->s, sl->ws, sl->L, o.vol, (int)(j % (uint64_t)T))) return rc;
  float* c = o.cuts;
  const size_t ncut = (size_t)N * N + 2 * (size_t)T * N;
  SSOCT_HIP(launch_cuts(T, N, o.vol, sl->x0, sl->y0, sl->q0, (p->flags & SSOCT_CUT_POWER) ? 1 : 0, c,
                        c + (size_t)N * N, c + (size_t)N * N + (size_t)T * N, sl->s));
  // the host copy runs on the copy stream while the next window is transformed
  SSOCT_HIP(hipEventRecord(o.ready, sl->s));
  SSOCT_HIP(hipStreamWaitEvent(sl->cs, o.ready, 0));
  SSOCT_HIP(hipMemcpyAsync(o.hcuts, c, ncut * sizeof(float), hipMemcpyDeviceToHost, sl->cs));
  SSOCT_HIP(hipLaunchHostFunc(sl->cs, slide_stamp, &o));
  SSOCT_HIP(hipEventRecord(o.done, sl->cs));
  sl->inflight.push_back(k);
  return SSOCT_OK;
}

// frames [first, first + n) are (or are being copied) in their ring slots on
// the stream: Fresnel stage in segments that end at ring wraps, chunk limits
// and window ends, emitting each window as its last frame is transformed
int advance(ssoct_slide* sl, int n, uint64_t first, const uint16_t* host) {
  ssoct_plan* p = sl->plan;
  const int T = p->T;
  const size_t fpx = (size_t)p->N * p->N;
  int rc = SSOCT_OK;
  if (!sl->have || first != sl->expect) {  // a new run: windows restart at its first frame
    if (sl->have) {
      sl->n_restart += 1;
      rc = SSOCT_EDROPPED;
    }
    sl->have = true;
    sl->run_start = first;
  }
  uint64_t seq = first;
  const uint64_t end = first + (uint64_t)n;
  while (seq < end) {
    const int pos = (int)(seq % (uint64_t)T);
    uint64_t stop = end;
    stop = stop < seq + (uint64_t)(T - pos) ? stop : seq + (uint64_t)(T - pos);   // ring wrap
    const uint64_t fr = (uint64_t)p->frames_run_frame();
    stop = stop < seq + fr ? stop : seq + fr;     // chunk buffer
    // next window end at or after seq: frame e with e + 1 - T >= run_start and (e + 1 - T - run_start) % hop == 0
    const uint64_t first_end = sl->run_start + (uint64_t)T - 1;
    uint64_t wend = first_end;
    if (seq > first_end) {
      const uint64_t steps = (seq - first_end + (uint64_t)sl->hop - 1) / (uint64_t)sl->hop;
      wend = first_end + steps * (uint64_t)sl->hop;
    }
    if (wend + 1 < stop) stop = wend + 1;
    const int cnt = (int)(stop - seq);
    if (host)
      SSOCT_HIP(hipMemcpyAsync(sl->ring + (size_t)pos * fpx, host + (size_t)(seq - first) * fpx,
                               (size_t)cnt * fpx * sizeof(uint16_t), hipMemcpyHostToDevice, sl->s));
    if (int r = render_chunk(p, sl->s, sl->ring, sl->ws, sl->L, pos, cnt)) return r;
    sl->n_frames += (uint64_t)cnt;
    seq = stop;
    if (seq - 1 == wend)
      if (int r = emit(sl, wend + 1 - (uint64_t)T)) return r;
  }
  sl->expect = end;
  return rc;
}

}  // namespace

extern "C" {

int ssoct_slide_create(ssoct_slide** out, ssoct_plan* p, const double* lambda, double pitch, double z,
                       const double* disp_phase, const double* zernike, int hop, int slots, int x0, int y0, int q0) {
  if (!out) return fail(SSOCT_EINVAL, "slide pointer is NULL");
  *out = nullptr;
  if (int rc = check_plan(p)) return rc;
  if (p->streaming) return fail(SSOCT_EINVAL, "the plan already serves a stream");
  if (hop < 1 || hop > p->T) return fail(SSOCT_EINVAL, "hop must be in [1, T]");
  if (slots < 1 || slots > 64) return fail(SSOCT_EINVAL, "slots must be in [1, 64]");
  if (p->flags & SSOCT_WRITE_ABS) return fail(SSOCT_EUNSUPPORTED, "sliding windows need a complex64 volume");
  if (p->general || !p->gate.empty())
    return fail(SSOCT_EUNSUPPORTED, "sliding windows take the rectangular gate of a sweep linear in k");
  if (x0 < 0 || x0 >= p->N || y0 < 0 || y0 >= p->N || q0 < 0 || q0 >= p->T)
    return fail(SSOCT_EINVAL, "cut position out of range");
  SSOCT_HIP(hipSetDevice(p->device));
  const int status = update_tables(p, lambda, pitch, z, disp_phase, zernike, false);
  if (status < 0) return status;
  SSOCT_HIP(hipStreamSynchronize(p->stream));  // tables ready

  ssoct_slide* sl = new (std::nothrow) ssoct_slide();
  if (!sl) return fail(SSOCT_ENOMEM, "host allocation failed");
  sl->plan = p;
  sl->hop = hop;
  sl->nslot = slots;
  sl->x0 = x0, sl->y0 = y0, sl->q0 = q0;
  sl->out.reset(new (std::nothrow) OutSlot[slots]);
  if (!sl->out) {
    delete sl;
    return fail(SSOCT_ENOMEM, "host allocation failed");
  }
  const int T = p->T, N = p->N;
  sl->L = ws_layout(T, N, p->flags & ~SSOCT_BACKWARD, p->F);
  const size_t ncut = (size_t)N * N + 2 * (size_t)T * N;
  hipError_t e = hipStreamCreateWithFlags(&sl->s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl->cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&sl->ring, (size_t)T * N * N * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&sl->ws, sl->L.total);
  for (int k = 0; k < slots && e == hipSuccess; ++k) {
    OutSlot& o = sl->out[k];
    e = hipMalloc(&o.vol, (size_t)T * N * N * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&o.cuts, ncut * sizeof(float));
    if (e == hipSuccess) e = hipHostMalloc(&o.hcuts, ncut * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&o.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&o.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    const int rc = (e == hipErrorOutOfMemory) ? fail(SSOCT_ENOMEM, "device or pinned allocation failed")
                                              : hip_fail(e, "ssoct_slide_create");
    slide_free(sl);
    return rc;
  }
  p->streaming = true;
  *out = sl;
  return status;
}

int ssoct_slide_push(ssoct_slide* sl, const uint16_t* host_frames, int nframes, uint64_t first_seq) {
  if (!sl) return fail(SSOCT_EINVAL, "slide is NULL");
  if (!host_frames || nframes < 0) return fail(SSOCT_EINVAL, "bad frames");
  std::lock_guard<std::mutex> lock(sl->m);
  if (sl->have && first_seq < sl->expect) return fail(SSOCT_EINVAL, "frames must arrive in increasing order");
  SSOCT_HIP(hipSetDevice(sl->plan->device));
  return nframes == 0 ? SSOCT_OK : advance(sl, nframes, first_seq, host_frames);
}

int ssoct_slide_ring(ssoct_slide* sl, uint16_t** device_ring) {
  if (!sl || !device_ring) return fail(SSOCT_EINVAL, "NULL argument");
  *device_ring = sl->ring;
  return SSOCT_OK;
}

int ssoct_slide_advance(ssoct_slide* sl, int nframes, uint64_t first_seq) {
  if (!sl) return fail(SSOCT_EINVAL, "slide is NULL");
  if (nframes < 0) return fail(SSOCT_EINVAL, "bad frame count");
  std::lock_guard<std::mutex> lock(sl->m);
  if (sl->have && first_seq < sl->expect) return fail(SSOCT_EINVAL, "frames must arrive in increasing order");
  SSOCT_HIP(hipSetDevice(sl->plan->device));
  return nframes == 0 ? SSOCT_OK : advance(sl, nframes, first_seq, nullptr);
}

int ssoct_slide_pop(ssoct_slide* sl, int wait, uint64_t* window_start, int* slot, float* cut_xy, float* cut_xz,
                    float* cut_yz, double* latency_ms) {
  if (!sl) return fail(SSOCT_EINVAL, "slide is NULL");
  SSOCT_HIP(hipSetDevice(sl->plan->device));
  int k;
  {
    std::lock_guard<std::mutex> lock(sl->m);
    if (sl->inflight.empty()) return fail(SSOCT_EAGAIN, "no window in flight");
    k = sl->inflight.front();
  }
  OutSlot& o = sl->out[k];
  if (wait) {
    SSOCT_HIP(hipEventSynchronize(o.done));
  } else {
    const hipError_t q = hipEventQuery(o.done);
    if (q == hipErrorNotReady) return fail(SSOCT_EAGAIN, "window not finished");
    if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
  }
  const int T = sl->plan->T, N = sl->plan->N;
  if (cut_xy) std::memcpy(cut_xy, o.hcuts, (size_t)N * N * sizeof(float));
  if (cut_xz) std::memcpy(cut_xz, o.hcuts + (size_t)N * N, (size_t)T * N * sizeof(float));
  if (cut_yz) std::memcpy(cut_yz, o.hcuts + (size_t)N * N + (size_t)T * N, (size_t)T * N * sizeof(float));
  int64_t td = o.t_done.load();
  if (td == 0) td = slide_now_ns();
  if (latency_ms) *latency_ms = (double)(td - o.t_submit) * 1e-6;
  if (window_start) *window_start = o.start;
  if (slot) *slot = k;
  std::lock_guard<std::mutex> lock(sl->m);
  sl->inflight.pop_front();
  o.busy = false;
  sl->n_done += 1;
  return SSOCT_OK;
}

int ssoct_slide_volume(ssoct_slide* sl, int slot, const void** device_volume) {
  if (!sl || !device_volume) return fail(SSOCT_EINVAL, "NULL argument");
  if (slot < 0 || slot >= sl->nslot) return fail(SSOCT_EINVAL, "slot out of range");
  *device_volume = sl->out[slot].vol;
  return SSOCT_OK;
}

int ssoct_slide_stats(ssoct_slide* sl, uint64_t* counters) {
  if (!sl || !counters) return fail(SSOCT_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(sl->m);
  counters[0] = sl->n_done;
  counters[1] = sl->n_drop;
  counters[2] = sl->n_frames;
  counters[3] = sl->n_restart;
  counters[4] = sl->inflight.size();
  return SSOCT_OK;
}

int ssoct_slide_destroy(ssoct_slide* sl) {
  if (!sl) return SSOCT_OK;
  (void)hipSetDevice(sl->plan->device);
  slide_free(sl);
  return SSOCT_OK;
}

}  // extern "C"
