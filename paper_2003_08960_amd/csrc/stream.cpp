// Streaming renderer of consecutive sweeps (ssoct_stream_*).
//
// The real-time system described after Eq. 7 buffers the camera stream so
// that no frame is lost and the depth transform (Eq. 7) only ever sees the
// consecutive frames of one sweep.  Here a ring of volume slots plays that role on the GPU: frames are
// copied into a slot in sweep order (sequence numbers are checked; a gap or a
// full ring discards the incomplete sweep instead of mixing sweeps), and a
// slot is rendered by HIP graphs captured at stream creation, on the slot's
// own stream, so consecutive volumes overlap on the GPU.  Host-fed frames
// start the Fresnel stage of each chunk of frames as soon as that chunk has
// landed (one small graph per chunk), and the last frame of a sweep launches
// the depth transform + cuts + copy of the cuts to pinned host memory; a
// device-filled slot replays one graph of the whole volume.
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "plan.hpp"

using namespace ssoct;

namespace {

enum SlotState { FREE = 0, FILLING = 1, ACQUIRED = 2, INFLIGHT = 3 };

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Slot {
  uint16_t* frames = nullptr;  // device [T][N][N]
  char* ws = nullptr;          // device workspace
  float2* vol = nullptr;       // device volume
  float* cuts = nullptr;       // device cuts xy | xz | yz
  float* hcuts = nullptr;      // pinned host copy of the cuts
  hipStream_t s = nullptr;
  hipGraphExec_t exec = nullptr;          // whole volume: Fresnel + depth + cuts + D2H
  std::vector<hipGraphExec_t> chunk;      // Fresnel stage of one chunk of frames
  hipGraphExec_t tail = nullptr;          // depth + cuts + D2H
  hipEvent_t landed = nullptr;  // host-fed frames have arrived
  hipEvent_t idle = nullptr;    // earlier work of the slot is over (before its frames are overwritten)
  hipEvent_t done = nullptr;    // volume finished
  int state = FREE;
  int filled = 0;
  int chunks_run = 0;
  uint64_t vseq = 0;
  int64_t t_submit = 0;
  std::atomic<int64_t> t_done{0};
};

void stamp_done(void* arg) { static_cast<Slot*>(arg)->t_done.store(now_ns()); }

}  // namespace

struct ssoct_stream {
  ssoct_plan* plan = nullptr;
  int nslot = 0;
  int x0 = 0, y0 = 0, q0 = 0;
  int F = 0;                   // frames per Fresnel chunk the graphs were captured with
  hipStream_t copy = nullptr;
  std::unique_ptr<Slot[]> slots;
  std::mutex m;
  int filling = -1;
  uint64_t expect = 0;
  bool have_expect = false;
  std::deque<int> inflight;
  uint64_t n_done = 0, n_drop_frames = 0, n_drop_sweeps = 0;
};

namespace {

void stream_free(ssoct_stream* st) {
  if (!st) return;
  if (st->slots) {
    for (int k = 0; k < st->nslot; ++k) {
      Slot& s = st->slots[k];
      if (s.s) (void)hipStreamSynchronize(s.s);
      if (s.exec) (void)hipGraphExecDestroy(s.exec);
      for (hipGraphExec_t g : s.chunk)
        if (g) (void)hipGraphExecDestroy(g);
      if (s.tail) (void)hipGraphExecDestroy(s.tail);
      if (s.landed) (void)hipEventDestroy(s.landed);
      if (s.idle) (void)hipEventDestroy(s.idle);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.s) (void)hipStreamDestroy(s.s);
      (void)hipFree(s.frames);
      (void)hipFree(s.ws);
      (void)hipFree(s.vol);
      (void)hipFree(s.cuts);
      if (s.hcuts) (void)hipHostFree(s.hcuts);
    }
  }
  if (st->copy) {
    (void)hipStreamSynchronize(st->copy);
    (void)hipStreamDestroy(st->copy);
  }
  if (st->plan) st->plan->streaming = false;
  delete st;
}

// after the slot's Fresnel work (or with it, for a whole-volume graph): the
// rest of the volume, its completion stamp and event
int finish(ssoct_stream* st, int k, hipGraphExec_t g) {
  Slot& s = st->slots[k];
  s.t_done.store(0);
  s.t_submit = now_ns();
  SSOCT_HIP(hipGraphLaunch(g, s.s));
  SSOCT_HIP(hipLaunchHostFunc(s.s, stamp_done, &s));
  SSOCT_HIP(hipEventRecord(s.done, s.s));
  s.state = INFLIGHT;
  st->inflight.push_back(k);
  return SSOCT_OK;
}

// launch the Fresnel graphs of every chunk of slot k whose frames have all been
// queued on the copy stream (the slot stream waits for those copies)
int run_landed_chunks(ssoct_stream* st, int k) {
  Slot& s = st->slots[k];
  const int T = st->plan->T, F = st->F;
  if (s.chunk.empty()) {  // whole-volume graph: wait for every frame
    if (s.filled < T) return SSOCT_OK;
    SSOCT_HIP(hipEventRecord(s.landed, st->copy));
    SSOCT_HIP(hipStreamWaitEvent(s.s, s.landed, 0));
    return SSOCT_OK;
  }
  const int ready = s.filled == T ? (int)s.chunk.size() : s.filled / F;
  if (ready <= s.chunks_run) return SSOCT_OK;
  SSOCT_HIP(hipEventRecord(s.landed, st->copy));
  SSOCT_HIP(hipStreamWaitEvent(s.s, s.landed, 0));
  for (; s.chunks_run < ready; ++s.chunks_run) SSOCT_HIP(hipGraphLaunch(s.chunk[s.chunks_run], s.s));
  return SSOCT_OK;
}

// capture what `enqueue` puts on stream s into an executable graph
template <class Fn>
int capture(hipStream_t s, hipGraphExec_t* out, Fn enqueue) {
  hipGraph_t g = nullptr;
  SSOCT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  const int rc = enqueue();
  const hipError_t ee = hipStreamEndCapture(s, &g);
  if (rc != SSOCT_OK || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != SSOCT_OK ? rc : hip_fail(ee, "hipStreamEndCapture");
  }
  const hipError_t ie = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
  return SSOCT_OK;
}

int free_slot(ssoct_stream* st) {
  for (int k = 0; k < st->nslot; ++k)
    if (st->slots[k].state == FREE) return k;
  return -1;
}

}  // namespace

extern "C" {

int ssoct_stream_create(ssoct_stream** out, ssoct_plan* p, const double* lambda, double pitch, double z,
                        const double* disp_phase, const double* zernike, int slots, int x0, int y0, int q0) {
  if (!out) return fail(SSOCT_EINVAL, "stream pointer is NULL");
  *out = nullptr;
  if (int rc = check_plan(p)) return rc;
  if (p->streaming) return fail(SSOCT_EINVAL, "the plan already serves a stream");
  if (slots < 1 || slots > 64) return fail(SSOCT_EINVAL, "slots must be in [1, 64]");
  if (p->flags & SSOCT_WRITE_ABS) return fail(SSOCT_EUNSUPPORTED, "streaming needs a complex64 volume");
  if (x0 < 0 || x0 >= p->N || y0 < 0 || y0 >= p->N || q0 < 0 || q0 >= p->T)
    return fail(SSOCT_EINVAL, "cut position out of range");
  SSOCT_HIP(hipSetDevice(p->device));
  const int status = update_tables(p, lambda, pitch, z, disp_phase, zernike, false);
  if (status < 0) return status;
  SSOCT_HIP(hipStreamSynchronize(p->stream));  // tables ready before any capture

  ssoct_stream* st = new (std::nothrow) ssoct_stream();
  if (!st) return fail(SSOCT_ENOMEM, "host allocation failed");
  st->plan = p;
  st->nslot = slots;
  st->x0 = x0, st->y0 = y0, st->q0 = q0;
  st->slots.reset(new (std::nothrow) Slot[slots]);
  if (!st->slots) {
    delete st;
    return fail(SSOCT_ENOMEM, "host allocation failed");
  }
  const int T = p->T, N = p->N;
  const WsLayout L = ws_layout(T, N, p->flags & ~SSOCT_BACKWARD, p->F);
  const size_t ncut = (size_t)N * N + 2 * (size_t)T * N;
  const int F = p->frames_run();
  // chunk-wise Fresnel graphs need the frame order; the depth-first order starts with all frames
  const int nch = p->depth_first() ? 0 : (T + F - 1) / F;
  st->F = F;
  const bool power = (p->flags & SSOCT_CUT_POWER) != 0;
  hipError_t e = hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking);
  int rc = SSOCT_OK;
  for (int k = 0; k < slots && e == hipSuccess && rc == SSOCT_OK; ++k) {
    Slot& s = st->slots[k];
    e = hipMalloc(&s.frames, (size_t)T * N * N * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc(&s.ws, L.total);
    if (e == hipSuccess) e = hipMalloc(&s.vol, (size_t)T * N * N * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&s.cuts, ncut * sizeof(float));
    if (e == hipSuccess) e = hipHostMalloc(&s.hcuts, ncut * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.landed, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.idle, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemsetAsync(s.frames, 0, (size_t)T * N * N * sizeof(uint16_t), s.s);
    if (e != hipSuccess) break;
    auto tail = [&]() -> int {
      if (int r = render_depth(p, s.s, s.ws, L, s.vol)) return r;
      float* c = s.cuts;
      SSOCT_HIP(launch_cuts(T, N, s.vol, x0, y0, q0, power ? 1 : 0, c, c + (size_t)N * N,
                            c + (size_t)N * N + (size_t)T * N, s.s));
      SSOCT_HIP(hipMemcpyAsync(s.hcuts, c, ncut * sizeof(float), hipMemcpyDeviceToHost, s.s));
      return SSOCT_OK;
    };
    rc = capture(s.s, &s.exec, [&]() -> int {
      if (int r = render_core(p, s.s, s.frames, s.ws, L, s.vol, nullptr)) return r;   // whichever order applies
      float* c = s.cuts;
      SSOCT_HIP(launch_cuts(T, N, s.vol, x0, y0, q0, power ? 1 : 0, c, c + (size_t)N * N,
                            c + (size_t)N * N + (size_t)T * N, s.s));
      SSOCT_HIP(hipMemcpyAsync(s.hcuts, c, ncut * sizeof(float), hipMemcpyDeviceToHost, s.s));
      return SSOCT_OK;
    });
    if (rc == SSOCT_OK && nch > 0) rc = capture(s.s, &s.tail, tail);
    s.chunk.assign(nch, nullptr);
    for (int c = 0; c < nch && rc == SSOCT_OK; ++c) {
      const int t0 = c * F;
      rc = capture(s.s, &s.chunk[c],
                   [&]() { return render_chunk(p, s.s, s.frames, s.ws, L, t0, T - t0 < F ? T - t0 : F); });
    }
  }
  if (e == hipSuccess && rc == SSOCT_OK) {
    for (int k = 0; k < slots && e == hipSuccess; ++k) e = hipStreamSynchronize(st->slots[k].s);
  }
  if (e != hipSuccess || rc != SSOCT_OK) {
    if (rc == SSOCT_OK)
      rc = (e == hipErrorOutOfMemory) ? fail(SSOCT_ENOMEM, "device or pinned allocation failed")
                                      : hip_fail(e, "ssoct_stream_create");
    stream_free(st);
    return rc;
  }
  p->streaming = true;
  *out = st;
  return status;
}

int ssoct_stream_push_frames(ssoct_stream* st, const uint16_t* host, int nframes, uint64_t first_seq) {
  if (!st) return fail(SSOCT_EINVAL, "stream is NULL");
  if (!host || nframes < 0) return fail(SSOCT_EINVAL, "bad frames");
  ssoct_plan* p = st->plan;
  const int T = p->T;
  const size_t fpx = (size_t)p->N * p->N;
  SSOCT_HIP(hipSetDevice(p->device));
  std::lock_guard<std::mutex> lock(st->m);
  int rc = SSOCT_OK;
  int i = 0;
  while (i < nframes) {
    const uint64_t seq = first_seq + (uint64_t)i;
    const int pos = (int)(seq % (uint64_t)T);
    if (st->filling >= 0 && (!st->have_expect || seq != st->expect)) {  // gap: discard the partial sweep
      Slot& s = st->slots[st->filling];
      st->n_drop_frames += (uint64_t)s.filled;
      st->n_drop_sweeps += 1;
      s.state = FREE;
      st->filling = -1;
      rc = SSOCT_EDROPPED;
    }
    if (st->filling < 0) {
      if (pos != 0) {  // wait for the next sweep start
        st->n_drop_frames += 1;
        rc = SSOCT_EDROPPED;
        ++i;
        continue;
      }
      const int k = free_slot(st);
      if (k < 0) {  // ring full: this sweep is lost
        st->n_drop_sweeps += 1;
        st->n_drop_frames += 1;
        rc = SSOCT_EDROPPED;
        ++i;
        continue;
      }
      Slot& s = st->slots[k];
      // the copies into this slot wait for whatever its stream still runs
      // (Fresnel chunks of a discarded sweep read the frames buffer)
      SSOCT_HIP(hipEventRecord(s.idle, s.s));
      SSOCT_HIP(hipStreamWaitEvent(st->copy, s.idle, 0));
      s.state = FILLING;
      s.filled = 0;
      s.chunks_run = 0;
      s.vseq = seq / (uint64_t)T;
      st->filling = k;
    }
    const int k = st->filling;
    Slot& s = st->slots[k];
    const int run = (nframes - i) < (T - pos) ? (nframes - i) : (T - pos);
    SSOCT_HIP(hipMemcpyAsync(s.frames + (size_t)pos * fpx, host + (size_t)i * fpx, (size_t)run * fpx * 2,
                             hipMemcpyHostToDevice, st->copy));
    s.filled += run;
    st->expect = seq + (uint64_t)run;
    st->have_expect = true;
    i += run;
    if (int r = run_landed_chunks(st, k)) return r;
    if (pos + run == T) {
      st->filling = -1;
      if (int r = finish(st, k, s.chunk.empty() ? s.exec : s.tail)) return r;
    }
  }
  return rc;
}

int ssoct_stream_acquire(ssoct_stream* st, int* slot, uint16_t** device_frames) {
  if (!st || !slot || !device_frames) return fail(SSOCT_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(st->m);
  const int k = free_slot(st);
  if (k < 0) return fail(SSOCT_EAGAIN, "no free slot");
  st->slots[k].state = ACQUIRED;
  *slot = k;
  *device_frames = st->slots[k].frames;
  return SSOCT_OK;
}

int ssoct_stream_submit(ssoct_stream* st, int slot, uint64_t volume_seq) {
  if (!st) return fail(SSOCT_EINVAL, "stream is NULL");
  SSOCT_HIP(hipSetDevice(st->plan->device));
  std::lock_guard<std::mutex> lock(st->m);
  if (slot < 0 || slot >= st->nslot || st->slots[slot].state != ACQUIRED)
    return fail(SSOCT_EINVAL, "slot was not acquired");
  st->slots[slot].vseq = volume_seq;
  return finish(st, slot, st->slots[slot].exec);
}

int ssoct_stream_pop(ssoct_stream* st, int wait, uint64_t* volume_seq, int* slot, float* cut_xy, float* cut_xz,
                     float* cut_yz, double* latency_ms) {
  if (!st) return fail(SSOCT_EINVAL, "stream is NULL");
  SSOCT_HIP(hipSetDevice(st->plan->device));
  int k;
  {
    std::lock_guard<std::mutex> lock(st->m);
    if (st->inflight.empty()) return fail(SSOCT_EAGAIN, "no volume in flight");
    k = st->inflight.front();
  }
  Slot& s = st->slots[k];
  if (wait) {
    SSOCT_HIP(hipEventSynchronize(s.done));
  } else {
    const hipError_t q = hipEventQuery(s.done);
    if (q == hipErrorNotReady) return fail(SSOCT_EAGAIN, "volume not finished");
    if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
  }
  const int T = st->plan->T, N = st->plan->N;
  if (cut_xy) std::memcpy(cut_xy, s.hcuts, (size_t)N * N * sizeof(float));
  if (cut_xz) std::memcpy(cut_xz, s.hcuts + (size_t)N * N, (size_t)T * N * sizeof(float));
  if (cut_yz) std::memcpy(cut_yz, s.hcuts + (size_t)N * N + (size_t)T * N, (size_t)T * N * sizeof(float));
  int64_t td = s.t_done.load();
  if (td == 0) td = now_ns();
  if (latency_ms) *latency_ms = (double)(td - s.t_submit) * 1e-6;
  if (volume_seq) *volume_seq = s.vseq;
  if (slot) *slot = k;
  std::lock_guard<std::mutex> lock(st->m);
  st->inflight.pop_front();
  s.state = FREE;
  st->n_done += 1;
  return SSOCT_OK;
}

int ssoct_stream_slot_volume(ssoct_stream* st, int slot, const void** device_volume) {
  if (!st || !device_volume) return fail(SSOCT_EINVAL, "NULL argument");
  if (slot < 0 || slot >= st->nslot) return fail(SSOCT_EINVAL, "slot out of range");
  *device_volume = st->slots[slot].vol;
  return SSOCT_OK;
}

int ssoct_stream_stats(ssoct_stream* st, uint64_t* counters) {
  if (!st || !counters) return fail(SSOCT_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lock(st->m);
  counters[0] = st->n_done;
  counters[1] = st->n_drop_frames;
  counters[2] = st->n_drop_sweeps;
  counters[3] = st->inflight.size();
  return SSOCT_OK;
}

int ssoct_stream_destroy(ssoct_stream* st) {
  if (!st) return SSOCT_OK;
  (void)hipSetDevice(st->plan->device);
  stream_free(st);
  return SSOCT_OK;
}

}  // extern "C"
