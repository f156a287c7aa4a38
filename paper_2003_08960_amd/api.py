"""Thin PyTorch-facing wrapper of the C ABI: torch provides device memory and
streams; every step of the computation runs in libssoct.so."""
from __future__ import annotations

import ctypes

import torch

from . import native

PRECISIONS = {
    "fp32": native.PREC_FP32,
    "fp32_fft": native.PREC_FP32 | native.DEPTH_FFT,
    "fp16": native.PREC_FP16,
    "bf16": native.PREC_BF16,
    "fp16_split": native.PREC_FP16 | native.SPLIT,
    "bf16_split": native.PREC_BF16 | native.SPLIT,
    # the depth transform factored 16 x T/16 on MFMA, per operand precision
    "fp32_4step": native.PREC_FP32 | native.DEPTH_4STEP,
    "fp16_4step": native.PREC_FP16 | native.DEPTH_4STEP,
    "bf16_4step": native.PREC_BF16 | native.DEPTH_4STEP,
    "fp16_split_4step": native.PREC_FP16 | native.SPLIT | native.DEPTH_4STEP,
    "bf16_split_4step": native.PREC_BF16 | native.SPLIT | native.DEPTH_4STEP,
}


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _check_tensor(t: torch.Tensor, name: str, dtype, shape, device):
    """Every buffer handed to the library: right dtype, shape, contiguity and device (the kernels
    index it with the plan's sizes, so anything else would be read or written out of bounds)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous tensor of shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")


def _check_frames(frames: torch.Tensor, T: int, N: int, device=None):
    if frames.dtype != torch.uint16:
        raise TypeError("frames must be torch.uint16")
    if tuple(frames.shape) != (T, N, N) or not frames.is_contiguous() or not frames.is_cuda:
        raise ValueError(f"frames must be a contiguous CUDA tensor of shape {(T, N, N)}")
    if device is not None and frames.device != device:
        raise ValueError(f"frames must be on {device}, got {frames.device}")


class Plan:
    """A libssoct plan for sweeps of T frames of N x N pixels, with its workspace."""

    def __init__(self, T: int, N: int, precision: str = "fp32", exact_chirp: bool = False,
                 eq6_phase: bool = False, write_abs: bool = False, cut_power: bool = False,
                 nonuniform_k: bool = False, angular_spectrum: bool = False,
                 backward: bool = False, profile: bool = False, device=None):
        self.lib = native.load()
        self.T, self.N = int(T), int(N)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        flags = PRECISIONS[precision]
        flags |= native.CHIRP_EXACT if exact_chirp else 0
        flags |= native.EQ6_PHASE if eq6_phase else 0
        flags |= native.WRITE_ABS if write_abs else 0
        flags |= native.NONUNIFORM_K if nonuniform_k else 0
        flags |= native.ANGULAR_SPECTRUM if angular_spectrum else 0
        flags |= native.CUT_POWER if cut_power else 0
        flags |= native.BACKWARD if backward else 0
        flags |= native.PROFILE if profile else 0
        flags |= native.PROFILE_KERNELS if profile == "kernels" else 0
        self.flags = flags
        self.precision = precision
        self.write_abs = write_abs
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            self._stream = stream.cuda_stream
            h = ctypes.c_void_p()
            native.check(self.lib.ssoct_plan_create(ctypes.byref(h), self.T, self.N, flags,
                                                    ctypes.c_void_p(self._stream)))
            self._h = h
            nbytes = self.lib.ssoct_workspace_size(self.T, self.N, flags)
            if nbytes == 0:
                raise native.SsoctError(native.EUNSUPPORTED, "unsupported size")
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    # -- stream follows torch's current stream on the plan's device
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            native.check(self.lib.ssoct_plan_set_stream(self._h, ctypes.c_void_p(s)))
            self._stream = s

    def close(self):
        """Release the plan (raises while a Stream or Slide still uses it)."""
        if getattr(self, "_h", None) is not None and self._h.value:
            native.check(self.lib.ssoct_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def render(self, frames: torch.Tensor, lam, pitch: float, z: float, disp_phase=None, zernike=None,
               out: torch.Tensor | None = None) -> torch.Tensor:
        """Complex volume V [T, N, N] (complex64), or |V| (float32) for a write_abs plan."""
        T, N = self.T, self.N
        _check_frames(frames, T, N, self.device)
        if out is None:
            if self.write_abs:
                out = torch.empty((T, N, N), dtype=torch.float32, device=self.device)
            else:
                out = torch.empty((T, N, N), dtype=torch.complex64, device=self.device)
        _check_tensor(out, "out", torch.float32 if self.write_abs else torch.complex64, (T, N, N), self.device)
        lam_c = native.host_doubles(lam, T)
        ph_c = native.host_doubles(disp_phase, T)
        zc_c = native.host_doubles(zernike, 15)
        self._sync_stream()
        self.last_status = native.check(self.lib.ssoct_plan_render(
            self._h, ctypes.c_void_p(_ptr(frames)), lam_c, float(pitch), float(z), ph_c, zc_c,
            ctypes.c_void_p(_ptr(self.workspace)), self.workspace.numel(), ctypes.c_void_p(_ptr(out))))
        return out

    def render_noalloc(self, frames: torch.Tensor, lam, pitch: float, z: float, disp_phase=None, zernike=None,
                       out: torch.Tensor | None = None) -> torch.Tensor:
        """ssoct_plan_render_noalloc: the same volume as render(), with the workspace in the library's
        static device array (no allocation inside the call; `out` must be given for a call that may
        not allocate either)."""
        T, N = self.T, self.N
        _check_frames(frames, T, N, self.device)
        if out is None:
            out = torch.empty((T, N, N), dtype=torch.float32 if self.write_abs else torch.complex64,
                              device=self.device)
        _check_tensor(out, "out", torch.float32 if self.write_abs else torch.complex64, (T, N, N), self.device)
        self._sync_stream()
        self.last_status = native.check(self.lib.ssoct_plan_render_noalloc(
            self._h, ctypes.c_void_p(_ptr(frames)), native.host_doubles(lam, T), float(pitch), float(z),
            native.host_doubles(disp_phase, T), native.host_doubles(zernike, 15), ctypes.c_void_p(_ptr(out))))
        return out

    def cuts(self, vol: torch.Tensor, x0: int, y0: int, q0: int):
        """(cut_xy [N, N], cut_xz [T, N], cut_yz [T, N]) of the envelope."""
        T, N = self.T, self.N
        _check_tensor(vol, "vol", torch.complex64, (T, N, N), self.device)
        xy = torch.empty((N, N), dtype=torch.float32, device=self.device)
        xz = torch.empty((T, N), dtype=torch.float32, device=self.device)
        yz = torch.empty((T, N), dtype=torch.float32, device=self.device)
        self._sync_stream()
        native.check(self.lib.ssoct_cuts(self._h, ctypes.c_void_p(_ptr(vol)), int(x0), int(y0), int(q0),
                                         ctypes.c_void_p(_ptr(xy)), ctypes.c_void_p(_ptr(xz)),
                                         ctypes.c_void_p(_ptr(yz))))
        return xy, xz, yz

    def backward(self, frames, lam, pitch, z, grad_vol: torch.Tensor, disp_phase=None, zernike=None):
        """(dL/dz, dL/dc[15], dL/dphi[T]) as a float64 device tensor of 2 + 15 + T entries."""
        T, N = self.T, self.N
        _check_frames(frames, T, N, self.device)
        _check_tensor(grad_vol, "grad_vol", torch.complex64, (T, N, N), self.device)
        out = torch.empty(2 + 15 + T, dtype=torch.float64, device=self.device)
        self._sync_stream()
        native.check(self.lib.ssoct_backward(
            self._h, ctypes.c_void_p(_ptr(frames)), native.host_doubles(lam, T), float(pitch), float(z),
            native.host_doubles(disp_phase, T), native.host_doubles(zernike, 15), ctypes.c_void_p(_ptr(grad_vol)),
            ctypes.c_void_p(_ptr(self.workspace)), self.workspace.numel(), ctypes.c_void_p(_ptr(out))))
        return out

    def backward_sharpness(self, frames, lam, pitch, z, disp_phase=None, zernike=None):
        """[L, dL/dz, dL/dc (15), dL/dphi (T)] for L = sum |V|^4, float64 device tensor."""
        T, N = self.T, self.N
        _check_frames(frames, T, N, self.device)
        out = torch.empty(2 + 15 + T, dtype=torch.float64, device=self.device)
        self._sync_stream()
        native.check(self.lib.ssoct_backward_sharpness(
            self._h, ctypes.c_void_p(_ptr(frames)), native.host_doubles(lam, T), float(pitch), float(z),
            native.host_doubles(disp_phase, T), native.host_doubles(zernike, 15),
            ctypes.c_void_p(_ptr(self.workspace)), self.workspace.numel(), ctypes.c_void_p(_ptr(out))))
        return out

    def set_gate(self, gate=None):
        """Apodising gate g_t (T real weights) applied before the depth transform; None: rectangular."""
        native.check(self.lib.ssoct_plan_set_gate(self._h, native.host_doubles(gate, self.T)))

    def profile_read(self):
        """Mean times (ms) per render since the last read: (tables, Fresnel stage, depth transform,
        renders averaged, all row-pass launches, all column-pass launches)."""
        ms = (ctypes.c_float * 6)()
        native.check(self.lib.ssoct_profile_read(self._h, ms))
        return tuple(ms)

    # -- launch shapes ---------------------------------------------------------------------------
    def get_tuning(self):
        """[frames per chunk, column workgroups, depth workgroups, evaluation order, rows per row group
        (depth-first order), column tile width, depth pixels per workgroup (FFT and factored forms),
        dense K chunk, column radix order] (include/ssoct.h)."""
        t = (ctypes.c_int * native.TUNING_LEN)()
        native.check(self.lib.ssoct_plan_get_tuning(self._h, t))
        return [int(x) for x in t]

    def set_tuning(self, tuning):
        """Set launch shapes; a shorter list keeps the plan's current values of the entries it omits."""
        vals = [int(x) for x in tuning]
        if not 1 <= len(vals) <= native.TUNING_LEN:
            raise ValueError(f"tuning has 1 to {native.TUNING_LEN} entries")
        vals += self.get_tuning()[len(vals):]
        t = (ctypes.c_int * native.TUNING_LEN)(*vals)
        native.check(self.lib.ssoct_plan_set_tuning(self._h, t))

    def tuning_key(self, disp_phase=None, zernike=None) -> str:
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        flags = self.flags & ~(native.PROFILE | native.PROFILE_KERNELS)
        return (f"{arch}|T{self.T}|N{self.N}|flags{flags}|disp{int(disp_phase is not None)}"
                f"|zern{int(zernike is not None)}")

    def tune(self, frames, lam, pitch, z, disp_phase=None, zernike=None, cache_path: str | None = None,
             out: torch.Tensor | None = None):
        """Pick launch shapes by timing candidates (ssoct_plan_tune, which also keeps its choice in a
        process-wide cache); with `cache_path`, reuse or store the choice in a JSON file keyed by GPU
        architecture, T, N, plan flags and whether dispersion and aberration are given.  `out` is an
        optional volume buffer to render into while timing."""
        key = self.tuning_key(disp_phase, zernike)
        if cache_path:
            cached = _load_cache(cache_path).get(key)
            if cached is not None:
                self.set_tuning(cached)
                return list(cached)
        _check_frames(frames, self.T, self.N, self.device)
        out = self.render(frames, lam, pitch, z, disp_phase, zernike, out=out)
        t = (ctypes.c_int * native.TUNING_LEN)()
        self._sync_stream()
        native.check(self.lib.ssoct_plan_tune(
            self._h, ctypes.c_void_p(_ptr(frames)), native.host_doubles(lam, self.T), float(pitch), float(z),
            native.host_doubles(disp_phase, self.T), native.host_doubles(zernike, 15),
            ctypes.c_void_p(_ptr(self.workspace)), self.workspace.numel(), ctypes.c_void_p(_ptr(out)), t))
        choice = [int(x) for x in t]
        if cache_path:
            data = _load_cache(cache_path)
            data[key] = choice
            _store_cache(cache_path, data)
        return choice


def render(frames: torch.Tensor, lam, pitch: float, z: float, out: torch.Tensor | None = None) -> torch.Tensor:
    """ssoct_render: the complex volume [T, N, N] (complex64) of one sweep of uint16 frames [T, N, N]
    on their device, with the library's cached FP32 default plan, on torch's current stream."""
    lib = native.load()
    if frames.dtype != torch.uint16 or frames.dim() != 3 or frames.shape[1] != frames.shape[2] \
            or not frames.is_contiguous() or not frames.is_cuda:
        raise ValueError("frames must be a contiguous CUDA uint16 tensor [T, N, N]")
    T, N = int(frames.shape[0]), int(frames.shape[1])
    if out is None:
        out = torch.empty((T, N, N), dtype=torch.complex64, device=frames.device)
    _check_tensor(out, "out", torch.complex64, (T, N, N), frames.device)
    with torch.cuda.device(frames.device):
        stream = torch.cuda.current_stream(frames.device).cuda_stream
        native.check(lib.ssoct_render(ctypes.c_void_p(_ptr(frames)), T, N, native.host_doubles(lam, T), float(pitch),
                                      float(z), ctypes.c_void_p(_ptr(out)), ctypes.c_void_p(stream)))
    return out


def render_release():
    """ssoct_render_release: free the plans and workspaces cached by render()."""
    native.check(native.load().ssoct_render_release())


def tune_cache_clear():
    """ssoct_tune_cache_clear: forget the launch shapes ssoct_plan_tune chose in this process."""
    native.check(native.load().ssoct_tune_cache_clear())


def _load_cache(path):
    import json
    import os
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def _store_cache(path, data):
    import json
    import os
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class _DeviceArray:
    """__cuda_array_interface__ view of library-owned device memory (no copy)."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 3, "strides": None}


class Stream:
    """ssoct_stream: continuous rendering of consecutive sweeps with a ring of volume slots."""

    def __init__(self, plan: Plan, lam, pitch, z, disp_phase=None, zernike=None, slots: int = 3,
                 x0: int | None = None, y0: int | None = None, q0: int | None = None):
        self.plan, self.lib = plan, plan.lib
        self.T, self.N = plan.T, plan.N
        self.x0 = self.N // 2 if x0 is None else int(x0)
        self.y0 = self.N // 2 if y0 is None else int(y0)
        self.q0 = self.T // 4 if q0 is None else int(q0)
        h = ctypes.c_void_p()
        with torch.cuda.device(plan.device):
            native.check(self.lib.ssoct_stream_create(
                ctypes.byref(h), plan._h, native.host_doubles(lam, self.T), float(pitch), float(z),
                native.host_doubles(disp_phase, self.T), native.host_doubles(zernike, 15), int(slots),
                self.x0, self.y0, self.q0))
        self._h = h
        self._keep = []   # host buffers pushed and not yet popped

    def push_frames(self, host_frames, first_seq: int) -> int:
        """Push frames [n, N, N] uint16 (numpy array or CPU tensor; pinned memory is copied
        asynchronously).  Returns OK or EDROPPED."""
        arr = host_frames
        if isinstance(arr, torch.Tensor):
            if arr.is_cuda or arr.dtype != torch.uint16 or not arr.is_contiguous():
                raise ValueError("host_frames must be a contiguous CPU uint16 tensor")
            ptr, n = arr.data_ptr(), arr.shape[0]
        else:
            import numpy as np
            if arr.dtype != np.uint16 or not arr.flags["C_CONTIGUOUS"]:
                raise ValueError("host_frames must be a C-contiguous uint16 array")
            ptr, n = arr.ctypes.data, arr.shape[0]
        if tuple(arr.shape[1:]) != (self.N, self.N):
            raise ValueError("frame shape mismatch")
        self._keep.append(((int(first_seq) + n - 1) // self.T, arr))   # alive until its sweep is popped
        rc = self.lib.ssoct_stream_push_frames(self._h, ctypes.c_void_p(ptr), int(n), ctypes.c_uint64(first_seq))
        if rc == native.EDROPPED:
            return rc
        return native.check(rc)

    def acquire(self):
        """(slot, device frame buffer as a torch uint16 tensor [T, N, N]) or None if no slot is free."""
        slot = ctypes.c_int()
        ptr = ctypes.c_void_p()
        rc = self.lib.ssoct_stream_acquire(self._h, ctypes.byref(slot), ctypes.byref(ptr))
        if rc == native.EAGAIN:
            return None
        native.check(rc)
        view = torch.as_tensor(_DeviceArray(ptr.value, (self.T, self.N, self.N), "<u2"), device=self.plan.device)
        return slot.value, view

    def submit(self, slot: int, volume_seq: int):
        native.check(self.lib.ssoct_stream_submit(self._h, int(slot), ctypes.c_uint64(volume_seq)))

    def pop(self, wait: bool = True, cuts: bool = True):
        """Oldest finished volume as a dict (seq, slot, latency_ms, cut_xy, cut_xz, cut_yz), or None."""
        import numpy as np
        seq = ctypes.c_uint64()
        slot = ctypes.c_int()
        lat = ctypes.c_double()
        xy = np.empty((self.N, self.N), np.float32) if cuts else None
        xz = np.empty((self.T, self.N), np.float32) if cuts else None
        yz = np.empty((self.T, self.N), np.float32) if cuts else None
        ptr = (lambda a: ctypes.c_void_p(a.ctypes.data) if a is not None else None)
        rc = self.lib.ssoct_stream_pop(self._h, 1 if wait else 0, ctypes.byref(seq), ctypes.byref(slot), ptr(xy),
                                       ptr(xz), ptr(yz), ctypes.byref(lat))
        if rc == native.EAGAIN:
            return None
        native.check(rc)
        self._keep = [(v, a) for v, a in self._keep if v > int(seq.value)]
        return {"seq": int(seq.value), "slot": int(slot.value), "latency_ms": float(lat.value),
                "cut_xy": xy, "cut_xz": xz, "cut_yz": yz}

    def slot_volume(self, slot: int) -> torch.Tensor:
        """Device complex volume of a slot (a view, valid until the slot is reused: a read of the view on
        torch's stream must have completed, e.g. torch.cuda.synchronize(), before the slot is acquired,
        pushed into or submitted again)."""
        ptr = ctypes.c_void_p()
        native.check(self.lib.ssoct_stream_slot_volume(self._h, int(slot), ctypes.byref(ptr)))
        raw = torch.as_tensor(_DeviceArray(ptr.value, (self.T, self.N, self.N, 2), "<f4"), device=self.plan.device)
        return torch.view_as_complex(raw)

    def stats(self):
        c = (ctypes.c_uint64 * 4)()
        native.check(self.lib.ssoct_stream_stats(self._h, c))
        return {"done": int(c[0]), "dropped_frames": int(c[1]), "dropped_sweeps": int(c[2]), "in_flight": int(c[3])}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ssoct_stream_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Slide:
    """ssoct_slide: sliding-window depth transform (gate of T frames advanced by `hop`) over a frame stream."""

    def __init__(self, plan: Plan, lam, pitch, z, disp_phase=None, zernike=None, hop: int = 13, slots: int = 2,
                 x0: int | None = None, y0: int | None = None, q0: int | None = None):
        self.plan, self.lib = plan, plan.lib
        self.T, self.N = plan.T, plan.N
        self.x0 = self.N // 2 if x0 is None else int(x0)
        self.y0 = self.N // 2 if y0 is None else int(y0)
        self.q0 = self.T // 4 if q0 is None else int(q0)
        h = ctypes.c_void_p()
        with torch.cuda.device(plan.device):
            native.check(self.lib.ssoct_slide_create(
                ctypes.byref(h), plan._h, native.host_doubles(lam, self.T), float(pitch), float(z),
                native.host_doubles(disp_phase, self.T), native.host_doubles(zernike, 15), int(hop), int(slots),
                self.x0, self.y0, self.q0))
        self._h = h
        self._keep = []   # (last frame, host buffer) until a finished window ends at or after that frame

    def push(self, host_frames, first_seq: int) -> int:
        """Frames [n, N, N] uint16 (numpy array or CPU tensor). Returns OK, or EDROPPED after a sequence gap."""
        arr = host_frames
        if isinstance(arr, torch.Tensor):
            if arr.is_cuda or arr.dtype != torch.uint16 or not arr.is_contiguous():
                raise ValueError("host_frames must be a contiguous CPU uint16 tensor")
            ptr, n = arr.data_ptr(), arr.shape[0]
        else:
            import numpy as np
            if arr.dtype != np.uint16 or not arr.flags["C_CONTIGUOUS"]:
                raise ValueError("host_frames must be a C-contiguous uint16 array")
            ptr, n = arr.ctypes.data, arr.shape[0]
        if tuple(arr.shape[1:]) != (self.N, self.N):
            raise ValueError("frame shape mismatch")
        self._keep.append((int(first_seq) + n - 1, arr))
        rc = self.lib.ssoct_slide_push(self._h, ctypes.c_void_p(ptr), int(n), ctypes.c_uint64(first_seq))
        return rc if rc == native.EDROPPED else native.check(rc)

    def ring(self) -> torch.Tensor:
        """The device frame ring [T, N, N] uint16 (frame seq in slot seq % T)."""
        ptr = ctypes.c_void_p()
        native.check(self.lib.ssoct_slide_ring(self._h, ctypes.byref(ptr)))
        return torch.as_tensor(_DeviceArray(ptr.value, (self.T, self.N, self.N), "<u2"), device=self.plan.device)

    def advance(self, n: int, first_seq: int) -> int:
        """Frames first_seq .. first_seq + n - 1 are in the ring: transform them (and emit windows)."""
        rc = self.lib.ssoct_slide_advance(self._h, int(n), ctypes.c_uint64(first_seq))
        return rc if rc == native.EDROPPED else native.check(rc)

    def pop(self, wait: bool = True, cuts: bool = True):
        """Oldest finished window as a dict (start, slot, latency_ms, cut_xy, cut_xz, cut_yz), or None."""
        import numpy as np
        start = ctypes.c_uint64()
        slot = ctypes.c_int()
        lat = ctypes.c_double()
        xy = np.empty((self.N, self.N), np.float32) if cuts else None
        xz = np.empty((self.T, self.N), np.float32) if cuts else None
        yz = np.empty((self.T, self.N), np.float32) if cuts else None
        ptr = (lambda a: ctypes.c_void_p(a.ctypes.data) if a is not None else None)
        rc = self.lib.ssoct_slide_pop(self._h, 1 if wait else 0, ctypes.byref(start), ctypes.byref(slot), ptr(xy),
                                      ptr(xz), ptr(yz), ctypes.byref(lat))
        if rc == native.EAGAIN:
            return None
        native.check(rc)
        last = int(start.value) + self.T - 1
        self._keep = [(v, a) for v, a in self._keep if v > last]
        return {"start": int(start.value), "slot": int(slot.value), "latency_ms": float(lat.value),
                "cut_xy": xy, "cut_xz": xz, "cut_yz": yz}

    def volume(self, slot: int) -> torch.Tensor:
        """Device complex volume of an output slot (a view, valid until the slot is reused: the next
        push or advance may start a window in it on the library's stream, so a read of the view, e.g. a
        clone on torch's stream, must have completed, e.g. torch.cuda.synchronize(), before that call)."""
        ptr = ctypes.c_void_p()
        native.check(self.lib.ssoct_slide_volume(self._h, int(slot), ctypes.byref(ptr)))
        raw = torch.as_tensor(_DeviceArray(ptr.value, (self.T, self.N, self.N, 2), "<f4"), device=self.plan.device)
        return torch.view_as_complex(raw)

    def stats(self):
        c = (ctypes.c_uint64 * 5)()
        native.check(self.lib.ssoct_slide_stats(self._h, c))
        return {"done": int(c[0]), "dropped_windows": int(c[1]), "frames": int(c[2]), "restarts": int(c[3]),
                "in_flight": int(c[4])}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ssoct_slide_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
