"""Thin PyTorch-facing wrapper of the C ABI: torch provides device memory and
streams; every step of the computation runs in libssoct.so."""
from __future__ import annotations

import ctypes

import torch

from . import native

PRECISIONS = {
    "fp32": native.PREC_FP32,
    "fp16": native.PREC_FP16,
    "bf16": native.PREC_BF16,
    "fp16_split": native.PREC_FP16 | native.SPLIT,
    "bf16_split": native.PREC_BF16 | native.SPLIT,
}


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _check_frames(frames: torch.Tensor, T: int, N: int):
    if frames.dtype != torch.uint16:
        raise TypeError("frames must be torch.uint16")
    if tuple(frames.shape) != (T, N, N) or not frames.is_contiguous() or not frames.is_cuda:
        raise ValueError(f"frames must be a contiguous CUDA tensor of shape {(T, N, N)}")


class Plan:
    """A libssoct plan for sweeps of T frames of N x N pixels, with its workspace."""

    def __init__(self, T: int, N: int, precision: str = "fp32", exact_chirp: bool = False,
                 eq6_phase: bool = False, write_abs: bool = False, cut_power: bool = False,
                 backward: bool = False, profile: bool = False, device=None):
        self.lib = native.load()
        self.T, self.N = int(T), int(N)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        flags = PRECISIONS[precision]
        flags |= native.CHIRP_EXACT if exact_chirp else 0
        flags |= native.EQ6_PHASE if eq6_phase else 0
        flags |= native.WRITE_ABS if write_abs else 0
        flags |= native.CUT_POWER if cut_power else 0
        flags |= native.BACKWARD if backward else 0
        flags |= native.PROFILE if profile else 0
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
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ssoct_plan_destroy(self._h)
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
        _check_frames(frames, T, N)
        if out is None:
            if self.write_abs:
                out = torch.empty((T, N, N), dtype=torch.float32, device=self.device)
            else:
                out = torch.empty((T, N, N), dtype=torch.complex64, device=self.device)
        lam_c = native.host_doubles(lam, T)
        ph_c = native.host_doubles(disp_phase, T)
        zc_c = native.host_doubles(zernike, 15)
        self._sync_stream()
        self.last_status = native.check(self.lib.ssoct_render(
            self._h, ctypes.c_void_p(_ptr(frames)), lam_c, float(pitch), float(z), ph_c, zc_c,
            ctypes.c_void_p(_ptr(self.workspace)), self.workspace.numel(), ctypes.c_void_p(_ptr(out))))
        return out

    def cuts(self, vol: torch.Tensor, x0: int, y0: int, q0: int):
        """(cut_xy [N, N], cut_xz [T, N], cut_yz [T, N]) of the envelope."""
        T, N = self.T, self.N
        if vol.dtype != torch.complex64 or tuple(vol.shape) != (T, N, N) or not vol.is_contiguous():
            raise ValueError("vol must be a contiguous complex64 tensor [T, N, N]")
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
        _check_frames(frames, T, N)
        if grad_vol.dtype != torch.complex64 or tuple(grad_vol.shape) != (T, N, N) or not grad_vol.is_contiguous():
            raise ValueError("grad_vol must be a contiguous complex64 tensor [T, N, N]")
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
        _check_frames(frames, T, N)
        out = torch.empty(2 + 15 + T, dtype=torch.float64, device=self.device)
        self._sync_stream()
        native.check(self.lib.ssoct_backward_sharpness(
            self._h, ctypes.c_void_p(_ptr(frames)), native.host_doubles(lam, T), float(pitch), float(z),
            native.host_doubles(disp_phase, T), native.host_doubles(zernike, 15),
            ctypes.c_void_p(_ptr(self.workspace)), self.workspace.numel(), ctypes.c_void_p(_ptr(out))))
        return out

    def profile_read(self):
        """Mean stage times (ms) since the last read: (tables, fresnel stage, depth transform, count)."""
        ms = (ctypes.c_float * 4)()
        native.check(self.lib.ssoct_profile_read(self._h, ms))
        return tuple(ms)
