"""ctypes binding of libssoct.so (argument marshalling only).

The names and argument order follow include/ssoct.h.  Every compute step
runs in the HIP library; if the library is missing this module raises: there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

# SSOCT_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("SSOCT_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libssoct.so")

# status codes and flags (include/ssoct.h)
OK = 0
WARN_UNDERSAMPLED = 1
EINVAL = -1
EUNSUPPORTED = -2
EHIP = -3
ENOMEM = -4
EALIAS = -5
EDROPPED = -6
EAGAIN = -7

PREC_FP32 = 0
PREC_FP16 = 1
PREC_BF16 = 2
SPLIT = 4
CHIRP_EXACT = 8
EQ6_PHASE = 16
WRITE_ABS = 32
CUT_POWER = 64
BACKWARD = 128
PROFILE = 256
PROFILE_KERNELS = 512
DEPTH_FFT = 1024
NONUNIFORM_K = 2048
ANGULAR_SPECTRUM = 4096
DEPTH_4STEP = 8192
TUNING_LEN = 9          # entries of a plan's launch-shape tuning array (SSOCT_TUNING_LEN)

EXPORTS = (
    "ssoct_version", "ssoct_last_error", "ssoct_workspace_size", "ssoct_plan_create",
    "ssoct_plan_set_stream", "ssoct_plan_destroy", "ssoct_render", "ssoct_render_release", "ssoct_plan_render",
    "ssoct_plan_render_noalloc", "ssoct_cuts", "ssoct_backward",
    "ssoct_backward_sharpness", "ssoct_plan_set_gate", "ssoct_profile_read", "ssoct_plan_tune", "ssoct_plan_get_tuning",
    "ssoct_plan_set_tuning", "ssoct_tune_cache_clear", "ssoct_stream_create", "ssoct_stream_push_frames", "ssoct_stream_acquire",
    "ssoct_stream_submit", "ssoct_stream_pop", "ssoct_stream_slot_volume", "ssoct_stream_stats",
    "ssoct_stream_destroy", "ssoct_slide_create", "ssoct_slide_push", "ssoct_slide_ring", "ssoct_slide_advance",
    "ssoct_slide_pop", "ssoct_slide_volume", "ssoct_slide_stats", "ssoct_slide_destroy",
)

_NAMES = {EINVAL: "EINVAL", EUNSUPPORTED: "EUNSUPPORTED", EHIP: "EHIP", ENOMEM: "ENOMEM", EALIAS: "EALIAS",
          EDROPPED: "EDROPPED", EAGAIN: "EAGAIN"}


class SsoctError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ssoct error {_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

c_void_p, c_int, c_double, c_size_t, c_uint32 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                                 ctypes.c_size_t, ctypes.c_uint32)
_dptr = ctypes.POINTER(ctypes.c_double)
_fptr = ctypes.POINTER(ctypes.c_float)


def _declare(lib):
    lib.ssoct_version.restype = c_int
    lib.ssoct_version.argtypes = []
    lib.ssoct_last_error.restype = ctypes.c_char_p
    lib.ssoct_last_error.argtypes = []
    lib.ssoct_workspace_size.restype = c_size_t
    lib.ssoct_workspace_size.argtypes = [c_int, c_int, c_uint32]
    lib.ssoct_plan_create.restype = c_int
    lib.ssoct_plan_create.argtypes = [ctypes.POINTER(c_void_p), c_int, c_int, c_uint32, c_void_p]
    lib.ssoct_plan_set_stream.restype = c_int
    lib.ssoct_plan_set_stream.argtypes = [c_void_p, c_void_p]
    lib.ssoct_plan_destroy.restype = c_int
    lib.ssoct_plan_destroy.argtypes = [c_void_p]
    lib.ssoct_render.restype = c_int
    lib.ssoct_render.argtypes = [c_void_p, c_int, c_int, _dptr, c_double, c_double, c_void_p, c_void_p]
    lib.ssoct_render_release.restype = c_int
    lib.ssoct_render_release.argtypes = []
    lib.ssoct_plan_render.restype = c_int
    lib.ssoct_plan_render.argtypes = [c_void_p, c_void_p, _dptr, c_double, c_double, _dptr, _dptr, c_void_p,
                                      c_size_t, c_void_p]
    lib.ssoct_plan_render_noalloc.restype = c_int
    lib.ssoct_plan_render_noalloc.argtypes = [c_void_p, c_void_p, _dptr, c_double, c_double, _dptr, _dptr, c_void_p]
    lib.ssoct_cuts.restype = c_int
    lib.ssoct_cuts.argtypes = [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p]
    lib.ssoct_backward.restype = c_int
    lib.ssoct_backward.argtypes = [c_void_p, c_void_p, _dptr, c_double, c_double, _dptr, _dptr, c_void_p, c_void_p,
                                   c_size_t, c_void_p]
    lib.ssoct_backward_sharpness.restype = c_int
    lib.ssoct_backward_sharpness.argtypes = [c_void_p, c_void_p, _dptr, c_double, c_double, _dptr, _dptr, c_void_p,
                                             c_size_t, c_void_p]
    lib.ssoct_plan_set_gate.restype = c_int
    lib.ssoct_plan_set_gate.argtypes = [c_void_p, _dptr]
    lib.ssoct_profile_read.restype = c_int
    lib.ssoct_profile_read.argtypes = [c_void_p, _fptr]
    _iptr = ctypes.POINTER(c_int)
    lib.ssoct_plan_tune.restype = c_int
    lib.ssoct_plan_tune.argtypes = [c_void_p, c_void_p, _dptr, c_double, c_double, _dptr, _dptr, c_void_p, c_size_t,
                                    c_void_p, _iptr]
    lib.ssoct_plan_get_tuning.restype = c_int
    lib.ssoct_plan_get_tuning.argtypes = [c_void_p, _iptr]
    lib.ssoct_plan_set_tuning.restype = c_int
    lib.ssoct_plan_set_tuning.argtypes = [c_void_p, _iptr]
    lib.ssoct_tune_cache_clear.restype = c_int
    lib.ssoct_tune_cache_clear.argtypes = []
    lib.ssoct_stream_create.restype = c_int
    lib.ssoct_stream_create.argtypes = [ctypes.POINTER(c_void_p), c_void_p, _dptr, c_double, c_double, _dptr, _dptr,
                                        c_int, c_int, c_int, c_int]
    lib.ssoct_stream_push_frames.restype = c_int
    lib.ssoct_stream_push_frames.argtypes = [c_void_p, c_void_p, c_int, ctypes.c_uint64]
    lib.ssoct_stream_acquire.restype = c_int
    lib.ssoct_stream_acquire.argtypes = [c_void_p, _iptr, ctypes.POINTER(c_void_p)]
    lib.ssoct_stream_submit.restype = c_int
    lib.ssoct_stream_submit.argtypes = [c_void_p, c_int, ctypes.c_uint64]
    lib.ssoct_stream_pop.restype = c_int
    lib.ssoct_stream_pop.argtypes = [c_void_p, c_int, ctypes.POINTER(ctypes.c_uint64), _iptr, c_void_p, c_void_p,
                                     c_void_p, _dptr]
    lib.ssoct_stream_slot_volume.restype = c_int
    lib.ssoct_stream_slot_volume.argtypes = [c_void_p, c_int, ctypes.POINTER(c_void_p)]
    lib.ssoct_stream_stats.restype = c_int
    lib.ssoct_stream_stats.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    lib.ssoct_stream_destroy.restype = c_int
    lib.ssoct_stream_destroy.argtypes = [c_void_p]
    lib.ssoct_slide_create.restype = c_int
    lib.ssoct_slide_create.argtypes = [ctypes.POINTER(c_void_p), c_void_p, _dptr, c_double, c_double, _dptr, _dptr,
                                       c_int, c_int, c_int, c_int, c_int]
    lib.ssoct_slide_push.restype = c_int
    lib.ssoct_slide_push.argtypes = [c_void_p, c_void_p, c_int, ctypes.c_uint64]
    lib.ssoct_slide_ring.restype = c_int
    lib.ssoct_slide_ring.argtypes = [c_void_p, ctypes.POINTER(c_void_p)]
    lib.ssoct_slide_advance.restype = c_int
    lib.ssoct_slide_advance.argtypes = [c_void_p, c_int, ctypes.c_uint64]
    lib.ssoct_slide_pop.restype = c_int
    lib.ssoct_slide_pop.argtypes = [c_void_p, c_int, ctypes.POINTER(ctypes.c_uint64), _iptr, c_void_p, c_void_p,
                                    c_void_p, _dptr]
    lib.ssoct_slide_volume.restype = c_int
    lib.ssoct_slide_volume.argtypes = [c_void_p, c_int, ctypes.POINTER(c_void_p)]
    lib.ssoct_slide_stats.restype = c_int
    lib.ssoct_slide_stats.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    lib.ssoct_slide_destroy.restype = c_int
    lib.ssoct_slide_destroy.argtypes = [c_void_p]
    return lib


def load():
    """Load libssoct.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (binds libamdhip64 first)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2003_08960_amd.build`")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def check(rc: int) -> int:
    """Raise SsoctError for a negative status, return warnings (> 0) unchanged."""
    if rc < 0:
        raise SsoctError(rc, load().ssoct_last_error().decode(errors="replace"))
    return rc


def host_doubles(values, n: int | None = None):
    """A ctypes double array (kept alive by the caller) or None."""
    if values is None:
        return None
    vals = [float(v) for v in values]
    if n is not None and len(vals) != n:
        raise ValueError(f"expected {n} values, got {len(vals)}")
    return (ctypes.c_double * len(vals))(*vals)
