"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/ssoct.h declares, and rejects bad arguments before any
HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssoct.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2003_08960_amd import native
    if not os.path.exists(native.LIB_PATH):
        from paper_2003_08960_amd import build
        build.build()
    return native.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssoct_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ssoct_plan_create", "ssoct_render", "ssoct_plan_render", "ssoct_cuts", "ssoct_backward",
                     "ssoct_backward_sharpness", "ssoct_workspace_size"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2003_08960_amd import native
    names = declared_functions()
    assert sorted(native.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n), n


def test_version(lib):
    assert lib.ssoct_version() == 1


def test_workspace_size(lib):
    from paper_2003_08960_amd import native
    T, N = 256, 1024
    stack = T * N * N * 8
    ws = lib.ssoct_workspace_size(T, N, 0)
    assert stack < ws <= stack + (256 << 20)     # H stack + row-transformed chunk buffers
    # FFT-form plans hold a 256 MiB chunk buffer (the depth-first order's chunk), others 128 MiB
    assert lib.ssoct_workspace_size(T, N, 0) == stack + (128 << 20)
    assert lib.ssoct_workspace_size(T, N, native.DEPTH_FFT) == stack + (256 << 20)
    wsb = lib.ssoct_workspace_size(T, N, native.BACKWARD)
    assert wsb >= 2 * stack
    for bad in ((0, 128), (1025, 128), (8, 100), (8, 8), (8, 4096)):
        assert lib.ssoct_workspace_size(bad[0], bad[1], 0) == 0


def test_plan_create_rejects_bad_sizes(lib):
    from paper_2003_08960_amd import native
    for T, N in ((0, 128), (1025, 128), (4, 100), (4, 8), (4, 4096)):
        h = ctypes.c_void_p(1234)
        rc = lib.ssoct_plan_create(ctypes.byref(h), T, N, 0, None)
        assert rc == native.EUNSUPPORTED
        assert not h.value
        assert lib.ssoct_last_error()
    h = ctypes.c_void_p()
    assert lib.ssoct_plan_create(ctypes.byref(h), 8, 64, native.PREC_FP32 | native.SPLIT, None) == native.EINVAL
    assert lib.ssoct_plan_create(ctypes.byref(h), 8, 64, 3, None) == native.EINVAL
    assert lib.ssoct_plan_create(None, 8, 64, 0, None) == native.EINVAL
    fft = native.DEPTH_FFT
    assert lib.ssoct_plan_create(ctypes.byref(h), 16, 64, fft | native.PREC_BF16 | native.SPLIT, None) == native.EINVAL
    assert lib.ssoct_plan_create(ctypes.byref(h), 16, 64, fft | native.PREC_FP16, None) == native.EINVAL
    for T in (8, 100, 512):
        assert lib.ssoct_plan_create(ctypes.byref(h), T, 64, fft, None) == native.EUNSUPPORTED
    assert lib.ssoct_plan_create(ctypes.byref(h), 16, 64, fft | native.NONUNIFORM_K, None) == native.EINVAL
    for f in (native.EQ6_PHASE, native.CHIRP_EXACT):
        assert lib.ssoct_plan_create(ctypes.byref(h), 16, 64, native.ANGULAR_SPECTRUM | f, None) == native.EINVAL
    f4 = native.DEPTH_4STEP
    for T in (16, 48, 512):
        assert lib.ssoct_plan_create(ctypes.byref(h), T, 64, f4, None) == native.EUNSUPPORTED
    assert lib.ssoct_plan_create(ctypes.byref(h), 64, 64, f4 | fft, None) == native.EINVAL
    assert lib.ssoct_plan_create(ctypes.byref(h), 64, 64, f4 | native.NONUNIFORM_K, None) == native.EINVAL
    assert not h.value
    g = (ctypes.c_double * 4)(1, 1, 1, 1)
    assert lib.ssoct_plan_set_gate(None, g) == native.EINVAL


def test_null_plan_is_rejected(lib):
    from paper_2003_08960_amd import native
    lam = (ctypes.c_double * 4)(1e-6, 1e-6, 1e-6, 1e-6)
    assert lib.ssoct_plan_render(None, None, lam, 1e-5, 0.1, None, None, None, 0, None) == native.EINVAL
    # the five-argument form checks its pointers and sizes before any HIP call
    assert lib.ssoct_render(None, 8, 64, lam, 1e-5, 0.1, None, None) == native.EINVAL
    assert lib.ssoct_render(ctypes.c_void_p(64), 8, 100, lam, 1e-5, 0.1, ctypes.c_void_p(64), None) == \
        native.EUNSUPPORTED
    assert lib.ssoct_render(ctypes.c_void_p(64), 0, 64, lam, 1e-5, 0.1, ctypes.c_void_p(64), None) == \
        native.EUNSUPPORTED
    assert lib.ssoct_render_release() == native.OK     # nothing cached: nothing to release
    assert lib.ssoct_cuts(None, None, 0, 0, 0, None, None, None) == native.EINVAL
    assert lib.ssoct_backward(None, None, lam, 1e-5, 0.1, None, None, None, None, 0, None) == native.EINVAL
    assert lib.ssoct_backward_sharpness(None, None, lam, 1e-5, 0.1, None, None, None, 0, None) == native.EINVAL
    ms = (ctypes.c_float * 6)()
    assert lib.ssoct_profile_read(None, ms) == native.EINVAL
    assert lib.ssoct_plan_destroy(None) == native.OK
    assert b"NULL" in lib.ssoct_last_error() or b"null" in lib.ssoct_last_error()


def test_binding_raises_with_message(lib):
    from paper_2003_08960_amd import native
    with pytest.raises(native.SsoctError) as e:
        native.check(native.EINVAL)
    assert "EINVAL" in str(e.value)
    assert native.check(native.WARN_UNDERSAMPLED) == native.WARN_UNDERSAMPLED


def test_stream_and_tuning_entry_points_reject_null(lib):
    from paper_2003_08960_amd import native
    lam = (ctypes.c_double * 4)(1e-6, 1e-6, 1e-6, 1e-6)
    h = ctypes.c_void_p(99)
    assert lib.ssoct_stream_create(ctypes.byref(h), None, lam, 1e-5, 0.1, None, None, 2, 0, 0, 0) == native.EINVAL
    assert not h.value
    assert lib.ssoct_stream_create(None, None, lam, 1e-5, 0.1, None, None, 2, 0, 0, 0) == native.EINVAL
    assert lib.ssoct_stream_push_frames(None, None, 1, 0) == native.EINVAL
    slot = ctypes.c_int()
    ptr = ctypes.c_void_p()
    assert lib.ssoct_stream_acquire(None, ctypes.byref(slot), ctypes.byref(ptr)) == native.EINVAL
    assert lib.ssoct_stream_submit(None, 0, 0) == native.EINVAL
    assert lib.ssoct_stream_pop(None, 1, None, None, None, None, None, None) == native.EINVAL
    c = (ctypes.c_uint64 * 4)()
    assert lib.ssoct_stream_stats(None, c) == native.EINVAL
    assert lib.ssoct_stream_destroy(None) == native.OK
    t = (ctypes.c_int * native.TUNING_LEN)()
    assert lib.ssoct_plan_get_tuning(None, t) == native.EINVAL
    assert lib.ssoct_plan_set_tuning(None, t) == native.EINVAL
    assert lib.ssoct_plan_tune(None, None, lam, 1e-5, 0.1, None, None, None, 0, None, t) == native.EINVAL


def test_slide_entry_points_reject_null(lib):
    from paper_2003_08960_amd import native
    lam = (ctypes.c_double * 4)(1e-6, 1e-6, 1e-6, 1e-6)
    h = ctypes.c_void_p(7)
    assert lib.ssoct_slide_create(ctypes.byref(h), None, lam, 1e-5, 0.1, None, None, 1, 1, 0, 0, 0) == native.EINVAL
    assert not h.value
    assert lib.ssoct_slide_create(None, None, lam, 1e-5, 0.1, None, None, 1, 1, 0, 0, 0) == native.EINVAL
    assert lib.ssoct_slide_push(None, None, 1, 0) == native.EINVAL
    ptr = ctypes.c_void_p()
    assert lib.ssoct_slide_ring(None, ctypes.byref(ptr)) == native.EINVAL
    assert lib.ssoct_slide_advance(None, 1, 0) == native.EINVAL
    assert lib.ssoct_slide_pop(None, 1, None, None, None, None, None, None) == native.EINVAL
    assert lib.ssoct_slide_volume(None, 0, ctypes.byref(ptr)) == native.EINVAL
    c = (ctypes.c_uint64 * 5)()
    assert lib.ssoct_slide_stats(None, c) == native.EINVAL
    assert lib.ssoct_slide_destroy(None) == native.OK
