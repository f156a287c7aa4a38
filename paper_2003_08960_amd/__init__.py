"""MI355X-native renderer for swept-source holographic OCT (arXiv 2003.08960).

The compute path is libssoct.so (hand-written HIP kernels for gfx950 behind a
C ABI, include/ssoct.h); this package holds its build script, the ctypes
binding, a torch-facing wrapper (Plan), an autograd Function and the seeded
synthetic input generator.
"""
__all__ = ["Plan", "native", "synth"]


def __getattr__(name):
    if name == "Plan":
        from .api import Plan
        return Plan
    raise AttributeError(name)
