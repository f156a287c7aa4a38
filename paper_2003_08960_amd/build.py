"""Build libssoct.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

    python -m paper_2003_08960_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libssoct.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = "gfx950"

HIP_SOURCES = ["tables.hip", "stage_a.hip", "depth.hip", "depth_fft.hip", "depth_4step.hip", "misc.hip", "noalloc.hip"]
CPP_SOURCES = ["abi.cpp", "stream.cpp", "slide.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", f"-I{os.path.join(ROOT, 'include')}"]
# packed FP32 instructions are kept out of every kernel (the compiler would otherwise form them from
# scalar and float2 code)
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast", "-munsafe-fp-atomics"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libssoct.so")


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"command failed ({res.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False, jobs: int | None = None, out: str | None = None,
          defines: dict | None = None) -> str:
    """Compile every source and link libssoct.so (or `out`); `defines` are -D
    tuning macros of the kernels (a variant build goes to its own object dir)."""
    cc = hipcc()
    out = out or OUT
    defs = [f"-D{k}={v}" for k, v in sorted((defines or {}).items())]
    bdir = BUILD if not defs else os.path.join(BUILD, "variant_" + "_".join(d[2:] for d in defs).replace("=", ""))
    os.makedirs(bdir, exist_ok=True)
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmds.append([cc, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + DEVICE + defs)
        objs.append(obj)
    for src in CPP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmds.append([cc, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + [f"--offload-arch={ARCH}"] + defs)
        objs.append(obj)
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for res in ex.map(_run, cmds):
            if verbose and res.strip():
                print(res)
    tmp = out + ".tmp"
    _run([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv)
    print(path)
