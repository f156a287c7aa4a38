#!/usr/bin/env python3
"""Throughput of the paper-shaped render on one MI355X.

Workload: one sweep of T = 256 uint16 frames of 1024 x 1024 (synthetic,
seeded: 200 point scatterers + speckle, 12 um pixels, 870 -> 800 nm sweep,
z = 0.3 m), frames resident in HBM.  One step = one whole render (tables,
rescale + chirp + 2-D DFT of every frame, depth DFT, complex volume written)
plus the three envelope cuts.  Every precision form of the depth transform
is timed; the headline value is the fastest form whose error against the
FP64 oracle (sampled pixel columns) is within 1e-4.

    python bench.py [--steps K] [--warmup W]

Prints progress on stderr and ONE JSON line on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gvoxel/s per volume, FP32 vs split-prec MFMA depth-DFT at rel-L2≤1e-4; %HBM"
HBM_PEAK = 8.0e12                       # B/s, MI355X HBM3E
MFMA_PEAK = {"fp32": 157.3e12, "fp16": 2.5e15, "bf16": 2.5e15}
FRESNEL_BYTES_PER_VOXEL = 10            # u16 frame in + H out
DEPTH_BYTES_PER_VOXEL = 16              # H in + complex64 volume out
PATH_BYTES_PER_VOXEL = 26
SPLIT_BAR = 1e-4
FP32_BAR = 1e-5
PAPER_GVOXEL_S = 10.0                   # paper's table (TITAN Xp, sliding STFT), context only


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def depth_products(form: str) -> int:
    return 3 if form.endswith("_split") else 1


def depth_flops(T: int, N: int, form: str) -> float:
    # real form of the complex DFT matrix: 4 T^2 real flops per pixel per product
    return 4.0 * T * T * N * N * depth_products(form)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2003_08960_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counters, if taken on this exact kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def sampled_pixels(sw, n_random=6, seed=5):
    N = sw.frames.shape[1]
    rng = np.random.default_rng(seed)
    pix = [(int(u), int(v)) for u, v, _, _ in sw.scatterers[:4]]
    pix += [(int(a), int(b)) for a, b in rng.integers(0, N, size=(n_random, 2))]
    pix.append((N // 2, N // 2))
    return pix


def cpu_baseline(sw, n_frames=32, n_cols=65536):
    """The FP64 oracle timed on a bounded sample of the same workload, scaled to one volume."""
    from oracle import ssoct_oracle as O
    T, N, _ = sw.frames.shape
    s = O.scale_factors(sw.lam)
    alpha = O.chirp_rates(sw.lam, sw.pitch, sw.z)
    t0 = time.perf_counter()
    for t in range(n_frames):
        J = O.rescale(sw.frames[t], s[t])
        O.fresnel_fft(O.chirp(N, alpha[t]) * J)
    t_frames = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    h = rng.standard_normal((T, n_cols)) + 1j * rng.standard_normal((T, n_cols))
    t0 = time.perf_counter()
    O.depth_dft(h)
    t_depth = time.perf_counter() - t0
    per_volume = t_frames / n_frames * T + t_depth * (N * N / n_cols)
    return {
        "value": T * N * N / per_volume / 1e9,
        "unit": "Gvoxel/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle steps 1-2 (rescale, chirp, Fresnel DFT) on {n_frames} of {T} frames of {N}x{N} "
                   f"and the depth DFT on {n_cols} of {N * N} pixel columns, numpy FP64 single thread, "
                   f"scaled to one {T}x{N}x{N} volume ({per_volume:.1f} s/volume)"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forms", default="fp32,fp16_split,bf16_split,fp16,bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one untimed 1 GiB device-to-device copy first: the reference kernel that "
                         "scales rocprofv3 FETCH_SIZE/WRITE_SIZE readings to bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the render of one sweep runs on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2003_08960_amd import native, synth
    from paper_2003_08960_amd.api import Plan

    native.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    log("generating the paper-shaped sweep (T=256, N=1024)")
    sw = synth.make_config("paper")
    T, N, _ = sw.frames.shape
    voxels = T * N * N
    frames = torch.from_numpy(sw.frames).to(dev)

    pix = sampled_pixels(sw)
    ref_cols = None
    if not args.no_accuracy:
        from oracle import ssoct_oracle as O
        log(f"oracle reference on {len(pix)} sampled pixel columns")
        ref_cols = O.render_columns(sw.frames, sw.lam, sw.pitch, sw.z, pix)

    forms = {}
    x0, y0, q0 = N // 2, N // 2, T // 4
    for form in [f for f in args.forms.split(",") if f]:
        plan = Plan(T, N, precision=form, profile=True)
        vol = torch.empty((T, N, N), dtype=torch.complex64, device=dev)
        for _ in range(args.warmup):
            plan.render(frames, sw.lam, sw.pitch, sw.z, out=vol)
            plan.cuts(vol, x0, y0, q0)
        torch.cuda.synchronize()
        plan.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.render(frames, sw.lam, sw.pitch, sw.z, out=vol)
            plan.cuts(vol, x0, y0, q0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stage = plan.profile_read()
        ms = (t1 - t0) * 1e3 / args.steps
        rec = {"ms_per_step": ms, "gvoxel_s": voxels / (ms * 1e-3) / 1e9,
               "stage_ms": {"tables": stage[0], "fresnel": stage[1], "depth": stage[2]},
               "hbm_frac_path": PATH_BYTES_PER_VOXEL * voxels / (ms * 1e-3) / HBM_PEAK}
        if ref_cols is not None:
            got = np.stack([vol[:, u, v].cpu().numpy() for u, v in pix], axis=1)
            rec["rel_l2_sampled"] = float(np.linalg.norm(got - ref_cols) / np.linalg.norm(ref_cols))
        forms[form] = rec
        log(f"{form}: {ms:.3f} ms/step, {rec['gvoxel_s']:.1f} Gvoxel/s, stages {stage[1]:.3f} / {stage[2]:.3f} ms"
            + (f", rel-L2 {rec['rel_l2_sampled']:.2e}" if "rel_l2_sampled" in rec else ""))
        del plan, vol
        torch.cuda.empty_cache()

    def ok(f):
        r = forms[f]
        return "rel_l2_sampled" not in r or r["rel_l2_sampled"] <= (FP32_BAR if f == "fp32" else SPLIT_BAR)

    eligible = [f for f in forms if ok(f)] or list(forms)
    head = max(eligible, key=lambda f: forms[f]["gvoxel_s"])
    hr = forms[head]
    prec = head.split("_")[0]

    # roofline of the dominant kernel of the headline form, from the live HIP-event stage times
    st = hr["stage_ms"]
    if st["depth"] >= st["fresnel"]:
        flops = depth_flops(T, N, head)
        byts = DEPTH_BYTES_PER_VOXEL * voxels
        t = st["depth"] * 1e-3
        if flops / MFMA_PEAK[prec] >= byts / HBM_PEAK:
            roof = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": MFMA_PEAK[prec] / 1e12, "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": byts / t / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
        roof["kernel"] = "k_depth (depth DFT, 1 launch per step)"
        roof["traffic"] = traffic_record(f"k_depth_{head}")
    else:
        byts = FRESNEL_BYTES_PER_VOXEL * voxels
        t = st["fresnel"] * 1e-3
        roof = {"bound": "hbm", "achieved": byts / t / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "kernel": "k_row_pass + k_col_pass (Fresnel stage, all frame chunks)",
                "traffic": traffic_record(f"fresnel_{head}")}
    roof["frac"] = roof["achieved"] / roof["peak"]

    out = {
        "metric": METRIC,
        "value": hr["gvoxel_s"],
        "unit": "Gvoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32" if head == "fp32" else f"{prec}{'-split' if head.endswith('_split') else ''} depth DFT, f32 acc; "
                  "f32 Fresnel stage"),
        "data": "synthetic",
        "config": {"workload": f"paper-shaped sweep: T={T} uint16 frames of {N}x{N}, 200 scatterers + speckle, "
                               "one rectangular depth gate of all frames, complex64 volume + 3 cuts",
                   "T": T, "N": N, "form": head, "pitch_m": sw.pitch, "z_m": sw.z},
        "roofline": roof,
        "hbm_frac_whole_path": hr["hbm_frac_path"],
        "forms": forms,
        "paper_context_gvoxel_s": PAPER_GVOXEL_S,
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample (CPU)")
        out["cpu_baseline"] = cpu_baseline(sw)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
