"""Seeded random sweep over valid combinations of sizes, depth forms and
options, each compared with the FP64 oracle (and, for the dense forms, to the
same bars as the targeted tests)."""
import numpy as np
import pytest
import torch

from oracle import ssoct_oracle as O
from paper_2003_08960_amd import synth

pytestmark = pytest.mark.gpu

FORMS = ["fp32", "fp32_fft", "fp16_split", "bf16_split", "fp32_4step", "bf16_split_4step", "fp16_split_4step"]


def make_case(seed):
    rng = np.random.default_rng(1000 + seed)
    form = FORMS[seed % len(FORMS)]
    N = int(rng.choice([16, 32, 64, 128, 256]))
    if form == "fp32_fft":
        T = int(rng.choice([16, 32, 64]))
    elif form.endswith("_4step"):
        T = int(rng.choice([32, 64]))
    else:
        T = int(rng.integers(1, 70))
    prop = "as" if rng.random() < 0.3 else "fresnel"
    opts = {}
    if prop == "fresnel":
        opts["exact_chirp"] = bool(rng.random() < 0.3)
        opts["eq6_phase"] = bool(rng.random() < 0.3)
        opts["zern"] = rng.normal(0, 0.3, 15) if rng.random() < 0.4 else None
    opts["disp"] = rng.normal(0, 1.0, T) if rng.random() < 0.4 else None
    opts["gate"] = rng.uniform(0.2, 1.0, T) if rng.random() < 0.4 else None
    opts["nonuniform_k"] = form in ("fp32", "fp16_split", "bf16_split") and T > 1 and rng.random() < 0.3
    opts["order"] = int(rng.random() < 0.5) if form == "fp32_fft" else 0
    opts["chunk"] = int(rng.integers(1, 9))
    bend = 0.25 if opts["nonuniform_k"] else 0.0
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9, bend=bend) if T > 1 else np.array([850e-9])
    pitch = float(rng.choice([8e-6, 12e-6, 20e-6]))
    z = float(rng.choice([0.01, 0.05, 0.3])) if prop == "fresnel" else float(rng.choice([-0.003, 0.002, 0.01]))
    opts["radix"] = int(rng.random() < 0.5) if prop == "fresnel" and N not in (16, 256) else 0
    frames = synth.random_frames(T, N, seed=seed, lo=0, hi=65535)
    return form, prop, T, N, lam, pitch, z, frames, opts


@pytest.mark.parametrize("seed", range(64))
def test_random_configuration(gpu_lib, seed):
    from paper_2003_08960_amd.api import Plan
    form, prop, T, N, lam, pitch, z, frames, o = make_case(seed)
    print(f"\n[gpu] random {seed}: {form} {prop} T={T} N={N} z={z} "
          f"{ {k: (v if not isinstance(v, np.ndarray) else 'array') for k, v in o.items()} }", flush=True)
    plan = Plan(T, N, precision=form, angular_spectrum=prop == "as", nonuniform_k=o["nonuniform_k"],
                exact_chirp=o.get("exact_chirp", False), eq6_phase=o.get("eq6_phase", False))
    if o["gate"] is not None:
        plan.set_gate(o["gate"])
    tun = plan.get_tuning()
    plan.set_tuning([min(o["chunk"], tun[0]), 0, 0, o["order"], 0, 0, 0, 0, o["radix"]])
    V = plan.render(torch.from_numpy(frames).cuda(), lam, pitch, z, o["disp"], o.get("zern")).cpu().numpy()
    if prop == "as":
        ref = O.render_as(frames, lam, pitch, z, o["disp"], o["gate"], o["nonuniform_k"])
    else:
        ref = O.render(frames, lam, pitch, z, o["disp"], o.get("zern"), o["exact_chirp"], o["eq6_phase"],
                       gate=o["gate"], nonuniform_k=o["nonuniform_k"])
    err = float(np.linalg.norm(V - ref) / np.linalg.norm(ref))
    bar = 1e-4 if "split" in form else 1e-5
    print(f"rel-L2 {err:.3e} (bar {bar})")
    assert err <= bar
