"""Parity at the paper-shaped size (T = 256 frames of 1024 x 1024), in the
launch configuration bench.py times (default chunking and grids), on pixel
columns the oracle evaluates by direct sums, plus exact properties of the
whole volume."""
import numpy as np
import pytest
import torch

from oracle import ssoct_oracle as O
from paper_2003_08960_amd import synth

pytestmark = pytest.mark.gpu

T, N = 256, 1024
PITCH, Z = 12e-6, 0.3
PIXELS = [(0, 0), (N // 2, N // 2), (N - 1, N - 1), (3, N - 2), (640, 700), (N // 2 + N // 8, N // 2 + N // 8)]


@pytest.fixture(scope="module")
def case():
    frames = synth.random_frames(T, N, seed=2024, lo=0, hi=65535)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    ref = O.render_columns(frames, lam, PITCH, Z, PIXELS)
    e_j = sum(float(np.sum(O.rescale(frames[t], s) ** 2)) for t, s in enumerate(O.scale_factors(lam)))
    return frames, lam, ref, e_j


@pytest.mark.parametrize("precision,bar", [("fp32_fft", 1e-5), ("fp32", 1e-5), ("bf16_split", 1e-4),
                                           ("fp16_split", 1e-4), ("fp32_4step", 1e-5), ("bf16_split_4step", 1e-4),
                                           ("fp16_split_4step", 1e-4)])
def test_paper_size_sampled_columns(gpu_lib, case, precision, bar):
    from paper_2003_08960_amd.api import Plan
    frames, lam, ref, e_j = case
    print(f"\n[gpu] full size T={T} N={N} {precision}", flush=True)
    plan = Plan(T, N, precision=precision)
    fr = torch.from_numpy(frames).cuda()
    V = plan.render(fr, lam, PITCH, Z)
    got = np.stack([V[:, u, v].cpu().numpy() for u, v in PIXELS], axis=1)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"{precision}: sampled rel-L2 {err:.3e}")
    assert err <= bar
    # Parseval over the whole volume: sum |V|^2 = T N^2 sum_t ||J_t||^2 (J: rescaled frames)
    e_v = float(torch.sum(torch.abs(V.to(torch.complex128)) ** 2).item())
    assert abs(e_v / (T * N * N * e_j) - 1.0) <= (1e-5 if precision.startswith("fp32") else 1e-4)
    xy, xz, yz = plan.cuts(V, N // 2, N // 2, T // 4)
    assert torch.allclose(xy, torch.abs(V[T // 4]), rtol=1e-6, atol=0)
