"""The allocation-free render entry point (ssoct_plan_render_noalloc) against
the render with a caller workspace (ssoct_plan_render), through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2003_08960_amd import native, synth

pytestmark = pytest.mark.gpu


def _case(T, N, seed):
    frames = synth.random_frames(T, N, seed)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    return torch.from_numpy(frames).cuda(), lam


def test_noalloc_matches_the_workspace_render(gpu_lib):
    """Two calls in a row on one device, the second on a smaller input: each volume equals the
    ordinary render's bit for bit.  The first (T = 96, N = 512) needs its frame chunk lowered from 64
    to 32 frames to fit the 256 MiB array; the second is the tiny size in split BF16 with dispersion
    and aberration."""
    from paper_2003_08960_amd.api import Plan
    cases = [(96, 512, "fp32", False), (32, 128, "bf16_split", True)]
    for i, (T, N, prec, extras) in enumerate(cases):
        print(f"\n[gpu] noalloc call {i}: T={T} N={N} {prec}", flush=True)
        fr, lam = _case(T, N, seed=300 + i)
        rng = np.random.default_rng(i)
        disp = rng.uniform(-1, 1, T) if extras else None
        zern = rng.normal(0, 0.3, 15) if extras else None
        plan = Plan(T, N, precision=prec)
        ref = plan.render(fr, lam, 12e-6, 0.3, disp, zern)
        out = torch.full((T, N, N), float("nan"), dtype=torch.complex64, device="cuda")
        got = plan.render_noalloc(fr, lam, 12e-6, 0.3, disp, zern, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref), (T, N, prec)
        plan.close()


def test_noalloc_with_the_second_radix_order(gpu_lib):
    """The allocation-free render follows the plan's launch shapes: with the column transforms in the
    second radix order (4 16 16 at N = 1024 is 8 16 at N = 128) it equals the ordinary render of the
    same plan bit for bit."""
    from paper_2003_08960_amd.api import Plan
    T, N = 32, 128
    print(f"\n[gpu] noalloc radix order 1: T={T} N={N} fp32_fft", flush=True)
    fr, lam = _case(T, N, seed=310)
    plan = Plan(T, N, precision="fp32_fft")
    t = plan.get_tuning()
    t[8] = 1
    plan.set_tuning(t)
    ref = plan.render(fr, lam, 12e-6, 0.3)
    got = plan.render_noalloc(fr, lam, 12e-6, 0.3, out=torch.empty_like(ref))
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    plan.close()


def test_noalloc_rejects_a_workspace_beyond_the_array(gpu_lib):
    from paper_2003_08960_amd.api import Plan
    T, N = 256, 1024        # H alone is 2 GiB
    plan = Plan(T, N, precision="fp32_fft")
    fr = torch.zeros((T, N, N), dtype=torch.uint16, device="cuda")
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    with pytest.raises(native.SsoctError) as e:
        plan.render_noalloc(fr, lam, 12e-6, 0.3, out=torch.empty((T, N, N), dtype=torch.complex64, device="cuda"))
    assert e.value.code == native.EUNSUPPORTED
    assert "256 MiB" in str(e.value)
