"""GPU parity of the apodised gate and of the depth transform for sweeps that
are not linear in k (SSOCT_NONUNIFORM_K), against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import ssoct_oracle as O
from paper_2003_08960_amd import native, synth

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


@pytest.fixture(scope="module")
def chirped():
    cfg = synth.SweepConfig(T=32, N=128, pitch=20e-6, z=0.3, lam_max=870e-9, lam_min=800e-9, n_scatterers=5,
                            k_bend=0.3, name="chirped")
    return synth.make_sweep(cfg, seed=21)


def render(sw, precision, gate=None, nonuniform_k=False, **kw):
    from paper_2003_08960_amd.api import Plan
    T, N = sw.frames.shape[:2]
    print(f"\n[gpu] render T={T} N={N} {precision} gate={gate is not None} nonuniform_k={nonuniform_k}", flush=True)
    plan = Plan(T, N, precision=precision, nonuniform_k=nonuniform_k, **kw)
    if gate is not None:
        plan.set_gate(gate)
    V = plan.render(torch.from_numpy(sw.frames).cuda(), sw.lam, sw.pitch, sw.z)
    torch.cuda.synchronize()
    return plan, V


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-5), ("fp16_split", 1e-4), ("bf16_split", 1e-4),
                                           ("fp16", 2e-2)])
def test_nonuniform_k_matches_oracle(gpu_lib, chirped, precision, bar):
    _, V = render(chirped, precision, nonuniform_k=True)
    ref = O.render(chirped.frames, chirped.lam, chirped.pitch, chirped.z, nonuniform_k=True)
    err = rel_l2(V.cpu().numpy(), ref)
    print(f"{precision} rel-L2 {err:.3e}")
    assert err <= bar


@pytest.mark.parametrize("T", [1, 2, 33, 100, 130])
def test_nonuniform_k_ragged_sweeps(gpu_lib, T):
    frames = synth.random_frames(T, 32, seed=T + 5)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9, bend=0.2)
    from paper_2003_08960_amd.api import Plan
    if T == 1:
        lam = np.array([850e-9])
    plan = Plan(T, 32, nonuniform_k=True)
    V = plan.render(torch.from_numpy(frames).cuda(), lam, 20e-6, 0.05)
    assert rel_l2(V.cpu().numpy(), O.render(frames, lam, 20e-6, 0.05, nonuniform_k=True)) <= 1e-5


def test_nonuniform_k_refocuses_a_chirped_sweep(gpu_lib, chirped):
    """Each scatterer's envelope peaks at its generator bin only with the non-uniform transform."""
    _, Vn = render(chirped, "fp32", nonuniform_k=True)
    _, Vd = render(chirped, "fp32")
    An, Ad = torch.abs(Vn).cpu().numpy(), torch.abs(Vd).cpu().numpy()
    gain = []
    for u, v, q, _ in chirped.scatterers:
        u, v, q = int(u), int(v), int(q)
        col_n, col_d = An[:, u, v], Ad[:, u, v]
        assert int(np.argmax(col_n[1:])) + 1 == q
        gain.append(col_n[q] / col_d.max())
    assert min(gain) > 1.2


@pytest.mark.parametrize("precision,nonuniform", [("fp32", False), ("fp32_fft", False), ("bf16_split", False),
                                                  ("fp32", True)])
def test_hann_gate_matches_oracle(gpu_lib, chirped, precision, nonuniform):
    T = chirped.frames.shape[0]
    g = np.sin(np.pi * np.arange(T) / T) ** 2
    plan, V = render(chirped, precision, gate=g, nonuniform_k=nonuniform)
    ref = O.render(chirped.frames, chirped.lam, chirped.pitch, chirped.z, gate=g, nonuniform_k=nonuniform)
    bar = 1e-4 if precision.endswith("split") else 1e-5
    assert rel_l2(V.cpu().numpy(), ref) <= bar
    # clearing the gate restores the rectangular-gate volume bit for bit
    plan.set_gate(None)
    V0 = plan.render(torch.from_numpy(chirped.frames).cuda(), chirped.lam, chirped.pitch, chirped.z).clone()
    plan2, V1 = render(chirped, precision, nonuniform_k=nonuniform)
    assert torch.equal(V0, V1)


def test_gate_and_nonuniform_k_rejections(gpu_lib, chirped):
    from paper_2003_08960_amd.api import Plan, Slide, Stream
    T, N = chirped.frames.shape[:2]
    fr = torch.from_numpy(chirped.frames).cuda()
    plan = Plan(T, N, backward=True)
    plan.set_gate(np.hanning(T))
    with pytest.raises(native.SsoctError) as e:
        plan.backward_sharpness(fr, chirped.lam, chirped.pitch, chirped.z)
    assert e.value.code == native.EUNSUPPORTED
    with pytest.raises(native.SsoctError) as e:
        Slide(plan, chirped.lam, chirped.pitch, chirped.z, hop=4)
    assert e.value.code == native.EUNSUPPORTED
    plan.set_gate(None)
    st = Stream(plan, chirped.lam, chirped.pitch, chirped.z, slots=1)
    with pytest.raises(native.SsoctError):
        plan.set_gate(np.ones(T))                 # parameters are fixed while streaming
    st.close()
    plan.set_gate(np.ones(T))
    with pytest.raises(native.SsoctError) as e:
        Plan(T, N, nonuniform_k=True, backward=True).backward_sharpness(fr, chirped.lam, chirped.pitch, chirped.z)
    assert e.value.code == native.EUNSUPPORTED
