"""GPU parity of angular-spectrum propagation (SSOCT_ANGULAR_SPECTRUM) against
the FP64 oracle: every frame propagated at its own wavelength on the sensor
grid, then the depth transform."""
import numpy as np
import pytest
import torch

from oracle import ssoct_oracle as O
from paper_2003_08960_amd import native, synth

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def gpu_as(frames, lam, pitch, z, precision="fp32", disp=None, gate=None, **kw):
    from paper_2003_08960_amd.api import Plan
    T, N, _ = frames.shape
    print(f"\n[gpu] angular spectrum T={T} N={N} {precision} pitch={pitch} z={z}", flush=True)
    plan = Plan(T, N, precision=precision, angular_spectrum=True, **kw)
    if gate is not None:
        plan.set_gate(gate)
    V = plan.render(torch.from_numpy(np.ascontiguousarray(frames)).cuda(), lam, pitch, z, disp)
    torch.cuda.synchronize()
    return plan, V


@pytest.mark.parametrize("T,N,pitch,z", [(8, 16, 10e-6, 0.004), (5, 64, 12e-6, 0.002), (16, 128, 0.4e-6, 20e-6),
                                         (4, 256, 12e-6, 0.01), (3, 512, 6e-6, 0.003), (2, 1024, 12e-6, 0.05),
                                         (1, 2048, 5e-6, 0.001)])
def test_as_sizes(gpu_lib, T, N, pitch, z):
    frames = synth.random_frames(T, N, seed=N + T)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    _, V = gpu_as(frames, lam, pitch, z)
    ref = O.render_as(frames, lam, pitch, z)
    err = rel_l2(V.cpu().numpy(), ref)
    print(f"rel-L2 {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-5), ("fp32_fft", 1e-5), ("bf16_split", 1e-4),
                                           ("fp16_split", 1e-4)])
def test_as_forms_with_dispersion_and_gate(gpu_lib, precision, bar):
    T, N = 32, 128
    frames = synth.random_frames(T, N, seed=5)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    rng = np.random.default_rng(6)
    disp = rng.normal(0, 1.0, T)
    gate = np.hanning(T)
    _, V = gpu_as(frames, lam, 12e-6, 0.004, precision, disp=disp, gate=gate)
    ref = O.render_as(frames, lam, 12e-6, 0.004, disp, gate)
    assert rel_l2(V.cpu().numpy(), ref) <= bar


def test_as_point_source_focuses(gpu_lib):
    """A reflector at depth bin q_m recorded at z well below z_b (where the Fresnel transform is
    undersampled).  Its band-limited field on the sensor is the one that Eq. 6 refocuses at +z
    (the point propagated by -z: phase exp(+i k r)); interfering with a plane reference, it
    refocuses by +z, as with the Fresnel transform, to a peak at its pixel and depth bin; the twin
    image lands at T - q_m, defocused."""
    T, N, d, z, qm = 16, 128, 8e-6, 0.002, 5
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    assert z < N * d * d / lam.max()
    k = 2 * np.pi / lam
    dk = (k[-1] - k[0]) / (T - 1)
    delta = qm * np.pi / (T * dk)
    point = np.zeros((N, N))
    point[N // 2, N // 2 + 9] = 40.0
    frames = np.empty((T, N, N), np.uint16)
    for t in range(T):
        E = np.exp(2j * (k[t] - k[0]) * delta) * O.as_propagate(point, lam[t], d, -z)
        frames[t] = np.clip(np.round(4000 * np.abs(1.0 + E) ** 2), 0, 65535).astype(np.uint16)
    plan, V = gpu_as(frames, lam, d, z)
    A = torch.abs(V).cpu().numpy()
    A[0] = 0.0                                                  # reference (DC) bin
    q, i, j = np.unravel_index(np.argmax(A), A.shape)
    assert (q, i, j) == (qm, N // 2, N // 2 + 9)
    assert A[T - qm].max() < 0.3 * A[qm, i, j]                  # twin image: defocused
    ref = O.render_as(frames, lam, d, z)
    assert rel_l2(V.cpu().numpy(), ref) <= 1e-5


def test_as_sliding_window(gpu_lib):
    from paper_2003_08960_amd.api import Plan, Slide
    T, N = 16, 64
    frames = synth.random_frames(2 * T + 3, N, seed=9)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    plan = Plan(T, N, angular_spectrum=True)
    sl = Slide(plan, lam, 10e-6, 0.003, hop=4, slots=2)
    got = {}
    for seq in range(0, frames.shape[0], 4):
        n = min(4, frames.shape[0] - seq)
        assert sl.push(np.ascontiguousarray(frames[seq:seq + n]), seq) == native.OK
        while (r := sl.pop(wait=True)) is not None:
            got[r["start"]] = sl.volume(r["slot"]).clone()
            torch.cuda.synchronize()      # the copy is done before a later window may reuse the slot
    sl.close()
    assert sorted(got) == list(range(0, frames.shape[0] - T + 1, 4))
    for j in got:
        idx = [(j + i) % T for i in range(T)]
        ref = O.render_as(frames[j:j + T], lam[idx], 10e-6, 0.003)
        assert rel_l2(got[j].cpu().numpy(), ref) <= 1e-5


def test_as_rejections(gpu_lib):
    from paper_2003_08960_amd.api import Plan
    for kw in ({"eq6_phase": True}, {"exact_chirp": True}):
        with pytest.raises(native.SsoctError) as e:
            Plan(8, 32, angular_spectrum=True, **kw)
        assert e.value.code == native.EINVAL
    frames = torch.from_numpy(synth.random_frames(8, 32, seed=1)).cuda()
    lam = synth.sweep_wavelengths(8, 870e-9, 800e-9)
    plan = Plan(8, 32, angular_spectrum=True, backward=True)
    with pytest.raises(native.SsoctError) as e:
        plan.render(frames, lam, 10e-6, 0.01, None, np.zeros(15))
    assert e.value.code == native.EUNSUPPORTED
    with pytest.raises(native.SsoctError) as e:
        plan.backward_sharpness(frames, lam, 10e-6, 0.01)
    assert e.value.code == native.EUNSUPPORTED


def test_as_column_walk_is_independent_of_the_workgroup_count(gpu_lib):
    """At N = 1024 the transfer-function column pass keeps its twiddles in LDS and prefetches the
    next tile, walking tiles across frames: one workgroup walking every tile, a grid that does not
    divide the tiles, more workgroups than tiles, and ragged frame chunks give bit-identical volumes;
    the default is within the FP32 bar of the oracle."""
    from paper_2003_08960_amd.api import Plan
    T, N, d, z = 16, 1024, 12e-6, 0.01
    frames = synth.random_frames(T, N, seed=93)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    fr = torch.from_numpy(frames).cuda()
    print(f"\n[gpu] angular-spectrum column grids T={T} N={N}", flush=True)
    plan = Plan(T, N, precision="fp32_fft", angular_spectrum=True)
    V0 = plan.render(fr, lam, d, z).clone()
    for F, cg in ((16, 1), (5, 37), (16, 4096), (7, 0)):
        plan.set_tuning([F, cg, 0])
        assert torch.equal(plan.render(fr, lam, d, z), V0), (F, cg)
    ref = O.render_as(frames, lam, d, z)
    err = rel_l2(V0.cpu().numpy(), ref)
    print(f"rel-L2 {err:.3e}")
    assert err <= 1e-5
