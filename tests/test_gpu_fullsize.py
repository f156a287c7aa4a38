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


# ---------------------------------------------------------------- every voxel of the paper-shaped sweep

def rel_l2_blocked(V, ref, nb=16):
    """rel-L2 of a device volume against an FP64 reference over all voxels, and over the bins q != 0
    (the DC bin of the interferograms dominates the norm), moving nb bins at a time to the host."""
    num = den = num_ac = den_ac = 0.0
    for q0 in range(0, ref.shape[0], nb):
        g = V[q0:q0 + nb].cpu().numpy().astype(np.complex128)
        r = ref[q0:q0 + nb]
        d2 = np.abs(g - r) ** 2
        r2 = np.abs(r) ** 2
        num += float(d2.sum())
        den += float(r2.sum())
        if q0 == 0:
            d2, r2 = d2[1:], r2[1:]
        num_ac += float(d2.sum())
        den_ac += float(r2.sum())
    return float(np.sqrt(num / den)), float(np.sqrt(num_ac / den_ac))


@pytest.fixture(scope="module")
def paper():
    """The paper-shaped synthetic sweep (200 scatterers + speckle, seed 3) and its FP64 oracle volume,
    computed once for the module (about a minute on the host)."""
    sw = synth.make_config("paper")
    print("\n[oracle] rendering the paper-shaped sweep in FP64", flush=True)
    ref = O.render(sw.frames, sw.lam, sw.pitch, sw.z)
    return sw, ref


@pytest.mark.parametrize("precision,order,radix,bar", [("fp32_fft", None, 0, 1e-5), ("fp32_fft", 0, 0, 1e-5),
                                                       ("fp32", None, 0, 1e-5), ("bf16_split", None, 0, 1e-4),
                                                       ("bf16_split_4step", None, 0, 1e-4),
                                                       ("fp32_fft", None, 1, 1e-5), ("bf16_split_4step", None, 1, 1e-4)])
def test_paper_volume_every_voxel(gpu_lib, paper, precision, order, radix, bar):
    """The whole 1024 x 1024 x 256 volume against the oracle, element by element, in the launch
    configuration the bench times (default chunking, grids and evaluation order: depth first for the
    FFT form), the FFT form also in the frame order, the column transforms also in the second radix
    order (4 16 16, which the tuner may choose), and the three cuts."""
    from paper_2003_08960_amd.api import Plan
    sw, ref = paper
    print(f"\n[gpu] paper volume, every voxel, {precision} order {order} radix order {radix}", flush=True)
    plan = Plan(T, N, precision=precision)
    t = plan.get_tuning()
    if order is not None:
        t[3] = order
    t[8] = radix
    plan.set_tuning(t)
    V = plan.render(torch.from_numpy(sw.frames).cuda(), sw.lam, sw.pitch, sw.z)
    err, err_ac = rel_l2_blocked(V, ref)
    print(f"{precision}: rel-L2 all voxels {err:.3e}, bins q != 0 {err_ac:.3e}")
    assert err <= bar
    xy, xz, yz = plan.cuts(V, N // 2, N // 2, T // 4)
    for got, want in zip((xy, xz, yz), O.cuts(ref, N // 2, N // 2, T // 4)):
        assert float(np.linalg.norm(got.cpu().numpy() - want) / np.linalg.norm(want)) <= bar
    plan.close()


def test_paper_stream_host_fed_volume(gpu_lib, paper):
    """One streamed volume of the paper-shaped sweep in the bench's streaming configuration (factored
    BF16-split depth form, tuned launch shapes), host-fed from pinned memory in 16-frame pushes: bit for
    bit the eager render of the same plan, and within the split bar of the oracle."""
    from paper_2003_08960_amd import native
    from paper_2003_08960_amd.api import Plan, Stream
    sw, ref = paper
    print("\n[gpu] paper-shaped stream, host-fed, bf16_split_4step tuned", flush=True)
    plan = Plan(T, N, precision="bf16_split_4step")
    fr = torch.from_numpy(sw.frames).cuda()
    tuning = plan.tune(fr, sw.lam, sw.pitch, sw.z)
    eager = plan.render(fr, sw.lam, sw.pitch, sw.z).clone()
    print(f"tuning {tuning}")
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=2)
    pinned = torch.from_numpy(sw.frames).pin_memory()
    for s0 in range(0, T, 16):
        assert st.push_frames(pinned[s0:s0 + 16], s0) == native.OK
    r = st.pop(wait=True)
    assert r["seq"] == 0
    V = st.slot_volume(r["slot"])
    assert torch.equal(V, eager)
    err, _ = rel_l2_blocked(V, ref)
    print(f"streamed volume rel-L2 {err:.3e}")
    assert err <= 1e-4
    st.close()
    plan.close()


def test_paper_sliding_window_hop13(gpu_lib, paper):
    """The paper's mode at its size: a gate of 256 frames advanced by 13 over a stream that repeats the
    sweep.  Window 0 is the sweep itself; window 13 holds frames 13 .. 268, i.e. the sweep rotated by 13
    frames with the wavelengths of its sweep positions, which the oracle renders in time order."""
    from paper_2003_08960_amd import native
    from paper_2003_08960_amd.api import Plan, Slide
    sw, ref = paper
    hop = 13
    print("\n[gpu] paper-shaped sliding windows, hop 13", flush=True)
    plan = Plan(T, N, precision="fp32_fft")
    sl = Slide(plan, sw.lam, sw.pitch, sw.z, hop=hop, slots=2)
    pinned = torch.from_numpy(sw.frames).pin_memory()
    got = {}
    seq = 0
    while seq < T + hop:
        n = min(hop, T + hop - seq)
        pos = seq % T
        if pos + n <= T:
            assert sl.push(pinned[pos:pos + n], seq) == native.OK
        else:
            assert sl.push(pinned[pos:], seq) == native.OK
            assert sl.push(pinned[:pos + n - T], seq + T - pos) == native.OK
        seq += n
        while (r := sl.pop(wait=True)) is not None:
            got[r["start"]] = sl.volume(r["slot"]).clone()
            torch.cuda.synchronize()      # the copy is done before a later window may reuse the slot
    sl.close()
    assert sorted(got) == [0, hop]
    err0, _ = rel_l2_blocked(got[0], ref)
    print(f"window 0 rel-L2 {err0:.3e}")
    assert err0 <= 1e-5
    idx = (np.arange(T) + hop) % T
    print("[oracle] rendering window 13 in FP64", flush=True)
    ref13 = O.render(sw.frames[idx], sw.lam[idx], sw.pitch, sw.z)
    err13, _ = rel_l2_blocked(got[hop], ref13)
    print(f"window 13 rel-L2 {err13:.3e}")
    assert err13 <= 1e-5
    plan.close()


def test_vjp_at_frame_size_1024(gpu_lib):
    """ssoct_backward with a random cotangent on 16 frames of 1024 x 1024 (dispersion and aberration on)
    against the oracle's adjoint."""
    from paper_2003_08960_amd.api import Plan
    Tb = 16
    rng = np.random.default_rng(1024)
    frames = synth.random_frames(Tb, N, seed=1024)
    lam = synth.sweep_wavelengths(Tb, 870e-9, 800e-9)
    phi = rng.uniform(-2, 2, Tb)
    zc = rng.normal(0, 0.3, 15)
    G = (rng.standard_normal((Tb, N, N)) + 1j * rng.standard_normal((Tb, N, N))).astype(np.complex64)
    print(f"\n[gpu] vjp T={Tb} N={N}", flush=True)
    plan = Plan(Tb, N, backward=True, precision="fp32_fft")
    g = plan.backward(torch.from_numpy(frames).cuda(), lam, PITCH, Z, torch.from_numpy(G).cuda(), phi, zc)
    g = g.cpu().numpy()
    dz, dc, dphi = O.vjp(frames, lam, PITCH, Z, G.astype(np.complex128), phi, zc)
    rel = lambda a, b: float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))
    print(f"dz {g[1]:.6e} vs {dz:.6e}; dc rel {rel(g[2:17], dc):.2e}; dphi rel {rel(g[17:], dphi):.2e}")
    assert abs(g[1] - dz) <= 1e-4 * abs(dz)
    assert rel(g[2:17], dc) <= 1e-4
    assert rel(g[17:], dphi) <= 1e-4
    plan.close()
