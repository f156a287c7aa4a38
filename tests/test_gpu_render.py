"""GPU parity of ssoct_render / ssoct_cuts against the FP64 oracle.

Bars: relative L2 error over all voxels <= 1e-5 for the FP32 path and
<= 1e-4 for the split FP16/BF16 depth transform; plain FP16/BF16 errors are
reported (they are expected above 1e-4) with a sanity bound.
"""
import numpy as np
import pytest
import torch

from oracle import ssoct_oracle as O
from paper_2003_08960_amd import native, synth

pytestmark = pytest.mark.gpu

FP32_BAR = 1e-5
SPLIT_BAR = 1e-4
PLAIN_SANITY = 2e-2


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def gpu_render(frames, lam, pitch, z, precision="fp32", disp=None, zern=None, **kw):
    from paper_2003_08960_amd.api import Plan
    T, N, _ = frames.shape
    print(f"\n[gpu] render T={T} N={N} precision={precision} disp={disp is not None} "
          f"zern={zern is not None} {kw}", flush=True)
    plan = Plan(T, N, precision=precision, **kw)
    fr = torch.from_numpy(np.ascontiguousarray(frames)).cuda()
    V = plan.render(fr, lam, pitch, z, disp, zern)
    torch.cuda.synchronize()
    return plan, fr, V


def random_case(T, N, seed, lo=0, hi=65535):
    frames = synth.random_frames(T, N, seed, lo, hi)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    return frames, lam


@pytest.fixture(scope="module")
def tiny():
    return synth.make_config("tiny")


@pytest.fixture(scope="module")
def mid():
    return synth.make_config("mid")


# ---------------------------------------------------------------- small sizes, every FFT length class

@pytest.mark.parametrize("T,N", [(4, 16), (5, 32), (7, 64), (33, 128), (3, 256), (2, 512), (2, 1024), (1, 2048)])
def test_fp32_small_sizes(gpu_lib, T, N):
    frames, lam = random_case(T, N, seed=100 + N + T)
    _, _, V = gpu_render(frames, lam, 20e-6, 0.05)
    ref = O.render(frames, lam, 20e-6, 0.05)
    err = rel_l2(V.cpu().numpy(), ref)
    print(f"rel-L2 {err:.3e}")
    assert err <= FP32_BAR


@pytest.mark.parametrize("T", [1, 2, 31, 33, 64, 100, 127, 129, 256, 300])
def test_fp32_ragged_sweeps(gpu_lib, T):
    """Sweep lengths that are not multiples of the depth-transform tiles (zero-padded K, odd T)."""
    N = 32
    frames, lam = random_case(T, N, seed=7 * T)
    _, _, V = gpu_render(frames, lam, 20e-6, 0.05)
    ref = O.render(frames, lam, 20e-6, 0.05)
    err = rel_l2(V.cpu().numpy(), ref)
    print(f"T={T} rel-L2 {err:.3e}")
    assert err <= FP32_BAR


@pytest.mark.parametrize("precision,bar", [("fp32", FP32_BAR), ("bf16_split", SPLIT_BAR), ("fp16_split", SPLIT_BAR)])
@pytest.mark.parametrize("T", [1000, 1024])
def test_longest_sweeps(gpu_lib, T, precision, bar):
    """The largest sweep the plan takes (T = 1024) and a ragged one below it, on the dense depth product."""
    N = 16
    frames, lam = random_case(T, N, seed=T)
    _, _, V = gpu_render(frames, lam, 20e-6, 0.05, precision=precision)
    ref = O.render(frames, lam, 20e-6, 0.05)
    err = rel_l2(V.cpu().numpy(), ref)
    print(f"T={T} {precision} rel-L2 {err:.3e}")
    assert err <= bar


# ---------------------------------------------------------------- tiny workload (T=32, N=128)

def test_tiny_fp32_and_cuts(gpu_lib, tiny):
    plan, fr, V = gpu_render(tiny.frames, tiny.lam, tiny.pitch, tiny.z)
    ref = O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z)
    err = rel_l2(V.cpu().numpy(), ref)
    err_nodc = rel_l2(V.cpu().numpy()[1:], ref[1:])
    print(f"rel-L2 {err:.3e}  (bins q>0: {err_nodc:.3e})")
    assert err <= FP32_BAR
    # cuts at a scatterer and at the default position
    for (x0, y0, q0) in ((int(tiny.scatterers[0, 1]), int(tiny.scatterers[0, 0]), int(tiny.scatterers[0, 2])),
                         (64, 64, 8)):
        xy, xz, yz = plan.cuts(V, x0, y0, q0)
        rxy, rxz, ryz = O.cuts(ref, x0, y0, q0)
        for a, b in ((xy, rxy), (xz, rxz), (yz, ryz)):
            assert rel_l2(a.cpu().numpy(), b) <= FP32_BAR
        # the cuts are exactly |V| of the GPU volume
        M = V.abs()
        assert torch.equal(xy, M[q0]) or rel_l2(xy.cpu().numpy(), M[q0].cpu().numpy()) < 1e-7


def test_tiny_options(gpu_lib, tiny):
    rng = np.random.default_rng(3)
    T = tiny.frames.shape[0]
    disp = rng.uniform(-3, 3, T)
    zern = rng.normal(0, 0.5, 15)
    cases = [dict(exact_chirp=True), dict(disp=disp), dict(zern=zern), dict(disp=disp, zern=zern, exact_chirp=True),
             dict(eq6_phase=True)]
    for kw in cases:
        k = dict(kw)
        d = k.pop("disp", None)
        z_ = k.pop("zern", None)
        _, _, V = gpu_render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, disp=d, zern=z_, **k)
        ref = O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, d, z_,
                       exact_chirp=k.get("exact_chirp", False), eq6_phase=k.get("eq6_phase", False))
        err = rel_l2(V.cpu().numpy(), ref)
        print(f"{sorted(kw)} rel-L2 {err:.3e}")
        assert err <= FP32_BAR


def test_tiny_focus_ground_truth(gpu_lib, tiny):
    _, _, V = gpu_render(tiny.frames, tiny.lam, tiny.pitch, tiny.z)
    M = V.abs().cpu().numpy()
    for u, v, q, _ in tiny.scatterers:
        u, v, q = int(u), int(v), int(q)
        win = M[q, u - 2:u + 3, v - 2:v + 3]
        assert np.unravel_index(np.argmax(win), win.shape) == (2, 2)


def test_write_abs_and_power_cuts(gpu_lib, tiny):
    from paper_2003_08960_amd.api import Plan
    T, N, _ = tiny.frames.shape
    fr = torch.from_numpy(tiny.frames).cuda()
    plan = Plan(T, N, write_abs=True)
    A = plan.render(fr, tiny.lam, tiny.pitch, tiny.z)
    ref = O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z)
    assert A.dtype == torch.float32
    assert rel_l2(A.cpu().numpy(), np.abs(ref)) <= FP32_BAR
    plan2 = Plan(T, N, cut_power=True)
    V = plan2.render(fr, tiny.lam, tiny.pitch, tiny.z)
    xy, xz, yz = plan2.cuts(V, 10, 20, 5)
    rxy, rxz, ryz = O.cuts(ref, 10, 20, 5, power=True)
    assert rel_l2(xy.cpu().numpy(), rxy) <= 3 * FP32_BAR
    assert rel_l2(yz.cpu().numpy(), ryz) <= 3 * FP32_BAR


def test_deterministic_and_table_cache(gpu_lib, tiny):
    from paper_2003_08960_amd.api import Plan
    T, N, _ = tiny.frames.shape
    fr = torch.from_numpy(tiny.frames).cuda()
    plan = Plan(T, N)
    V1 = plan.render(fr, tiny.lam, tiny.pitch, tiny.z).clone()
    V2 = plan.render(fr, tiny.lam, tiny.pitch, tiny.z).clone()
    assert torch.equal(V1, V2)
    V3 = plan.render(fr, tiny.lam, tiny.pitch, 0.2)          # new z: tables rebuilt
    ref = O.render(tiny.frames, tiny.lam, tiny.pitch, 0.2)
    assert rel_l2(V3.cpu().numpy(), ref) <= FP32_BAR
    V4 = plan.render(fr, tiny.lam, tiny.pitch, tiny.z)
    assert torch.equal(V1, V4)


def test_zero_aberration_skips_the_screen(gpu_lib, tiny):
    """All-zero Zernike coefficients give A = 1: bit-identical to no aberration, before and after a non-zero set."""
    from paper_2003_08960_amd.api import Plan
    T, N, _ = tiny.frames.shape
    fr = torch.from_numpy(tiny.frames).cuda()
    plan = Plan(T, N)
    V0 = plan.render(fr, tiny.lam, tiny.pitch, tiny.z).clone()
    assert torch.equal(plan.render(fr, tiny.lam, tiny.pitch, tiny.z, None, np.zeros(15)), V0)
    zc = np.random.default_rng(3).normal(0, 0.4, 15)
    V1 = plan.render(fr, tiny.lam, tiny.pitch, tiny.z, None, zc).clone()
    assert rel_l2(V1.cpu().numpy(), O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, None, zc)) <= FP32_BAR
    assert torch.equal(plan.render(fr, tiny.lam, tiny.pitch, tiny.z, None, -0.0 * zc), V0)


def test_bad_arguments_raise(gpu_lib, tiny):
    from paper_2003_08960_amd import native
    from paper_2003_08960_amd.api import Plan
    T, N, _ = tiny.frames.shape
    fr = torch.from_numpy(tiny.frames).cuda()
    plan = Plan(T, N)
    with pytest.raises(native.SsoctError):
        plan.render(fr, tiny.lam, tiny.pitch, 0.0)
    bad = np.array(tiny.lam)
    bad[3] = -1
    with pytest.raises(native.SsoctError):
        plan.render(fr, bad, tiny.pitch, tiny.z)
    with pytest.raises(native.SsoctError):
        V = plan.render(fr, tiny.lam, tiny.pitch, tiny.z)
        plan.cuts(V, N, 0, 0)
    # undersampled distance: computed, with a warning status
    plan.render(fr, tiny.lam, tiny.pitch, 0.01)
    assert plan.last_status == native.WARN_UNDERSAMPLED


# ---------------------------------------------------------------- mid workload (T=128, N=512)

@pytest.mark.parametrize("precision,bar", [("fp32", FP32_BAR), ("fp32_fft", FP32_BAR), ("fp16_split", SPLIT_BAR),
                                           ("bf16_split", SPLIT_BAR), ("fp16", PLAIN_SANITY), ("bf16", PLAIN_SANITY),
                                           ("fp32_4step", FP32_BAR), ("fp16_split_4step", SPLIT_BAR),
                                           ("bf16_split_4step", SPLIT_BAR), ("fp16_4step", PLAIN_SANITY),
                                           ("bf16_4step", PLAIN_SANITY)])
def test_mid_precisions(gpu_lib, mid, precision, bar):
    _, _, V = gpu_render(mid.frames, mid.lam, mid.pitch, mid.z, precision=precision)
    ref = _mid_ref(mid)
    Vn = V.cpu().numpy()
    err = rel_l2(Vn, ref)
    err_nodc = rel_l2(Vn[1:], ref[1:])
    print(f"{precision}: rel-L2 {err:.3e} (bins q>0: {err_nodc:.3e})")
    assert err <= bar


_MID_REF = {}


def _mid_ref(mid):
    if "v" not in _MID_REF:
        _MID_REF["v"] = O.render(mid.frames, mid.lam, mid.pitch, mid.z)
    return _MID_REF["v"]


def test_profile_record_splits_the_fresnel_stage(gpu_lib):
    from paper_2003_08960_amd.api import Plan
    print("\n[gpu] profile record", flush=True)
    sw = synth.make_config("tiny")
    T, N = sw.frames.shape[:2]
    fr = torch.from_numpy(sw.frames).cuda()
    for F in (T, 5):
        plan = Plan(T, N, profile="kernels")
        plan.set_tuning([F, 0, 0])
        for _ in range(3):
            plan.render(fr, sw.lam, sw.pitch, sw.z)
        st = plan.profile_read()
        assert st[3] == 3
        assert st[4] > 0 and st[5] > 0 and st[2] > 0
        assert st[4] + st[5] <= st[1] * 1.05 + 1e-3
        with pytest.raises(native.SsoctError):
            plan.profile_read()                      # the record was reset
    plan = Plan(T, N, profile=True)                  # stage events only
    plan.render(fr, sw.lam, sw.pitch, sw.z)
    st = plan.profile_read()
    assert st[1] > 0 and st[4] == -1 and st[5] == -1


# ---------------------------------------------------------------- radix-FFT depth transform

@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("T,N", [(16, 64), (32, 32), (64, 16), (128, 32), (256, 16), (256, 64)])
def test_fft_depth_every_supported_length(gpu_lib, T, N, order):
    """Every T the FFT form takes, in both evaluation orders."""
    from paper_2003_08960_amd.api import Plan
    frames, lam = random_case(T, N, seed=3 * T + N)
    print(f"\n[gpu] fft depth T={T} N={N} order={order}", flush=True)
    plan = Plan(T, N, precision="fp32_fft")
    plan.set_tuning(plan.get_tuning()[:3] + [order])
    V = plan.render(torch.from_numpy(frames).cuda(), lam, 20e-6, 0.05)
    ref = O.render(frames, lam, 20e-6, 0.05)
    err = rel_l2(V.cpu().numpy(), ref)
    print(f"T={T} N={N} order={order} rel-L2 {err:.3e}")
    assert err <= FP32_BAR


def test_fft_depth_matches_dense_form_and_options(gpu_lib, tiny):
    """Dispersion and aberration, |V| output and cuts through the FFT form."""
    from paper_2003_08960_amd.api import Plan
    T = tiny.frames.shape[0]
    rng = np.random.default_rng(11)
    disp = rng.normal(0, 1.0, T)
    zern = rng.normal(0, 0.3, 15)
    _, _, V = gpu_render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, precision="fp32_fft", disp=disp, zern=zern)
    ref = O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, disp, zern)
    assert rel_l2(V.cpu().numpy(), ref) <= FP32_BAR
    N = tiny.frames.shape[1]
    plan = Plan(T, N, precision="fp32_fft", write_abs=True)
    fr = torch.from_numpy(tiny.frames).cuda()
    M = plan.render(fr, tiny.lam, tiny.pitch, tiny.z, disp, zern).cpu().numpy()
    assert rel_l2(M, np.abs(ref)) <= FP32_BAR


def test_fft_depth_rejections(gpu_lib):
    from paper_2003_08960_amd.api import Plan
    for T in (100, 512, 8):
        with pytest.raises(native.SsoctError) as e:
            Plan(T, 32, precision="fp32_fft")
        assert e.value.code == native.EUNSUPPORTED


# ---------------------------------------------------------------- depth-first order of the FFT form
# With the default chirp (lambda_1 for every frame) and no dispersion phase, the FFT form takes the
# depth DFT of the rescaled frames first and one 2-D transform per bin pair (q, T - q).

@pytest.mark.parametrize("aberr,eq6", [(False, False), (True, False), (False, True), (True, True)])
def test_depth_first_options(gpu_lib, tiny, aberr, eq6):
    from paper_2003_08960_amd.api import Plan
    zern = np.random.default_rng(5).normal(0, 0.3, 15) if aberr else None
    T, N = tiny.frames.shape[:2]
    plan = Plan(T, N, precision="fp32_fft", eq6_phase=eq6)
    plan.set_tuning(plan.get_tuning()[:3] + [1])
    V = plan.render(torch.from_numpy(tiny.frames).cuda(), tiny.lam, tiny.pitch, tiny.z, None, zern)
    ref = O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, None, zern, eq6_phase=eq6)
    err = rel_l2(V.cpu().numpy(), ref)
    print(f"aberr={aberr} eq6={eq6} rel-L2 {err:.3e}")
    assert err <= FP32_BAR


def test_depth_first_zero_dispersion_and_chunking(gpu_lib, tiny):
    """An all-zero dispersion array keeps the depth-first order; the number of bins per
    chunk (frames-per-chunk tuning) changes no bit of the volume."""
    from paper_2003_08960_amd.api import Plan
    T, N = tiny.frames.shape[:2]
    fr = torch.from_numpy(tiny.frames).cuda()
    plan = Plan(T, N, precision="fp32_fft")
    assert plan.get_tuning()[3] == 1                                        # the default order
    V0 = plan.render(fr, tiny.lam, tiny.pitch, tiny.z).clone()              # depth-first order
    plan.set_tuning(plan.get_tuning()[:3] + [0])
    Vf = plan.render(fr, tiny.lam, tiny.pitch, tiny.z).clone()              # frame order
    plan.set_tuning(plan.get_tuning()[:3] + [1])
    ref = O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z)
    assert rel_l2(V0.cpu().numpy(), ref) <= FP32_BAR
    assert rel_l2(Vf.cpu().numpy(), ref) <= FP32_BAR
    assert not torch.equal(V0, Vf)                                          # two rounding orders
    V1 = plan.render(fr, tiny.lam, tiny.pitch, tiny.z, np.zeros(T)).clone()
    assert torch.equal(V0, V1)
    for F in (1, 2, 3, 7, T):
        plan.set_tuning([F, 0, 0, 1])
        assert torch.equal(plan.render(fr, tiny.lam, tiny.pitch, tiny.z), V0), F
    Vd = plan.render(fr, tiny.lam, tiny.pitch, tiny.z, np.full(T, 0.5)).cpu().numpy()   # falls back to frame order
    assert rel_l2(Vd, O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, np.full(T, 0.5))) <= FP32_BAR


@pytest.mark.parametrize("T,N", [(256, 256), (128, 1024), (16, 2048)])
def test_depth_first_large_frames(gpu_lib, T, N):
    from paper_2003_08960_amd.api import Plan
    frames, lam = random_case(T, N, seed=T + N)
    print(f"\n[gpu] depth-first T={T} N={N}", flush=True)
    plan = Plan(T, N, precision="fp32_fft")
    plan.set_tuning(plan.get_tuning()[:3] + [1])
    V = plan.render(torch.from_numpy(frames).cuda(), lam, 12e-6, 0.3)
    pix = [(0, 0), (N // 2, N // 2), (N - 1, 3), (17, N - 5)]
    ref = O.render_columns(frames, lam, 12e-6, 0.3, pix)
    got = np.stack([V[:, u, v].cpu().numpy() for u, v in pix], axis=1)
    err = rel_l2(got, ref)
    print(f"T={T} N={N} sampled rel-L2 {err:.3e}")
    assert err <= FP32_BAR


def test_column_walk_is_independent_of_the_workgroup_count(gpu_lib):
    """At N = 1024 the column pass holds its twiddles in LDS and prefetches
    the next tile: any persistent grid, from one workgroup walking every tile
    to more workgroups than tiles, and ragged frame chunks give bit-identical
    volumes and gradients."""
    from paper_2003_08960_amd.api import Plan
    T, N = 16, 1024
    frames, lam = random_case(T, N, seed=91)
    fr = torch.from_numpy(frames).cuda()
    zern = np.random.default_rng(92).normal(0, 0.3, 15)
    print(f"\n[gpu] column grids T={T} N={N}", flush=True)
    plan = Plan(T, N, precision="fp32_fft", backward=True)
    V0 = plan.render(fr, lam, 12e-6, 0.3).clone()
    g0 = plan.backward_sharpness(fr, lam, 12e-6, 0.3, None, zern).clone()
    for F, cg in ((16, 1), (5, 37), (16, 4096), (7, 0)):
        plan.set_tuning([F, cg, 0])
        assert torch.equal(plan.render(fr, lam, 12e-6, 0.3), V0), (F, cg)
        assert torch.equal(plan.backward_sharpness(fr, lam, 12e-6, 0.3, None, zern), g0), (F, cg)


# Eq. 6 phase and aberration on large frames in both evaluation orders: the
# row passes keep the Eq. 6 factor in LDS up to N = 1024 and read it from
# memory at N = 2048; the column passes hold their twiddles in LDS and
# prefetch the next tile up to N = 1024, and keep both in registers at 2048.
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("N", [512, 1024, 2048])
def test_options_on_large_frames(gpu_lib, N, order):
    from paper_2003_08960_amd.api import Plan
    T = 16
    frames, lam = random_case(T, N, seed=7 * N + order)
    zern = np.random.default_rng(N).normal(0, 0.4, 15)
    print(f"\n[gpu] Eq. 6 phase + aberration T={T} N={N} order={order}", flush=True)
    plan = Plan(T, N, precision="fp32_fft", eq6_phase=True)
    plan.set_tuning(plan.get_tuning()[:3] + [order])
    V = plan.render(torch.from_numpy(frames).cuda(), lam, 12e-6, 0.3, None, zern)
    pix = [(0, 0), (N // 2, N // 2), (N - 1, 3), (17, N - 5), (N // 3, 2 * N // 3)]
    ref = O.render_columns(frames, lam, 12e-6, 0.3, pix, zernike_coeffs=zern, eq6_phase=True)
    got = np.stack([V[:, u, v].cpu().numpy() for u, v in pix], axis=1)
    err = rel_l2(got, ref)
    print(f"N={N} order={order} sampled rel-L2 {err:.3e}")
    assert err <= FP32_BAR


# ---------------------------------------------------------------- factored (16 x T/16) MFMA depth transform

FOURSTEP = [("fp32_4step", FP32_BAR), ("fp16_split_4step", SPLIT_BAR), ("bf16_split_4step", SPLIT_BAR),
            ("fp16_4step", PLAIN_SANITY), ("bf16_4step", PLAIN_SANITY)]


@pytest.mark.parametrize("precision,bar", FOURSTEP)
@pytest.mark.parametrize("T,N", [(32, 64), (64, 32), (128, 16), (256, 32)])
def test_4step_every_supported_length(gpu_lib, T, N, precision, bar):
    """Every T the factored form takes (T2 = T/16 = 2, 4, 8, 16), several 16-pixel tiles per workgroup."""
    from paper_2003_08960_amd.api import Plan
    frames, lam = random_case(T, N, seed=7 * T + N)
    print(f"\n[gpu] 4-step depth T={T} N={N} {precision}", flush=True)
    plan = Plan(T, N, precision=precision)
    V = plan.render(torch.from_numpy(frames).cuda(), lam, 20e-6, 0.05)
    ref = O.render(frames, lam, 20e-6, 0.05)
    err = rel_l2(V.cpu().numpy(), ref)
    print(f"T={T} N={N} {precision} rel-L2 {err:.3e}")
    assert err <= bar


def test_4step_options_abs_and_agreement_with_fft(gpu_lib, tiny):
    """Dispersion, aberration, Eq. 6 phase and the |V| output through the factored form; equal to the FFT form."""
    from paper_2003_08960_amd.api import Plan
    T, N, _ = tiny.frames.shape
    rng = np.random.default_rng(12)
    disp = rng.normal(0, 1.0, T)
    zern = rng.normal(0, 0.3, 15)
    ref = O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, disp, zern)
    fr = torch.from_numpy(tiny.frames).cuda()
    for prec, bar in (("fp32_4step", FP32_BAR), ("bf16_split_4step", SPLIT_BAR)):
        V = Plan(T, N, precision=prec).render(fr, tiny.lam, tiny.pitch, tiny.z, disp, zern)
        assert rel_l2(V.cpu().numpy(), ref) <= bar
        M = Plan(T, N, precision=prec, write_abs=True).render(fr, tiny.lam, tiny.pitch, tiny.z, disp, zern)
        assert rel_l2(M.cpu().numpy(), np.abs(ref)) <= bar
    ref6 = O.render(tiny.frames, tiny.lam, tiny.pitch, tiny.z, disp, zern, eq6_phase=True)
    V6 = Plan(T, N, precision="fp16_split_4step", eq6_phase=True).render(fr, tiny.lam, tiny.pitch, tiny.z, disp, zern)
    assert rel_l2(V6.cpu().numpy(), ref6) <= SPLIT_BAR
    Vf = Plan(T, N, precision="fp32_fft").render(fr, tiny.lam, tiny.pitch, tiny.z, disp, zern)
    V4 = Plan(T, N, precision="fp32_4step").render(fr, tiny.lam, tiny.pitch, tiny.z, disp, zern)
    assert rel_l2(V4.cpu().numpy(), Vf.cpu().numpy()) <= 2e-6


def test_4step_rejections(gpu_lib):
    from paper_2003_08960_amd.api import Plan
    for T in (16, 48, 512):
        with pytest.raises(native.SsoctError):
            Plan(T, 32, precision="fp32_4step")
    with pytest.raises(native.SsoctError):
        Plan(64, 32, precision="fp32_4step", nonuniform_k=True)


# ---------------------------------------------------------------- the five-argument render (default plans)

def test_five_argument_render(gpu_lib, tiny):
    """ssoct_render(frames, T, N, lambda, pitch, z, vol, stream): the problem statement of Eq. 5-7 as
    one call with a cached FP32 default plan (the FFT depth form where T allows, else the dense FP32
    product).  Matches the oracle, equals the explicit-plan render of that form bit for bit, reuses
    its plan across calls, and keeps separate plans per size."""
    from paper_2003_08960_amd import api
    from paper_2003_08960_amd.api import Plan
    sw = tiny
    T, N = sw.frames.shape[0], sw.frames.shape[1]
    print(f"\n[gpu] five-argument render T={T} N={N}", flush=True)
    fr = torch.from_numpy(sw.frames).cuda()
    V = api.render(fr, sw.lam, sw.pitch, sw.z)
    V2 = api.render(fr, sw.lam, sw.pitch, sw.z)          # cached plan, same tables
    torch.cuda.synchronize()
    ref = O.render(sw.frames, sw.lam, sw.pitch, sw.z)
    assert rel_l2(V.cpu().numpy(), ref) <= FP32_BAR
    assert torch.equal(V, V2)
    assert torch.equal(V, Plan(T, N, precision="fp32_fft").render(fr, sw.lam, sw.pitch, sw.z))
    # a T the FFT form does not take: the dense FP32 product
    frames, lam = random_case(20, 64, seed=77)
    f2 = torch.from_numpy(frames).cuda()
    W = api.render(f2, lam, 20e-6, 0.05)
    assert rel_l2(W.cpu().numpy(), O.render(frames, lam, 20e-6, 0.05)) <= FP32_BAR
    assert torch.equal(W, Plan(20, 64, precision="fp32").render(f2, lam, 20e-6, 0.05))
    # parameters change between calls: the cached plan rebuilds its tables
    V3 = api.render(fr, sw.lam, sw.pitch, 0.25)
    assert rel_l2(V3.cpu().numpy(), O.render(sw.frames, sw.lam, sw.pitch, 0.25)) <= FP32_BAR
    api.render_release()
    assert torch.equal(api.render(fr, sw.lam, sw.pitch, sw.z), V)   # a fresh default plan after the release
    api.render_release()


# ---------------------------------------------------------------- tuning alternatives (tiles, row groups)

@pytest.mark.parametrize("N,T", [(32, 16), (64, 16), (128, 16), (512, 16), (1024, 16), (2048, 2)])
def test_radix_orders_agree(gpu_lib, N, T):
    """Tuning entry 8: the column transforms with the small radix first (L 16 .. 16) and in the
    default order (16 .. 16 L) each meet the oracle bar, in the frame order with complex64 and
    BF16-split H and in the FFT form's depth-first order; the two orders differ by rounding only."""
    from paper_2003_08960_amd.api import Plan
    frames, lam = random_case(T, N, seed=500 + N)
    fr = torch.from_numpy(frames).cuda()
    ref = O.render(frames, lam, 20e-6, 0.05)
    cases = [("fp32", 0), ("bf16_split", 0)] + ([("fp32_fft", 0), ("fp32_fft", 1)] if T >= 16 else [])
    for precision, order in cases:
        print(f"\n[gpu] radix orders N={N} T={T} {precision} order {order}", flush=True)
        bar = SPLIT_BAR if "split" in precision else FP32_BAR
        plan = Plan(T, N, precision=precision)
        vols = []
        for radix in (0, 1):
            t = plan.get_tuning()
            t[3], t[8] = order, radix
            plan.set_tuning(t)
            assert plan.get_tuning()[8] == radix
            V = plan.render(fr, lam, 20e-6, 0.05).cpu().numpy()
            err = rel_l2(V, ref)
            print(f"radix order {radix}: rel-L2 {err:.3e}")
            assert err <= bar, (precision, order, radix)
            vols.append(V)
        assert rel_l2(vols[1], vols[0]) <= (SPLIT_BAR if "split" in precision else 2e-6)
        plan.close()


def test_radix_order_rejected_where_there_is_one(gpu_lib):
    """N = 16 and 256 are powers of 16 (one radix order), and the angular-spectrum column pass has
    one order: tuning entry 8 = 1 is an error there, and any value other than 0 or 1 everywhere."""
    from paper_2003_08960_amd.api import Plan
    for N, kw in ((16, {}), (256, {}), (1024, {"angular_spectrum": True})):
        plan = Plan(4, N, **kw)
        with pytest.raises(native.SsoctError):
            plan.set_tuning([0, 0, 0, 0, 0, 0, 0, 0, 1])
        plan.close()
    plan = Plan(4, 512)
    for bad in (2, -1):
        with pytest.raises(native.SsoctError):
            plan.set_tuning([0, 0, 0, 0, 0, 0, 0, 0, bad])
    plan.set_tuning([0, 0, 0, 0, 0, 0, 0, 0, 1])
    assert plan.get_tuning()[8] == 1
    plan.close()


@pytest.mark.parametrize("T", [64, 256])
def test_dense_k_chunk_changes_speed_not_results(gpu_lib, T):
    """Tuning entry 7: the dense depth product with half its default K chunk (32 of 64, 128 of 256
    frames) runs the same products in the same order, so the volume is bit-identical; other chunks
    are rejected."""
    from paper_2003_08960_amd.api import Plan
    N = 128
    frames, lam = random_case(T, N, seed=406 + T)
    fr = torch.from_numpy(frames).cuda()
    ref = O.render(frames, lam, 20e-6, 0.05)
    print(f"\n[gpu] dense K chunk T={T} N={N}", flush=True)
    for precision, bar in (("fp32", FP32_BAR), ("bf16_split", SPLIT_BAR), ("fp16_split", SPLIT_BAR)):
        plan = Plan(T, N, precision=precision)
        V0 = plan.render(fr, lam, 20e-6, 0.05).clone()
        assert rel_l2(V0.cpu().numpy(), ref) <= bar
        kc = T // 2
        plan.set_tuning([0, 0, 0, 0, 0, 0, 0, kc])
        assert torch.equal(plan.render(fr, lam, 20e-6, 0.05), V0), (precision, kc)
        for bad in (kc // 2, T, 48):
            with pytest.raises(native.SsoctError):
                plan.set_tuning([0, 0, 0, 0, 0, 0, 0, bad])
        plan.close()


def test_tiles_and_row_groups_change_speed_not_results(gpu_lib):
    """The tuner's tile choices at N = 1024: column tile widths 16 / 8 / 4, rows per row group of the
    depth-first order 2 / 4 / 8 and FFT depth workgroups of 16 / 32 / 64 pixels give bit-identical
    volumes in both evaluation orders (and in the split H format); the tuner's pick too; and the
    factored MFMA form gives the same volume with 16- or 32-pixel tiles."""
    from paper_2003_08960_amd.api import Plan
    T, N = 16, 1024
    frames, lam = random_case(T, N, seed=404)
    fr = torch.from_numpy(frames).cuda()
    print(f"\n[gpu] tiles and row groups T={T} N={N}", flush=True)
    ref = O.render(frames, lam, 12e-6, 0.3)
    for precision in ("fp32_fft", "bf16_split"):
        for order in ((0, 1) if precision == "fp32_fft" else (0,)):
            plan = Plan(T, N, precision=precision)
            plan.set_tuning(plan.get_tuning()[:3] + [order])
            V0 = plan.render(fr, lam, 12e-6, 0.3).clone()
            assert rel_l2(V0.cpu().numpy(), ref) <= (FP32_BAR if precision == "fp32_fft" else SPLIT_BAR)
            for rpg in (0, 2, 4, 8):
                for tile in (0, 8, 4):
                    for px in (0, 16, 64):
                        plan.set_tuning([T, 0, 0, order, rpg, tile, px])
                        assert torch.equal(plan.render(fr, lam, 12e-6, 0.3), V0), (precision, order, rpg, tile, px)
            choice = plan.tune(fr, lam, 12e-6, 0.3)
            print(precision, order, "tuned", choice)
            assert len(choice) == native.TUNING_LEN
            if choice[3] == order:
                assert torch.equal(plan.render(fr, lam, 12e-6, 0.3), V0)
            else:
                assert rel_l2(plan.render(fr, lam, 12e-6, 0.3).cpu().numpy(), ref) <= FP32_BAR
            plan.close()
    # the factored MFMA form's pixel tile: 16 or 32 pixels per workgroup, the same products per pixel
    T4 = 32
    frames4, lam4 = random_case(T4, N, seed=405)
    fr4 = torch.from_numpy(frames4).cuda()
    ref4 = O.render(frames4, lam4, 12e-6, 0.3)
    for precision in ("fp32_4step", "bf16_split_4step"):
        plan = Plan(T4, N, precision=precision)
        V0 = plan.render(fr4, lam4, 12e-6, 0.3).clone()
        assert rel_l2(V0.cpu().numpy(), ref4) <= (FP32_BAR if precision.startswith("fp32") else SPLIT_BAR)
        for px in (16, 32):
            plan.set_tuning([0, 0, 0, 0, 0, 0, px])
            assert torch.equal(plan.render(fr4, lam4, 12e-6, 0.3), V0), (precision, px)
        with pytest.raises(native.SsoctError):
            plan.set_tuning([0, 0, 0, 0, 0, 0, 64])
        plan.close()
