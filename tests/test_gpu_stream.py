"""GPU tests of the streaming renderer (HIP graph per slot) and of the launch-shape tuner.

Every volume that comes out of a stream is a replay of a captured graph; each
is compared with the eager ssoct_render of the same sweep (same kernels and
launch shapes: bitwise equal) and with the FP64 oracle, with eager work and
synchronisations between the replays."""
import numpy as np
import pytest
import torch

from oracle import ssoct_oracle as O
from paper_2003_08960_amd import native, synth

pytestmark = pytest.mark.gpu

T, N = 32, 128


@pytest.fixture(scope="module")
def sweeps():
    cfg = synth.SweepConfig(T=T, N=N, pitch=20e-6, z=0.3, lam_max=870e-9, lam_min=800e-9, n_scatterers=5,
                            name="stream")
    return [synth.make_sweep(cfg, seed=100 + i) for i in range(5)]


def eager(plan, sw):
    fr = torch.from_numpy(sw.frames).cuda()
    V = plan.render(fr, sw.lam, sw.pitch, sw.z).clone()
    cuts = [c.cpu().numpy() for c in plan.cuts(V, N // 2, N // 2, T // 4)]
    torch.cuda.synchronize()
    return V, cuts


def test_host_fed_stream_matches_eager_render(gpu_lib, sweeps):
    from paper_2003_08960_amd.api import Plan, Stream
    print("\n[gpu] stream host-fed", flush=True)
    plan = Plan(T, N)
    sw0 = sweeps[0]
    refs = [eager(plan, sw) for sw in sweeps[:4]]
    st = Stream(plan, sw0.lam, sw0.pitch, sw0.z, slots=3)
    rng = np.random.default_rng(0)
    allframes = np.concatenate([sw.frames for sw in sweeps[:4]])
    pinned = torch.from_numpy(allframes).pin_memory()
    seq = 0
    popped = []
    while seq < allframes.shape[0]:                      # pushes of random sizes, pops in between
        n = int(rng.integers(1, 20))
        n = min(n, allframes.shape[0] - seq)
        assert st.push_frames(pinned[seq:seq + n], seq) == native.OK
        seq += n
        if st.stats()["in_flight"] >= 2:
            popped.append(st.pop(wait=True))
            torch.cuda.synchronize()
            _ = (torch.ones(1000, device="cuda") * 2).sum().item()   # eager work between replays
    while True:
        r = st.pop(wait=True)
        if r is None:
            break
        popped.append(r)
    assert [r["seq"] for r in popped] == [0, 1, 2, 3]
    for r in popped:
        V, cuts = refs[r["seq"]]
        for got, want in zip((r["cut_xy"], r["cut_xz"], r["cut_yz"]), cuts):
            assert np.array_equal(got, want)
        assert r["latency_ms"] > 0
    st.close()


def test_stream_volume_matches_oracle(gpu_lib, sweeps):
    from paper_2003_08960_amd.api import Plan, Stream
    plan = Plan(T, N)
    sw = sweeps[1]
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=2)
    assert st.push_frames(np.ascontiguousarray(sw.frames), 5 * T) == native.OK
    r = st.pop(wait=True)
    assert r["seq"] == 5
    V = st.slot_volume(r["slot"]).cpu().numpy()
    ref = O.render(sw.frames, sw.lam, sw.pitch, sw.z)
    assert np.linalg.norm(V - ref) / np.linalg.norm(ref) <= 1e-5
    st.close()


def test_sequence_gap_discards_the_partial_sweep(gpu_lib, sweeps):
    from paper_2003_08960_amd.api import Plan, Stream
    plan = Plan(T, N)
    sw = sweeps[0]
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=3)
    f = [np.ascontiguousarray(s.frames) for s in sweeps[:3]]
    assert st.push_frames(f[0], 0) == native.OK                       # sweep 0 complete
    assert st.push_frames(f[1][:10], T) == native.OK                  # sweep 1 partial
    assert st.push_frames(f[1][12:], T + 12) == native.EDROPPED      # gap: sweep 1 dropped, rest skipped
    assert st.push_frames(f[2], 2 * T) == native.OK                   # sweep 2 complete
    s = st.stats()
    assert s["dropped_sweeps"] == 1 and s["dropped_frames"] == 10 + (T - 12)
    seqs = [st.pop(wait=True)["seq"] for _ in range(2)]
    assert seqs == [0, 2]
    assert st.pop(wait=True) is None
    st.close()


def test_full_ring_drops_sweeps_instead_of_mixing(gpu_lib, sweeps):
    from paper_2003_08960_amd.api import Plan, Stream
    plan = Plan(T, N)
    sw = sweeps[0]
    refs = [eager(plan, s) for s in sweeps[:4]]
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=2)
    codes = [st.push_frames(np.ascontiguousarray(s.frames), i * T) for i, s in enumerate(sweeps[:4])]
    assert codes[:2] == [native.OK, native.OK]
    assert native.EDROPPED in codes[2:]
    out = [st.pop(wait=True) for _ in range(2)]
    assert [r["seq"] for r in out] == [0, 1]
    for r in out:
        assert np.array_equal(r["cut_xy"], refs[r["seq"]][1][0])
    assert st.stats()["dropped_sweeps"] >= 1
    st.close()


def test_device_resident_slots(gpu_lib, sweeps):
    from paper_2003_08960_amd.api import Plan, Stream
    plan = Plan(T, N, precision="bf16_split")
    sw = sweeps[0]
    refs = [eager(plan, s) for s in sweeps[:3]]
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=2)
    order = [0, 1, 2, 1, 0, 2]                       # each slot graph is replayed more than once
    pending = 0
    for n, i in enumerate(order):
        got = st.acquire()
        if got is None:                              # both slots in flight: take the oldest out
            r = st.pop(wait=True)
            pending -= 1
            k = r["seq"] % 10
            assert torch.equal(st.slot_volume(r["slot"]), refs[k][0])
            assert np.array_equal(r["cut_xz"], refs[k][1][1])
            got = st.acquire()
        slot, buf = got
        buf.copy_(torch.from_numpy(sweeps[i].frames).cuda())
        torch.cuda.synchronize()
        st.submit(slot, 10 * n + i)
        pending += 1
    assert st.acquire() is None
    while pending:
        r = st.pop(wait=True)
        pending -= 1
        k = r["seq"] % 10
        assert torch.equal(st.slot_volume(r["slot"]), refs[k][0])
        assert np.array_equal(r["cut_yz"], refs[k][1][2])
    assert st.stats()["done"] == len(order)
    st.close()


def test_tuning_changes_speed_not_results(gpu_lib, sweeps, tmp_path):
    from paper_2003_08960_amd.api import Plan
    sw = sweeps[2]
    plan = Plan(T, N)
    fr = torch.from_numpy(sw.frames).cuda()
    V0 = plan.render(fr, sw.lam, sw.pitch, sw.z).clone()
    cache = str(tmp_path / "tuning.json")
    choice = plan.tune(fr, sw.lam, sw.pitch, sw.z, cache_path=cache)
    assert 0 <= choice[0] <= T and len(choice) == native.TUNING_LEN      # 0: the order's default chunk
    V1 = plan.render(fr, sw.lam, sw.pitch, sw.z).clone()
    assert torch.equal(V0, V1)
    for tuning in ([1, 0, 0], [3, 7, 5], [T, 1024, 64]):
        plan.set_tuning(tuning)
        assert torch.equal(plan.render(fr, sw.lam, sw.pitch, sw.z), V0)
    plan2 = Plan(T, N)
    assert plan2.tune(fr, sw.lam, sw.pitch, sw.z, cache_path=cache) == choice   # from the cache
    plan.set_tuning([0, 0, 0])                                  # 0: the order's default chunk
    assert torch.equal(plan.render(fr, sw.lam, sw.pitch, sw.z), V0)
    with pytest.raises(native.SsoctError):
        plan.set_tuning([-1, 0, 0])
    with pytest.raises(native.SsoctError):
        plan.set_tuning([T + 1, 0, 0])
    with pytest.raises(native.SsoctError):
        plan.set_tuning([1, 0, 0, 2])
    for bad in ([1, 0, 0, 0, 3], [1, 0, 0, 0, 0, 5], [1, 0, 0, 0, 0, 0, 48], [1, 0, 0, 0, 0, 0, 0, 1]):
        with pytest.raises(native.SsoctError):
            plan.set_tuning(bad)


def test_tune_cache_in_the_library(gpu_lib, sweeps):
    """ssoct_plan_tune keeps its choice per (device, T, N, flags, order allowed, aberration): a second
    plan of the same kind takes it without timing (its volume buffer is left untouched); after
    ssoct_tune_cache_clear it times again.  Called through the C ABI with a NaN-filled volume."""
    import ctypes
    from paper_2003_08960_amd import api
    from paper_2003_08960_amd.api import Plan
    sw = sweeps[1]
    lib = native.load()
    fr = torch.from_numpy(sw.frames).cuda()
    api.tune_cache_clear()

    def tune(plan, vol):
        t = (ctypes.c_int * native.TUNING_LEN)()
        plan._sync_stream()
        native.check(lib.ssoct_plan_tune(
            plan._h, ctypes.c_void_p(fr.data_ptr()), native.host_doubles(sw.lam, T), sw.pitch, sw.z, None, None,
            ctypes.c_void_p(plan.workspace.data_ptr()), plan.workspace.numel(), ctypes.c_void_p(vol.data_ptr()), t))
        torch.cuda.synchronize()
        return [int(x) for x in t]

    nan = torch.view_as_complex(torch.full((T, N, N, 2), float("nan"), device="cuda"))   # NaN + NaN i
    p1 = Plan(T, N, precision="fp32_fft")
    vol = nan.clone()
    choice = tune(p1, vol)
    assert not torch.isnan(torch.view_as_real(vol)).any()          # timed: rendered into vol
    p2 = Plan(T, N, precision="fp32_fft")
    vol = nan.clone()
    assert tune(p2, vol) == choice and p2.get_tuning() == choice
    assert torch.isnan(torch.view_as_real(vol)).all()              # from the cache: nothing rendered
    p3 = Plan(T, N, precision="bf16_split")                          # another form: its own entry
    vol = nan.clone()
    tune(p3, vol)
    assert not torch.isnan(torch.view_as_real(vol)).any()
    api.tune_cache_clear()
    vol = nan.clone()
    assert len(tune(p2, vol)) == native.TUNING_LEN
    assert not torch.isnan(torch.view_as_real(vol)).any()          # timed again
    for p in (p1, p2, p3):
        p.close()


def test_chunkwise_fresnel_with_ragged_chunks_and_discarded_sweep(gpu_lib, sweeps):
    """Frames per chunk 5 (T = 32: six full chunks and a ragged one): the chunk
    graphs of a sweep that is then discarded must not disturb the next sweep
    rendered in the same slot."""
    from paper_2003_08960_amd.api import Plan, Stream
    print("\n[gpu] stream chunk-wise, F=5", flush=True)
    plan = Plan(T, N)
    plan.set_tuning([5, 0, 0])
    refs = [eager(plan, s) for s in sweeps[:3]]
    sw = sweeps[0]
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=1)
    f = [np.ascontiguousarray(s.frames) for s in sweeps[:3]]
    assert st.push_frames(f[0][:23], 0) == native.OK           # chunks 0-3 start, the sweep is cut short
    assert st.push_frames(f[0][24:], 24) == native.EDROPPED
    assert st.push_frames(f[1][:7], T) == native.OK
    assert st.push_frames(f[1][7:19], T + 7) == native.OK
    assert st.push_frames(f[1][19:], T + 19) == native.OK
    r = st.pop(wait=True)
    assert r["seq"] == 1
    assert torch.equal(st.slot_volume(r["slot"]), refs[1][0])
    assert np.array_equal(r["cut_xy"], refs[1][1][0])
    for j in range(0, T, 3):                                    # sweep 2 three frames at a time
        assert st.push_frames(f[2][j:j + 3], 2 * T + j) == native.OK
    r = st.pop(wait=True)
    assert r["seq"] == 2
    assert torch.equal(st.slot_volume(r["slot"]), refs[2][0])
    s = st.stats()
    assert s["dropped_sweeps"] == 1 and s["done"] == 2
    st.close()


def test_stream_with_fft_depth_form(gpu_lib, sweeps):
    """The FFT form in the depth-first order streams through one whole-volume graph per slot."""
    from paper_2003_08960_amd.api import Plan, Stream
    plan = Plan(T, N, precision="fp32_fft")
    plan.set_tuning(plan.get_tuning()[:3] + [1])
    refs = [eager(plan, s) for s in sweeps[:3]]
    sw = sweeps[0]
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=2)
    allframes = np.concatenate([s.frames for s in sweeps[:3]])
    for j in range(0, allframes.shape[0], 9):
        assert st.push_frames(np.ascontiguousarray(allframes[j:j + 9]), j) == native.OK
        if st.stats()["in_flight"] >= 1:       # keep a slot free for the next sweep
            r = st.pop(wait=True)
            assert torch.equal(st.slot_volume(r["slot"]), refs[r["seq"]][0])
    while True:
        r = st.pop(wait=True)
        if r is None:
            break
        assert torch.equal(st.slot_volume(r["slot"]), refs[r["seq"]][0])
        assert np.array_equal(r["cut_xz"], refs[r["seq"]][1][1])
    assert st.stats()["done"] == 3
    st.close()


@pytest.mark.parametrize("precision", ["bf16_split_4step", "fp32_4step"])
def test_stream_with_factored_depth_form(gpu_lib, sweeps, precision):
    """The factored MFMA form inside the per-slot graphs: every volume bitwise equal to an eager render."""
    from paper_2003_08960_amd.api import Plan, Stream
    plan = Plan(T, N, precision=precision)
    refs = [eager(plan, s) for s in sweeps[:3]]
    sw = sweeps[0]
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=3)
    allframes = np.concatenate([s.frames for s in sweeps[:3]])
    for j in range(0, allframes.shape[0], 7):
        assert st.push_frames(np.ascontiguousarray(allframes[j:j + 7]), j) == native.OK
    got = 0
    while True:
        r = st.pop(wait=True)
        if r is None:
            break
        assert torch.equal(st.slot_volume(r["slot"]), refs[r["seq"]][0])
        got += 1
    assert got == 3 and st.stats()["dropped_sweeps"] == 0
    st.close()


def test_binding_guards(gpu_lib, sweeps):
    """Buffers of the wrong shape, dtype or device are refused before any launch, and a plan cannot
    be released while a stream uses it."""
    from paper_2003_08960_amd.api import Plan, Stream
    plan = Plan(T, N)
    sw = sweeps[0]
    fr = torch.from_numpy(sw.frames).cuda()
    with pytest.raises(ValueError):
        plan.render(fr, sw.lam, sw.pitch, sw.z, out=torch.empty((T, N, N - 1), dtype=torch.complex64, device="cuda"))
    with pytest.raises(TypeError):
        plan.render(fr, sw.lam, sw.pitch, sw.z, out=torch.empty((T, N, N), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        plan.render(fr, sw.lam, sw.pitch, sw.z, out=torch.empty((T, N, N), dtype=torch.complex64))
    with pytest.raises(ValueError):
        plan.cuts(torch.empty((T, N, N), dtype=torch.complex64, device="cuda")[:, :, ::1].transpose(1, 2), 0, 0, 0)
    st = Stream(plan, sw.lam, sw.pitch, sw.z, slots=1)
    with pytest.raises(native.SsoctError):
        plan.close()
    st.close()
    plan.close()
