"""GPU tests of the sliding-window depth transform (ssoct_slide_*).

Every window that comes out is compared with the FP64 oracle's render of
the same T consecutive frames in time order, each frame rescaled with the
wavelength of its sweep position (frame seq is recorded at lambda[seq % T]).
"""
import numpy as np
import pytest
import torch

from oracle import ssoct_oracle as O
from paper_2003_08960_amd import native, synth

pytestmark = pytest.mark.gpu

T, N = 32, 64
PITCH, Z = 20e-6, 0.05


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


@pytest.fixture(scope="module")
def stream_frames():
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    frames = synth.random_frames(3 * T + 9, N, seed=77)
    return frames, lam


def oracle_window(frames, lam, j, disp=None, zern=None):
    idx = [(j + i) % T for i in range(T)]
    d = None if disp is None else np.asarray(disp)[idx]
    return O.render(frames[j:j + T], np.asarray(lam)[idx], PITCH, Z, d, zern)


def run_host_fed(plan, frames, lam, hop, disp=None, zern=None, chunk=None):
    """Push frames in chunks of at most `hop`, popping every finished window; returns {start: (V, cuts)}."""
    from paper_2003_08960_amd.api import Slide
    sl = Slide(plan, lam, PITCH, Z, disp, zern, hop=hop, slots=2)
    out = {}
    chunk = chunk or hop
    rng = np.random.default_rng(3)
    seq = 0
    while seq < frames.shape[0]:
        n = int(rng.integers(1, chunk + 1))
        n = min(n, frames.shape[0] - seq)
        assert sl.push(np.ascontiguousarray(frames[seq:seq + n]), seq) == native.OK
        seq += n
        while True:
            r = sl.pop(wait=True)
            if r is None:
                break
            out[r["start"]] = (sl.volume(r["slot"]).clone(), (r["cut_xy"], r["cut_xz"], r["cut_yz"]))
            torch.cuda.synchronize()      # the copy is done before a later window may reuse the slot
            torch.cuda.synchronize()      # the copy is done before a later window may reuse the slot
    assert sl.stats()["dropped_windows"] == 0
    sl.close()
    return out


@pytest.mark.parametrize("precision,bar,radix", [("fp32", 1e-5, 0), ("fp32_fft", 1e-5, 0), ("bf16_split", 1e-4, 0),
                                                 ("fp32_4step", 1e-5, 0), ("bf16_split_4step", 1e-4, 0),
                                                 ("fp32_fft", 1e-5, 1), ("bf16_split_4step", 1e-4, 1)])
def test_every_window_matches_the_oracle(gpu_lib, stream_frames, precision, bar, radix):
    """radix 1: the column transforms in the second radix order (set before the windows are set up)."""
    from paper_2003_08960_amd.api import Plan
    frames, lam = stream_frames
    hop = 5
    print(f"\n[gpu] slide {precision} hop={hop} radix order {radix}", flush=True)
    plan = Plan(T, N, precision=precision)
    t = plan.get_tuning()
    t[8] = radix
    plan.set_tuning(t)
    out = run_host_fed(plan, frames, lam, hop)
    starts = sorted(out)
    assert starts == list(range(0, frames.shape[0] - T + 1, hop))
    for j in starts:
        V, cuts = out[j]
        ref = oracle_window(frames, lam, j)
        err = rel_l2(V.cpu().numpy(), ref)
        assert err <= bar, (j, err)
        ref_xy = np.abs(ref[T // 4])
        assert rel_l2(cuts[0], ref_xy) <= bar


def test_dispersion_and_aberration_follow_the_sweep_position(gpu_lib, stream_frames):
    from paper_2003_08960_amd.api import Plan
    frames, lam = stream_frames
    rng = np.random.default_rng(9)
    disp = rng.normal(0, 1.0, T)
    zern = rng.normal(0, 0.3, 15)
    plan = Plan(T, N)
    out = run_host_fed(plan, frames, lam, hop=7, disp=disp, zern=zern)
    for j in (7, 21, sorted(out)[-1]):
        assert rel_l2(out[j][0].cpu().numpy(), oracle_window(frames, lam, j, disp, zern)) <= 1e-5


def test_device_resident_ring_equals_host_fed(gpu_lib, stream_frames):
    """A periodic stream (frame seq = sweep frame seq % T) through the device ring and through pushes."""
    from paper_2003_08960_amd.api import Plan, Slide
    frames, lam = stream_frames
    sweep = frames[:T]
    periodic = np.concatenate([sweep, sweep, sweep[:11]])
    plan = Plan(T, N, precision="fp32_fft")
    hop = 6
    ref = run_host_fed(plan, periodic, lam, hop)
    sl = Slide(plan, lam, PITCH, Z, hop=hop, slots=2)
    sl.ring().copy_(torch.from_numpy(sweep).cuda())
    torch.cuda.synchronize()
    got = {}
    seq = 0
    while seq < periodic.shape[0]:
        n = min(hop, periodic.shape[0] - seq)
        assert sl.advance(n, seq) == native.OK
        seq += n
        while True:
            r = sl.pop(wait=True)
            if r is None:
                break
            got[r["start"]] = sl.volume(r["slot"]).clone()
            torch.cuda.synchronize()      # the copy is done before a later window may reuse the slot
    sl.close()
    assert sorted(got) == sorted(ref)
    for j in got:
        assert torch.equal(got[j], ref[j][0])
    # a static scene: every window has the same envelope
    a = torch.abs(got[0])
    for j in got:
        assert torch.allclose(torch.abs(got[j]), a, rtol=1e-4, atol=1e-2 * float(a.max()))


def test_sequence_gap_restarts_the_windows(gpu_lib, stream_frames):
    from paper_2003_08960_amd.api import Plan, Slide
    frames, lam = stream_frames
    plan = Plan(T, N)
    sl = Slide(plan, lam, PITCH, Z, hop=5, slots=4)
    assert sl.push(np.ascontiguousarray(frames[:41]), 0) == native.OK
    starts = []
    while (r := sl.pop(wait=True)) is not None:
        starts.append(r["start"])
    assert starts == [0, 5]
    assert sl.push(np.ascontiguousarray(frames[45:45 + T + 4]), 45) == native.EDROPPED
    got = {}
    while (r := sl.pop(wait=True)) is not None:
        got[r["start"]] = sl.volume(r["slot"]).clone()
        torch.cuda.synchronize()      # the copy is done before a later window may reuse the slot
    assert sorted(got) == [45]
    assert rel_l2(got[45].cpu().numpy(), oracle_window(frames, lam, 45)) <= 1e-5
    assert sl.stats()["restarts"] == 1
    with pytest.raises(native.SsoctError):
        sl.push(np.ascontiguousarray(frames[:2]), 3)          # out of order
    sl.close()


def test_full_output_ring_drops_windows(gpu_lib, stream_frames):
    from paper_2003_08960_amd.api import Plan, Slide
    frames, lam = stream_frames
    plan = Plan(T, N)
    sl = Slide(plan, lam, PITCH, Z, hop=4, slots=1)
    assert sl.push(np.ascontiguousarray(frames[:2 * T]), 0) == native.OK
    s = sl.stats()
    assert s["in_flight"] == 1 and s["dropped_windows"] == (2 * T - T) // 4
    r = sl.pop(wait=True)
    assert r["start"] == 0
    assert rel_l2(sl.volume(r["slot"]).cpu().numpy(), oracle_window(frames, lam, 0)) <= 1e-5
    assert sl.pop(wait=True) is None
    sl.close()
