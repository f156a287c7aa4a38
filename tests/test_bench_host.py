"""Host-side logic of bench.py (no GPU): the counter summary that scales rocprofv3 FETCH_SIZE /
WRITE_SIZE readings to HBM bytes, and the roofline arithmetic of the depth-first order."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write_counters(path, counter, dispatches):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(dispatches):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_summarize_counters_scales_by_the_copy(tmp_path):
    # a 1 GiB copy that counts half its fetched bytes and all its written bytes, and a small copy
    gib_kib = (1 << 30) / 1024
    fetch = [("__amd_rocclr_copyBuffer", gib_kib / 2), ("__amd_rocclr_copyBuffer", 3.0),
             ("void ssoct::k_row_pass_g<1024, false, false, 4>(float2 const*)", 100.0),
             ("void ssoct::k_row_pass_g<1024, false, false, 2>(float2 const*)", 20.0),
             ("void ssoct::k_col_pass<1024, 1, 0, false, 16>(float2 const*)", 50.0),
             ("ssoct::k_cuts(int)", 1.0)]
    write = [("__amd_rocclr_copyBuffer", gib_kib), ("__amd_rocclr_copyBuffer", 3.0),
             ("void ssoct::k_row_pass_g<1024, false, false, 4>(float2 const*)", 200.0),
             ("void ssoct::k_row_pass_g<1024, false, false, 2>(float2 const*)", 40.0),
             ("void ssoct::k_col_pass<1024, 1, 0, false, 16>(float2 const*)", 70.0),
             ("ssoct::k_cuts(int)", 1.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counters(fp, "FETCH_SIZE", fetch)
    _write_counters(wp, "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    table = bench.summarize_counters(f"depth_first:{fp}:{wp}", str(out))
    rec = json.loads(out.read_text())
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    assert rec["source_hash"] == bench.kernel_source_hash()
    k = rec["kernels"]
    assert set(k) == {"k_row_pass_g", "k_col_pass_v"}          # k_cuts has no label
    # the two template variants of the row pass are one label, weighted by dispatches
    assert k["k_row_pass_g"]["dispatches"] == 2
    assert k["k_row_pass_g"]["bytes_per_launch"] == pytest.approx((60.0 * 2 + 120.0) * 1024)
    assert k["k_col_pass_v"]["bytes_per_launch"] == pytest.approx((50.0 * 2 + 70.0) * 1024)
    assert k["k_col_pass_v"]["algorithmic_bytes_per_launch"] == pytest.approx(16 * 256 * 1024 ** 2 / 9)
    assert "k_col_pass_v" in table


@pytest.mark.parametrize("name,kind,label", [
    ("k_col_pass<1024, 1, 0, false, 16>", "frame", "k_col_pass_fp32"),
    ("k_col_pass<1024, 1, 2, false, 16>", "frame", "k_col_pass_bf16"),
    ("k_col_pass<1024, 1, 0, false, 16>", "depth_first", "k_col_pass_v"),
    ("k_col_pass<512, -1, 0, false, 16>", "frame", None),
    ("k_depth<0, 256, 8, 1, 0>", "frame", "k_depth_fp32"),
    ("k_depth<4, 256, 8, 1, 0>", "frame", "k_depth_bf16_split"),
    ("k_depth_4step<16, 4, 0>", "frame", "k_depth_4step_bf16_split_4step"),
    ("k_depth_fft<16, 1, 0, 32>", "frame", "k_depth_fft_fp32_fft"),
    ("k_rescale_dft_win<16>", "depth_first", "k_rescale_dft_win"),
])
def test_traffic_labels(name, kind, label):
    assert bench._traffic_label(name, kind) == label


def test_depth_first_algorithmic_bytes_sum_to_the_path():
    """Per-launch figures times launches give the depth-first order's bytes per render:
    stage 1 (2 + 8 (T/2+1)/T), row pass (8 (T/2+1)/T + 8) and column pass (16) B per voxel."""
    T, N, F = 256, 1024, 32
    nch = -(-(T // 2 + 1) // (F // 2))
    assert nch == 9
    total = (bench._algorithmic_bytes("k_rescale_dft_win", T, N, F)
             + nch * bench._algorithmic_bytes("k_row_pass_g", T, N, F)
             + nch * bench._algorithmic_bytes("k_col_pass_v", T, N, F))
    nb = T // 2 + 1
    assert total == pytest.approx((2 * T + 8 * nb + 8 * nb + 8 * T + 16 * T) * N * N)
    # the whole-path figure counts stage 1's traffic and the volume, not the 2-D round trip
    assert bench.path_bytes_per_voxel(T, True) == pytest.approx(2 + 16 * nb / T + 8)
    assert bench.path_bytes_per_voxel(T, False) == 26
