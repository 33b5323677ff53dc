"""Host-side accounting of the benchmark (no GPU): the algorithmic bytes and
operations it prices each kernel and stage at, the roofline and stage
fractions it derives from a profile, the gate on counter-measured traffic,
and the refusal of more than one GPU."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_fft_geometry_and_flops():
    pad, pix, otf = bench.fft_geometry(64, 48, 15, 80)
    assert (pad, pix, otf) == (78 * 62, 64 * 48, 80 * 41 * 8)
    c = 5.0 * 80 * math.log2(80)
    # 39 row pairs of the 78 padded rows, 2 x 41 column transforms, the
    # product, 32 row pairs of the 64 kept rows
    assert bench.fft_conv_flops(80, 78, 64) == pytest.approx(39 * c + 82 * c + 6 * 41 * 80 + 32 * c)


def _two_stamps():
    # one stamp on the one-workgroup form (path 2), one multi-pass (path 1)
    return [(32, 32, 15), (192, 192, 33)], [2, 1], [48, 240]


def test_kernel_table_bytes():
    geo, paths, sides = _two_stamps()
    t, stage, sizes = bench.kernel_table(geo, paths, sides, 7, 1, 5)
    pad0, pix0, otf0 = bench.fft_geometry(32, 32, 15, 48)
    pad1, pix1, otf1 = bench.fft_geometry(192, 192, 33, 240)
    assert sizes == dict(npad=pad0 + pad1, npix=pix0 + pix1, fused_stamps=1, multipass_stamps=1)
    assert t["k_fft2d"] == ("hbm", 7 * (4 * pad0 + 4 * pix0) + otf0)
    assert t["k_fft2d_chi2"] == ("hbm", 4 * pad0 + 8 * pix0 + otf0)
    Mh, Lh = 192 + 32, 240 // 2 + 1
    assert t["k_fft_rows"] == ("hbm", 7 * (4 * pad1 + 8 * Mh * Lh))
    assert t["k_fft_irows_chi2"] == ("hbm", 8 * 192 * Lh + 8 * pix1)
    assert t["k_gram"] == ("hbm", (pix0 + pix1) * (4 * 7 + 8))
    conv = stage["convolution"]
    assert conv["bytes"] == 7 * (4 * (pad0 + pad1) + 4 * (pix0 + pix1)) + otf0 + otf1
    assert conv["flops"] == pytest.approx(7 * (bench.fft_conv_flops(48, 46, 32) + bench.fft_conv_flops(240, 224, 192)))
    c2 = stage["convolution_chi2"]
    assert c2["bytes"] == 4 * (pad0 + pad1) + 8 * (pix0 + pix1) + otf0 + otf1


def test_kernel_table_kept_model():
    """A plain LM fit of one-component stamps: six convolved Jacobian
    channels, and the chi^2 passes also write the convolved model."""
    geo, paths, sides = _two_stamps()
    t0, s0, _ = bench.kernel_table(geo, paths, sides, 7, 1, 5)
    t1, s1, _ = bench.kernel_table(geo, paths, sides, 7, 1, 5, keep_model=True)
    pad0, pix0, otf0 = bench.fft_geometry(32, 32, 15, 48)
    pad1, pix1, otf1 = bench.fft_geometry(192, 192, 33, 240)
    assert t1["k_fft2d"][1] == t0["k_fft2d"][1] - (4 * pad0 + 4 * pix0)
    assert t1["k_fft_rows"][1] * 7 == t0["k_fft_rows"][1] * 6
    assert t1["k_fft2d_chi2"][1] == t0["k_fft2d_chi2"][1] + 4 * pix0
    assert t1["k_fft_irows_chi2"][1] == t0["k_fft_irows_chi2"][1] + 4 * pix1
    assert s1["convolution_chi2"]["bytes"] == s0["convolution_chi2"]["bytes"] + 4 * (pix0 + pix1)
    assert s1["convolution"]["flops"] * 7 == pytest.approx(s0["convolution"]["flops"] * 6)
    assert t1["k_gram"] == t0["k_gram"]   # six channels, the model, data and weight


def test_shared_image_counts_the_image_once():
    geo = [(256, 256, 33)] * 4
    t, stage, _ = bench.kernel_table(geo, [1] * 4, [288] * 4, 1, 1, 5, nimg=256 * 256, shared_otf=True)
    pad, pix, otf = bench.fft_geometry(256, 256, 33, 288)
    assert stage["convolution_chi2"]["bytes"] == 4 * 4 * pad + 8 * 256 * 256 + otf
    assert t["k_chi2"] == ("hbm", 4 * 4 * pix + 8 * 256 * 256)


def test_roofline_and_stage_fractions():
    table = {"k_a": ("alu", 2e12), "k_b": ("hbm", 4e9)}
    prof = {"k_a": (2, 100.0), "k_b": (1, 1.0)}          # (launches, total ms)
    peaks = {"fma_tflops": 75.0, "triad_gbs": 5000.0, "transcendental_gops": 15000.0}
    rl, kern = bench.roofline(prof, table, peaks)
    assert rl["kernel"] == "k_a" and rl["bound"] == "alu"
    # 2e12 operations in 50 ms
    assert rl["achieved"] == pytest.approx(40.0, rel=1e-3)
    assert rl["frac"] == pytest.approx(40.0 / bench.FP32_PEAK_TFLOPS, rel=1e-3)
    assert kern["k_b"]["gbs"] == pytest.approx(4000.0, rel=1e-3)
    assert kern["k_b"]["frac"] == pytest.approx(4000.0 / bench.HBM_PEAK_GBS, rel=1e-3)
    stage = {"convolution": dict(kernels=["k_b"], bytes=2e9, flops=1e10)}
    sf = bench.stage_fractions(prof, stage, peaks)["convolution"]
    assert sf["gbs"] == pytest.approx(2000.0, rel=1e-3)
    # floor: 1e10 operations at one per lane and cycle = half the FMA flop rate
    assert sf["alu_floor_us"] == pytest.approx(1e10 / (75e12 / 2) * 1e6, rel=1e-3)


def test_traffic_gated_by_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    import hashlib
    sha = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC", {("w", "k"): dict(sources={"k.hip": sha}, bytes=1.5e9,
                                                            summary="profiles/x.md")})
    rl = {"kernel": "k"}
    assert bench.measured_traffic("w", rl) == 1.5e9 and rl["traffic_source"] == "profiles/x.md"
    src.write_text("kernel source, changed\n")
    assert bench.measured_traffic("w", {"kernel": "k"}) is None   # counters older than the kernel
    assert bench.measured_traffic("w", {"kernel": "other"}) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
