"""Host logic of bench.py: the roofline arithmetic, the kernel-source hash that
guards stored counter results, and the single-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench


def test_roof_hbm_only():
    r = bench.roof(8e9, 2.0)  # 8 GB in 2 ms = 4 TB/s
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)
    assert "ceilings" not in r


def test_roof_ceilings_hbm_binding():
    # 1e9 elements at 9 bytes and 22 ops each in 2 ms
    r = bench.roof(9e9, 2.0, 1e9, 22)
    c = r["ceilings"]
    assert c["bytes_per_element"] == pytest.approx(9.0)
    assert c["hbm_elements_per_s"] == pytest.approx(8e12 / 9, rel=1e-9)
    assert c["valu_elements_per_s"] == pytest.approx(256 * 64 * 2.4e9 / 22, rel=1e-9)
    assert c["binding"] == "hbm" and c["arithmetic"] == "f64"
    assert c["frac_of_binding"] == pytest.approx(5e11 / (8e12 / 9), abs=1e-4)


def test_roof_ceilings_valu_binding():
    # 3 bytes and 22 FP64 ops per element: 2.67 T elt/s of HBM against 1.79 T of VALU
    r = bench.roof(3e9, 1.0, 1e9, 22)
    c = r["ceilings"]
    assert c["binding"] == "valu"
    assert c["frac_of_binding"] == pytest.approx(1e12 / (256 * 64 * 2.4e9 / 22), abs=1e-4)
    # the line names the binding ceiling: ALU, in lane-ops/s, HBM figures kept aside
    r0 = bench.roof(3e9, 1.0, 1e9, 22)
    assert r0["bound"] == "alu" and r0["unit"] == "T lane-ops/s"
    assert r0["achieved"] == pytest.approx(22.0) and r0["peak"] == pytest.approx(39.3216, abs=1e-3)
    assert r0["frac"] == pytest.approx(c["frac_of_binding"])
    assert r0["hbm"]["bound"] == "hbm" and r0["hbm"]["achieved"] == pytest.approx(3000.0)
    # in FP32 the VALU ceiling doubles (3.57 T elt/s) and HBM binds
    c = bench.roof(3e9, 1.0, 1e9, 22, fp32=True)["ceilings"]
    assert c["arithmetic"] == "f32" and c["binding"] == "hbm"
    assert c["valu_elements_per_s"] == pytest.approx(2 * 256 * 64 * 2.4e9 / 22, rel=1e-9)


def test_source_hash_tracks_kernel_sources():
    h = bench.source_hash("fwd_kernel_f64_f64_p2")
    assert len(h) == 16 and h == bench.source_hash("fwd_kernel_f64_f64_p2")
    for name in bench.KERNEL_SOURCES["fwd_kernel_f64_f64_p2"]:
        assert os.path.exists(os.path.join(ROOT, "paper_1702_05156_amd", "csrc", name))


def test_stored_traffic_only_for_current_sources():
    # counter results are reported only while the kernel's sources are those
    # they were taken on; otherwise the traffic is null
    path = os.path.join(ROOT, "profiles", "traffic_fwd_kernel_f64_f64_p2.json")
    with open(path) as fh:
        d = json.load(fh)
    assert 0.99 < d["traffic_bytes_per_launch"] / d["alg_bytes_per_launch"] < 1.2
    got = bench.load_traffic("fwd_kernel_f64_f64_p2")
    if d["source_hash"] == bench.source_hash("fwd_kernel_f64_f64_p2"):
        assert got == d["traffic_bytes_per_launch"]
    else:
        assert got is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "single" in (r.stdout + r.stderr)
