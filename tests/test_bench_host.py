"""Host-side pieces of bench.py (no GPU): the MFMA depth table, the per-visit
byte prices, the roofline arithmetic, the traffic lookup with its source-hash
check, and the one-GPU refusal."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_gram_depth_covers_d_plus_two():
    for d in range(1, 129):
        kp = bench.gram_kp(d)
        assert kp % 16 == 0 and kp >= d + 2
    assert [bench.gram_kp(d) for d in (2, 14, 15, 30, 62, 78, 126, 127)] == [16, 16, 32, 32, 64, 80, 128, 144]


def test_point_depth_covers_d():
    # interval tiles: K = d padded (the norm terms are added outside the MFMA)
    for d in range(1, 129):
        kp = bench.point_kp(d)
        assert kp % 16 == 0 and kp >= d
    assert [bench.point_kp(d) for d in (10, 16, 17, 64, 65, 128)] == [16, 16, 32, 64, 80, 128]
    st = {"kernels": {"block_search": {"visits": 1_000_000}}, "point_pair_evals": 0}
    r = bench.roofline("block_search", "average", 128, 1.0, 1, [st])
    assert r["bound"] == "mfma" and r["achieved"] == pytest.approx(1e6 * 2 * 128 / 1e-3 / 1e12)


def test_visit_prices():
    # FP64 centroid + size + cluster ID; avg-2 adds its FP64 spread term,
    # complete / average the FP32 box (8d + 4 + 4 + 8d = 40 B at d = 2)
    assert bench.visit_bytes("ward", 2) == 24
    assert bench.visit_bytes("avgsq", 2) == 32
    assert bench.visit_bytes("complete", 2) == 40
    assert bench.visit_bytes("average", 5) == 40 + 8 + 40


def test_roofline_arithmetic():
    st = {"kernels": {"ring_search": {"visits": 1_000_000}}, "point_pair_evals": 0}
    # 2 launches taking 1 ms in total: 1e6 visits x 40 B / 2 launches = 20 MB
    # per launch in 0.5 ms = 40 GB/s
    r = bench.roofline("ring_search", "complete", 2, 1.0, 2, [st])
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(40.0)
    assert r["frac"] == pytest.approx(40.0 / bench.PEAK_HBM_GBS)
    assert r["work_per_launch"] == pytest.approx(20e6)
    if r["traffic"] is not None:
        # measured bytes per launch over the same launch time
        assert r["measured_frac"] == pytest.approx(r["traffic"] / 0.5e-3 / 1e9 / bench.PEAK_HBM_GBS)
    # a Gram-search kernel at d = 10 is priced as FP16 MFMA work: 2K flops per pair
    r = bench.roofline("ring_search", "ward", 10, 1.0, 1, [st])
    assert r["bound"] == "mfma" and r["achieved"] == pytest.approx(1e6 * 2 * 16 / 1e-3 / 1e12)
    # Ward / avg-2 at 3 <= d <= 5: the slot's visits add box-tree gathers and
    # Gram pass-0 MFMA pairs, so the entry stays unpriced instead of mixing units
    r = bench.roofline("ring_search", "avgsq", 5, 1.0, 1, [st])
    assert r["bound"] is None and r["frac"] is None and r["work_per_launch"] is None
    assert r["avg_launch_ms"] == pytest.approx(1.0)
    # the same slot at d = 2 (grid rounds only) is priced as gathers
    r = bench.roofline("ring_search", "avgsq", 2, 1.0, 1, [st])
    assert r["bound"] == "hbm" and r["work_per_launch"] == pytest.approx(1e6 * bench.visit_bytes("avgsq", 2))


def test_traffic_lookup_follows_the_kernel_source():
    path = os.path.join(ROOT, "profiles", "blob50_1m_d2_complete_ring_search_traffic.md")
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    src = os.path.join(ROOT, "paper_2106_04727_amd", "csrc", "pc_round.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    got = bench.measured_traffic("ring_search", "complete", 2)
    if vals["kernel_source_sha256"] == sha:
        assert got == float(vals["hbm_bytes_per_launch"])
    else:
        assert got is None  # counters taken on other kernel code are not reported
    assert bench.measured_traffic("ring_search", "complete", 10) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
