"""Host checks of the benchmark's command line (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_record_is_tied_to_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    traffic, ops, valu, clock = bench.load_counters()
    # the committed record either matches the current sources or is ignored
    with open(bench.TRAFFIC_FILE) as f:
        sha = [l.split(":", 1)[1].strip() for l in f if l.startswith("kernel_sha")][0]
    if sha == bench.kernel_hash():
        assert traffic > 0 and ops > 0 and valu > 0 and clock > 0
        c = bench.contract_ceiling(valu, clock, 0.29)
        # 186 flop-eq per lane-step against 4 cycles per VALU quad-cycle at
        # 32 flops per SIMD cycle, scaled by the clock
        assert abs(c["frac_at_2.4GHz_full_busy"] - 186 * 64 / 32 / (4 * valu)) < 1e-12
        assert c["frac_at_measured_clock"] <= c["frac_at_2.4GHz_full_busy"] <= 1.0
    else:
        assert traffic is None and ops is None and valu is None and clock is None


def test_fp32_counter_record_is_tied_to_the_fp32_sources():
    sys.path.insert(0, ROOT)
    import bench
    kv = bench.read_summary(bench.FP32_COUNTER_FILE, "iod_mixed.hip")
    with open(bench.FP32_COUNTER_FILE) as f:
        sha = [l.split(":", 1)[1].strip() for l in f if l.startswith("kernel_sha")][0]
    if sha == bench.kernel_hash("iod_mixed.hip"):
        # the offset formulation does more arithmetic per step than the absolute one
        assert float(kv["total_32_ops_offset"]) > float(kv["total_32_ops_absolute"]) > 0
    else:
        assert kv is None
    # the FP64 record is keyed by another file's sources
    assert bench.kernel_hash("iod_mixed.hip") != bench.kernel_hash()
