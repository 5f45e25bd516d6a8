"""bench.py's host-side contract (CPU only): one GPU only, and the traffic
figure is withheld once the kernel's sources differ from the measured ones."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_keyed_by_sources():
    sys.path.insert(0, ROOT)
    import bench
    k = "k_count_mfma_lds<fp4>"
    digest = bench.sources_digest(k)
    saved = dict(bench.TRAFFIC)
    try:
        bench.TRAFFIC[k] = {"sources": digest, "bytes": 123}
        assert bench.traffic_bytes(k) == 123
        # counted on the 2D N = 131072 workload only
        assert bench.traffic_bytes(k, 16384, 4) is None
        assert bench.traffic_bytes(k, 1024, 2) is None
        bench.TRAFFIC[k] = {"sources": "0" * 16, "bytes": 123}
        assert bench.traffic_bytes(k) is None
        bench.TRAFFIC.pop(k)
        assert bench.traffic_bytes(k) is None
    finally:
        bench.TRAFFIC.clear()
        bench.TRAFFIC.update(saved)


def test_mfma_roofline_arithmetic():
    sys.path.insert(0, ROOT)
    import bench
    r = bench.mfma_roofline(131072, 0.1, True)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert abs(r["achieved"] - 2 * 375291379056640 / 0.1 / 1e12) < 1e-6 * r["achieved"]
    assert abs(r["frac"] - r["achieved"] / 10100.0) < 1e-12
