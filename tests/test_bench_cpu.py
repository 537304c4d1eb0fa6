"""Host-side checks of bench.py's contract (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    # The solver runs on one GPU; asking for several must fail loudly with a
    # JSON message, before anything touches a device.
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "error" in msg and "one GPU" in msg["error"]


def test_traffic_counters_name_their_sources():
    # The HBM traffic figure is tied to the kernel sources it was measured on
    # (bench.py reports it as null once they change); the hash must be over
    # files that exist.
    sys.path.insert(0, ROOT)
    import bench
    for f in bench.KERNEL_SOURCES:
        assert os.path.isfile(os.path.join(ROOT, f)), f
    sha = bench.kernel_sources_sha1()
    assert len(sha) == 40
    if bench.TRAFFIC is not None:
        assert set(bench.TRAFFIC) >= {"f64_bytes_per_launch", "fetch_scale", "source_sha1"}
