"""Host-side logic of bench.py (no GPU): the roofline record, the use of the
stored counter summary, and the refusal of multi-GPU runs."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (module level imports only the standard library)


def test_roofline_takes_the_class_with_the_largest_time():
    prof = {
        "stencil32": (11.6, 336, 336 * 84.3e6),
        "vector32": (7.7, 336, 336 * 125.8e6),
        "stencil64": (10.3, 160, 160 * 176.2e6),
        "scalars": (50.0, 10, 0.0),          # never the dominant class
        "basis_sum": (0.0, 0, 0.0),          # no launches
    }
    name, roof = bench.roofline_from_profile(prof)
    assert name == "stencil32"
    ms, n, nb = prof["stencil32"]
    assert abs(roof["achieved"] - nb / (ms * 1e-3) / 1e9) < 0.1
    assert abs(roof["frac"] - roof["achieved"] / bench.HBM_PEAK_GBS) < 1e-4
    assert roof["peak"] == 8000.0 and roof["unit"] == "GB/s" and roof["bound"] == "hbm"
    assert roof["launches"] == n and abs(roof["avg_launch_ms"] - ms / n) < 1e-5
    assert roof["traffic"] is None


def test_stored_traffic_only_for_the_measured_kernel():
    for kclass in ("iter32", "stencil32"):
        path = bench.counters_path(kclass)
        if not os.path.exists(path):
            assert bench.measured_traffic(kclass, 0) is None
            continue
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2204_01583_amd", "csrc", rec["kernel_source"]),
                   "rb").read()
        same_source = hashlib.sha256(src).hexdigest()[:16] == rec["kernel_source_sha256_16"]
        got = bench.measured_traffic(kclass, rec["variant"])
        if same_source:
            assert got == rec["traffic_bytes_per_launch"]
        else:
            assert got is None
        assert bench.measured_traffic(kclass, rec["variant"] + 1) is None   # another variant
    assert bench.measured_traffic("no_such_class", 0) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
