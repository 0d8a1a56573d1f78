"""Host-side contract of bench.py: one GPU only, and the measured-traffic
record it reads from the committed profile."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_profile_traffic_is_read_only_for_the_current_sources():
    sys.path.insert(0, ROOT)
    import bench
    path = os.path.join(ROOT, "profiles", "k_brick_fp32c_c3_4M_traffic.md")
    vals = dict(line.split(":", 1) for line in open(path)
                if ":" in line and not line.startswith(("#", "|", "`")))
    vals = {k.strip(): v.strip() for k, v in vals.items()}
    stored = float(vals["traffic_bytes_per_launch"])
    # a byte count per launch a little above the algorithmic 20 + 2 n_mean
    # bytes per atom-substep (n_mean = 20.41 on the 4M-atom system)
    assert 1.0 < stored / (4_000_000 * 60.8) < 1.3
    fresh = vals["csrc_sha256"] == bench.library_source_hash()
    assert bench.measured_traffic("k_brick_fp32c", 4_000_000) == (stored if fresh else None)
    assert bench.measured_traffic("k_brick_fp32c", 1_000_000) is None
    assert bench.measured_traffic("k_no_such_kernel", 4_000_000) is None
