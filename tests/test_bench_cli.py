"""Host logic of bench.py (no GPU needed): the one-GPU rule, the kernel
source hash that ties a counter profile to the sources it was taken on, and
the traffic ratio read from the committed profile."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_kernel_source_hash_is_stable_hex():
    a, b = bench.kernel_source_hash(), bench.kernel_source_hash()
    assert a == b and re.fullmatch(r"[0-9a-f]{64}", a)


def test_traffic_ratio_only_for_matching_sources():
    path = os.path.join(ROOT, "profiles", f"row_matvec_{bench.WORKLOAD}_counters.txt")
    text = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    assert m, "the counter summary records the hash of its kernel sources"
    ratio = bench.traffic_ratio_from_profile("row_matvec")
    if m.group(1) == bench.kernel_source_hash():
        # counters taken on these sources: a measured ratio of HBM-side to
        # algorithmic bytes (1 = no re-reads)
        assert ratio is not None and 0.9 < ratio < 2.0
    else:
        assert ratio is None


def test_cpu_worker_reports_one_run():
    # one process of the all-core CPU baseline: the oracle on one of the nine
    # runs, started without the GPU, reporting its own start and end
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-worker", "4", "--cpu-steps", "1"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stderr
    import json
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["run"] == 4 and out["steps"] == 1 and out["points"] == 1024 * 512
    assert out["t1"] > out["t0"]
