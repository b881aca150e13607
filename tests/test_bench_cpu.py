"""The benchmark's contract on the host: one GPU only, the counter summary it
reads for the HBM traffic, and the committed profile summaries."""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_traffic_summary_matches_the_kernel_sources():
    """The committed counter run was taken on the current forward kernel (its
    source hash), so the bench reports its traffic; another size gets none."""
    kv = {}
    with open(bench.PMC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    assert kv["kernel_sources_sha256_16"] == bench.kernel_hash()
    n = int(kv["n"])
    t = bench.traffic_from_profile(n)
    assert t == int(kv["traffic_bytes_per_launch"])
    # the counters read within a few percent of the algorithmic bytes
    assert abs(t / (bench.BYTES_PER_SAMPLE * n) - 1.0) < 0.05
    assert bench.traffic_from_profile(n // 2) is None


def test_profile_summaries_state_their_command():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))
    assert files
    for p in files:
        with open(p) as f:
            text = f.read()
        assert "rocprofv3" in text, p
        assert any(line.startswith("command") for line in text.splitlines()), p
        # summaries only: a few KB of text
        assert len(text) < 16384, p
