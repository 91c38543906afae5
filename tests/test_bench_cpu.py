"""bench.py's host-side contract, on the CPU: it refuses more than one GPU
with a message, prints the walk sources' hash, and the committed counter
summary that its traffic figure comes from was taken on the current walk
sources (else the figure would be reported as null)."""
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_sources_sha_matches_the_module():
    r = _run("--sources-sha")
    assert r.returncode == 0
    sha = r.stdout.strip()
    assert re.fullmatch(r"[0-9a-f]{64}", sha)
    assert sha == bench.walk_sources_sha256()


def test_committed_counters_name_their_sources():
    # the n=40 counter summary names the sources it was measured on; bench
    # reports its traffic figure only while the walk's sources still hash to
    # that value (after a change to the walk, null until re-profiled)
    fields = {}
    with open(bench.TRAFFIC_SUMMARY) as f:
        for line in f:
            key, sep, val = line.strip().strip("-* `").partition(":")
            if sep:
                fields[key.strip("` ")] = val.strip(" `")
    assert re.fullmatch(r"[0-9a-f]{64}", fields["kernel_sources_sha256"])
    assert float(fields["traffic_bytes_per_launch"]) > 0
    traffic = bench.committed_traffic()
    if fields["kernel_sources_sha256"] == bench.walk_sources_sha256():
        assert traffic == float(fields["traffic_bytes_per_launch"])
    else:
        assert traffic is None


def test_algorithmic_work_per_state():
    # 52 packed instructions per 64 states for the float16 screen, 66 for the
    # int16 screen; 1.5 per state (one DPP add, half a three-input minimum)
    # for the float32 screen
    assert bench.HALF_OPS_PER_STATE == 52 / 64
    assert bench.INT16_OPS_PER_STATE == 66 / 64
    assert bench.ALG_OPS_PER_STATE == 1.5
