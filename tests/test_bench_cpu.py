"""The benchmark script's host-side contract, on any machine (no GPU):
refusing more than one GPU before touching a device, the hash that keys the
stored counter results to the rate-kernel sources, and the lookup of those
results."""
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_source_hash_is_stable_and_covers_the_rate_kernel_sources():
    r1, r2 = _run("--source-sha"), _run("--source-sha")
    assert r1.returncode == 0 and r1.stdout == r2.stdout
    h = r1.stdout.strip()
    assert re.fullmatch(r"[0-9a-f]{64}", h)
    assert h == bench.kernel_source_sha()
    for name in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_2306_16493_amd", "csrc", name))
    assert "rates_wave.h" in bench.KERNEL_SOURCES


def test_traffic_lookup_matches_the_stored_entry_or_is_none():
    with open(os.path.join(ROOT, "profiles", "rates_wave_traffic.json")) as f:
        entries = json.load(f)["entries"]
    sha = bench.kernel_source_sha()
    assert bench.measured_traffic("no_such_workload", "fp32") is None
    for t in entries:
        got = bench.measured_traffic(t["workload"], t["precision"])
        if t["source_sha256"] != sha:
            continue  # counters taken on other sources are not reported
        want = t["fetch_kib_per_launch"] * 1024 * t["fetch_scale"] + t["write_kib_per_launch"] * 1024 * t["write_scale"]
        assert got == want
