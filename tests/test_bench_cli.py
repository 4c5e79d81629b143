"""CPU checks of the benchmark's command line: it runs on one GPU and says so
for more, and its traffic figure is tied to the kernel sources it was
measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a run that did not happen


def test_traffic_is_reported_only_for_the_kernel_sources_it_was_measured_on():
    sys.path.insert(0, ROOT)
    import bench
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    h = bench.kernel_source_hash()
    for key, rec in t.items():
        assert rec["fetch_bytes"] >= rec["algorithmic_bytes"] * 0.9, key
        got = bench.counted_traffic(key)
        if rec["kernel_sources"] == h:
            assert got == rec["fetch_bytes"] + rec["write_bytes"], key
        else:  # counters taken on other kernel sources: no traffic figure
            assert got is None, key
    assert bench.counted_traffic("no-such-workload") is None
