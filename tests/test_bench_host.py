"""Host-side checks of the benchmark: it refuses more than one GPU before touching
one, and the committed counter record it reads for roofline traffic is complete."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_is_complete():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    assert rec, "no kernel in the traffic record"
    for kernel, e in rec.items():
        assert kernel.startswith("k_") and "<" in kernel
        assert len(e["source_hash"]) == 16
        assert e["bytes_per_launch"] > 0 and e["fetch_kib"] > 0 and e["write_kib"] > 0
        # bytes = 1024 (FETCH x scale + WRITE x scale)
        want = 1024 * (e["fetch_kib"] * e["fetch_scale"] + e["write_kib"] * e["write_scale"])
        assert abs(e["bytes_per_launch"] - want) <= 1e-6 * want
        assert os.path.exists(os.path.join(ROOT, "profiles", e["summary"]))
