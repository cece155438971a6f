"""Host-side checks of the benchmark: it refuses more than one GPU before touching
one, and the committed counter record it reads for roofline traffic is complete."""
import json
import os
import re
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
        # the names bench.roofline() looks up: direction, spin, precision
        assert re.fullmatch(r"k_(m2a|a2m)_spin[02](<double>|<float>|_bf)", kernel), kernel
        assert len(e["source_hash"]) == 16
        assert e["bytes_per_launch"] > 0 and e["fetch_kib"] > 0 and e["write_kib"] > 0
        # bytes = 1024 (FETCH x scale + WRITE x scale)
        want = 1024 * (e["fetch_kib"] * e["fetch_scale"] + e["write_kib"] * e["write_scale"])
        assert abs(e["bytes_per_launch"] - want) <= 1e-6 * want
        assert os.path.exists(os.path.join(ROOT, "profiles", e["summary"]))


def test_mfma_record_is_complete():
    """The MFMA instruction counts the bench divides by live launch times: one
    record per FP64 Legendre kernel with the hash of the sources it was taken on
    (the bench drops a record whose kernel sources changed since)."""
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "mfma.json")) as fh:
        rec = json.load(fh)
    assert set(rec) >= {"k_m2a_spin2<double>", "k_a2m_spin2<double>", "k_m2a_spin0<double>", "k_a2m_spin0<double>"}
    for kernel, e in rec.items():
        assert e["flops_per_inst"] == 2 * 16 * 16 * 4
        assert 0 < e["mfma_busy"] < 1 and e["mfma_insts_per_launch"] > 0
        assert os.path.exists(os.path.join(ROOT, "profiles", e["summary"]))
        assert len(e["source_hash"]) == 16
        # executed flops never exceed the folded count of the same launch plus the
        # column padding (125 triples run in 128 map-set columns)
        spin = 0 if "spin0" in kernel else 2
        folded = bench.leg_flops(e["nside"], e["lmax"], spin, e["maps_per_launch"])
        ex = e["mfma_insts_per_launch"] * e["flops_per_inst"]
        assert 0.5 * folded < ex <= folded * 128 / 125 * (1 + 1e-9)
