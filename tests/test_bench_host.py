"""Host-side checks of the benchmark's bookkeeping (no GPU): the one-GPU guard,
the committed HBM-traffic summary and its source-hash gate."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

VH_64x16 = 64 * 64 * 64 * 16 // 2
PRECS = {"f64": 0, "f32": 1, "f16": 2}


def _traffic():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        return json.load(f)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus_requested"] == 2


def test_traffic_summary_is_consistent():
    """bytes_per_launch = (fetch KiB x fetch factor + write KiB x write factor) x 1024, and the
    measured traffic of every hop format lies between its algorithmic minimum (links, each
    input vector once, the output) and 20 % above it."""
    from paper_2502_03249_amd import model
    t = _traffic()
    ff, wf = t["copy_fetch_factor"], t["copy_write_factor"]
    keys = [k for k in t if k.startswith("hop_")]
    assert len(keys) == 6
    for k in keys:
        e = t[k]
        _, prec, recon = k.split("_")
        b = (e["fetch_kib"] * ff + e["write_kib"] * wf) * 1024
        # the factors are stored rounded to three decimals
        assert abs(b - e["bytes_per_launch"]) <= 2e-4 * e["bytes_per_launch"], k
        alg = model.hop_min_bytes(PRECS[prec], int(recon)) * VH_64x16
        assert 1.0 <= e["bytes_per_launch"] / alg <= 1.2, (k, e["bytes_per_launch"] / alg)
        # the output (one parity of colour vectors) is written once
        assert abs(e["write_kib"] * 1024 - model.spinor_bytes(PRECS[prec]) * VH_64x16) <= 0.01 * e["write_kib"] * 1024


def test_traffic_is_gated_on_the_hop_sources(monkeypatch):
    import bench
    t = _traffic()
    if t["hop_f16_12"]["src_hash"] == bench.src_hash():
        assert bench.traffic_for("hop_f16_12", VH_64x16) == t["hop_f16_12"]["bytes_per_launch"]
    monkeypatch.setattr(bench, "src_hash", lambda sources=None: "0" * 16)
    assert bench.traffic_for("hop_f16_12", VH_64x16) is None
    assert bench.traffic_for("no_such_kernel", VH_64x16) is None
