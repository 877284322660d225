"""The benchmark's contract on the CPU: one-GPU refusal, and the rule that HBM
traffic from rocprofv3 counters is reported only for the sweep source and
launch shape it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_traffic_requires_matching_source_and_shape(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    shape = "4,16,0,1,1,1,1"
    entry = {"kernel_source": bench.sweep_source_hash(), "shape": shape, "bytes_per_launch": 123456789}
    f.write_text(json.dumps({"sweep_f64|cube1M|m4": entry}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic("sweep_f64|cube1M|m4", shape) == 123456789
    assert bench.stored_traffic("sweep_f64|cube1M|m4", "2,16,0,1,1,1,1") is None   # other launch shape
    assert bench.stored_traffic("sweep_f64|cube1M|m2", shape) is None              # other workload
    f.write_text(json.dumps({"sweep_f64|cube1M|m4": dict(entry, kernel_source="0" * 16)}))
    assert bench.stored_traffic("sweep_f64|cube1M|m4", shape) is None              # other kernel source
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.stored_traffic("sweep_f64|cube1M|m4", shape) is None


def test_committed_traffic_is_consistent_with_shipped_shape():
    """The committed counters convert to bytes by the calibration factors they
    state, and were taken in the launch shape the shipped tuning file gives
    the 1M-node m = 4 sweep (so the default benchmark can report them)."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        t = json.load(fh)["sweep_f64|cube1M|m4"]
    fetch = t["fetch_kib_per_dispatch"] * 1024 * t["fetch_scale"]
    write = t["write_kib_per_dispatch"] * 1024 * t["write_scale"]
    assert abs(fetch - t["fetch_bytes"]) <= 1e-5 * t["fetch_bytes"]
    assert abs(write - t["write_bytes"]) <= 1e-5 * t["write_bytes"]
    assert t["bytes_per_launch"] == t["fetch_bytes"] + t["write_bytes"]
    # 941,192 interior rows of n = 70: 12n + 24 algorithmic bytes per row
    assert t["alg_read_bytes"] + t["alg_write_bytes"] == 941192 * (12 * 70 + 24)
    with open(os.path.join(ROOT, "paper_2502_12878_amd", "tuned_gfx950.json")) as fh:
        tuned = json.load(fh)
    # the Dirichlet problem's key (a key with Neumann rows ends in |nn<count>)
    keys = [k for k in tuned if k.startswith("sweep|") and k.split("|")[3:6] == ["941192", "65887360", "70"]
            and "|nn" not in k]
    assert len(keys) == 1
    assert ",".join(str(v) for v in tuned[keys[0]][:7]) == t["shape"]
