"""The autotuner's cache file: a store keeps every other entry of a valid
JSON file, also one whose arrays span several lines, and leaves valid JSON
with one entry per line."""
import json

import pytest

import rbf_inputs as ri

pytestmark = pytest.mark.gpu


def test_store_keeps_multiline_entries(tmp_path, monkeypatch):
    from paper_2502_12878_amd import Problem
    print("tuning cache: 3D side 12, m=2, n=20", flush=True)
    cache = tmp_path / "tuned.json"
    other = {"sweep|other-arch|L1|1|2|3|c0": [2, 4, 1, 0, 0, 0, 0, 0], "weights|other-arch|3|30": [8]}
    cache.write_text(json.dumps(other, indent=2))  # arrays over several lines
    monkeypatch.setenv("RBF_AUTOTUNE_CACHE", str(cache))
    monkeypatch.setenv("RBF_AUTOTUNE_FORCE", "1")
    xyz, typ = ri.jittered_grid(3, 12, 0.3, 61)
    p = Problem(0)
    p.set_nodes(xyz, typ)
    p.build_stencils(20)
    p.compute_weights(2)
    p.autotune()
    p.close()
    d = json.loads(cache.read_text())
    for k, v in other.items():
        assert d[k] == v
    assert any(k.startswith("sweep|") and k not in other for k in d)
    lines = [l for l in cache.read_text().splitlines() if '"' in l]
    assert len(lines) == len(d)  # one entry per line
