"""Host-side logic without a GPU: the autotuner's cache lookup and bench.py's profile
reader."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_autotune_lookup_nearest_bucket_per_order():
    from paper_2601_08277_amd import autotune
    cache = {"entries": [
        {"order": 3, "ppc": 2, "tile": [8, 8, 4], "path": "cell_valu"},
        {"order": 3, "ppc": 8, "tile": [8, 8, 8], "path": "cell_valu"},
        {"order": 3, "ppc": 32, "tile": [4, 4, 4], "path": "cell_valu"},
        {"order": 1, "ppc": 8, "tile": [8, 4, 4], "path": "cell_valu"},
    ]}
    assert autotune.lookup(cache, 3, 1)[0] == (8, 8, 4)
    assert autotune.lookup(cache, 3, 5)[0] == (8, 8, 8)       # log-nearest to 8
    assert autotune.lookup(cache, 3, 17)[0] == (4, 4, 4)      # log-nearest to 32
    assert autotune.lookup(cache, 1, 64)[0] == (8, 4, 4)      # only bucket of order 1
    assert autotune.lookup(cache, 2, 8) == ((8, 8, 4), "cell_valu")   # no entry: default


def test_committed_tune_cache_is_well_formed():
    from paper_2601_08277_amd import autotune
    path = os.path.join(ROOT, "paper_2601_08277_amd", "tune_cache.json")
    cache = autotune.load(path)
    assert cache["blocks_per_cu"] >= 1
    orders = {e["order"] for e in cache["entries"]}
    assert orders == {1, 2, 3}
    for e in cache["entries"]:
        assert len(e["tile"]) == 3 and all(t >= 4 for t in e["tile"])


def test_bench_traffic_reader(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "a.txt"
    src.write_text("kernel source")
    import hashlib
    sha = hashlib.sha256(b"kernel source").hexdigest()
    prof = tmp_path / "p.md"
    prof.write_text(f"# x\n\ntraffic_bytes_per_launch: 12345\nsource_sha256: {sha}\n"
                    f"source_files: a.txt\nworkload_key: n=128 ppc=8 tile=8x8x4 slack=0.5\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("auto", (8, 8, 4), 128, 8, 0.5) == 12345.0
    assert bench.measured_traffic("mfma_bf16", (8, 8, 4), 128, 8, 0.5) is None   # other kernel
    assert bench.measured_traffic("auto", (8, 8, 8), 128, 8, 0.5) is None        # other tile
    assert bench.measured_traffic("auto", (8, 8, 4), 128, 8, 0.25) is None       # other slack
    src.write_text("changed source")
    assert bench.measured_traffic("auto", (8, 8, 4), 128, 8, 0.5) is None        # stale counters


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode != 0 and "one GPU" in r.stderr
