"""Host-side logic of bench.py (no GPU): the one-GPU guard, the source-hash
rule for counted traffic, and the unit counts the rooflines divide by."""
import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_counted_traffic_follows_the_source_hash(tmp_path):
    # a summary whose source hash matches the sources is reported ...
    import hashlib
    h = hashlib.sha256()
    for f in bench.GAS_TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2303_02346_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    fresh = tmp_path / "fresh.md"
    fresh.write_text(f"traffic_bytes_per_launch: 12345\nsource-sha256: {h.hexdigest()[:16]}\n")
    assert bench.counted_traffic(str(fresh), bench.GAS_TRAFFIC_SOURCES) == 12345
    # ... one taken on other sources, or a missing one, is not
    stale = tmp_path / "stale.md"
    stale.write_text(f"traffic_bytes_per_launch: 12345\nsource-sha256: 0{h.hexdigest()[:15]}\n")
    assert bench.counted_traffic(str(stale), bench.GAS_TRAFFIC_SOURCES) is None
    assert bench.counted_traffic(str(tmp_path / "missing.md"), bench.GAS_TRAFFIC_SOURCES) is None


def test_gas_state_values():
    # three staggered velocity grids of (n + 1) n^2 faces and K cell scalars
    assert bench.sim_values(4, 2) == 3 * 5 * 16 + 2 * 64
    assert bench.sim_values(128, 2) * 8 == 84279296


def test_active_nodes_matches_brute_force():
    rng = np.random.default_rng(0)
    n = 16
    x = rng.uniform(0.2, 0.8, (300, 3))
    nodes = set()
    for p in x:
        b = np.floor(p * n - 0.5).astype(int)
        for di in range(3):
            for dj in range(3):
                for dk in range(3):
                    nodes.add((b[0] + di, b[1] + dj, b[2] + dk))
    assert bench.active_nodes(x, n) == len(nodes)
