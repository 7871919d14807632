"""Host-side parts of bench.py (no GPU): the refusal of more than one GPU,
and the method's bytes per phase, which sum to the floor of one generation
(write the points, read them to index, read them once to search, write the
row offsets, write col_idx)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_method_bytes_per_phase_sum_to_the_floor():
    for n, m in ((10_000, 29_457), (100_000_000, 998_392_276)):
        parts = {ph: bench.algorithmic_bytes(ph, n, m) for ph in ("sample", "keys+sort", "count", "emit")}
        assert parts["count"] == 16 * n + 8 * (n + 1)
        assert parts["emit"] == 4 * 2 * m
        assert sum(parts.values()) == 56 * n + 8 * m + 8
        # staging traffic, the sort passes and the index's records are the
        # design's traffic: no phase outside the table has method's bytes
        assert bench.algorithmic_bytes("gather", n, m) == 0


def test_source_hash_covers_the_kernel_sources():
    h = bench._source_sha()
    assert len(h) == 16 and int(h, 16) >= 0
    assert h == bench._source_sha()
