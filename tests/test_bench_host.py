"""Host-side checks of the benchmark's bookkeeping (no GPU)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_closed_form():
    # one level: every pixel read once and written once
    assert bench.algorithmic_bytes(8192, 8192, 1, 4) == 2 * 8192 * 8192 * 4 == 536870912
    # L levels of a 2^k square: 8 B/px * (4/3)(1 - 4^-L), exactly
    for L in range(1, 8):
        n = 4096
        expect = 8 * n * n * 4 * (1 - 4.0 ** -L) / 3
        assert bench.algorithmic_bytes(n, n, L, 4) == expect
    # odd sizes halve with ceil, as the transform does
    assert bench.algorithmic_bytes(5, 3, 2, 2) == 2 * 2 * (5 * 3 + 3 * 2)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

