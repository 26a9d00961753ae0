"""Host-side logic of bench.py (CPU only): the one-GPU guard and the
algorithmic byte counts the roofline divides by."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (module import does no GPU work)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == ""   # no JSON line for a refused run


def test_algorithmic_bytes_per_pair():
    # the bin vector (4^q bits), the 4-byte bin id, the 4-byte count, 1/8 byte of pass bit
    assert bench.algorithmic_bytes_per_pair(5) == 128 + 4 + 4 + 0.125
    assert bench.algorithmic_bytes_per_pair(6) == 512 + 4 + 4 + 0.125


def test_algorithmic_bytes_per_read():
    import numpy as np
    w = {"read_len": np.array([100, 150, 250], dtype=np.uint32)}
    # packed bases ceil(L / 4), read offset 8, length 4, tolerance 4, candidate offset 8
    assert bench.algorithmic_bytes_per_read(w) == (25 + 38 + 63) / 3 + 24
