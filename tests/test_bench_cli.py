"""Host-side parts of bench.py: a run on more than one GPU is refused with a
message before any GPU work, and the algorithmic byte model of the roofline
is 4 B per k-hop id, 4 B per adjacency entry and 32 B per non-isolated
vertex in FP32 (48 B in FP64)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    P, m, n = 496_749_070, 1_008_492, 122_633
    assert bench.algorithmic_bytes_per_iter(P, 2 * m, n, 8) == 4 * P + 8 * m + 32 * n
    assert bench.algorithmic_bytes_per_iter(P, 2 * m, n, 16) == 4 * P + 8 * m + 48 * n
    # the force kernel's share leaves out the position write
    assert bench.force_kernel_bytes(P, 2 * m, n, 8) == 4 * P + 8 * m + 24 * n
