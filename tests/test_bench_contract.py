"""bench.py's contract on the host: the one-GPU guard, and the algorithmic bytes and flops per
triangle that its roofline figures are computed from (the counts derived from the operator
form: eight vector passes plus the geometry and neighbour table, and the FMA count of one
fused CG iteration)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("p,nphi,expect", [(1, 3, 240), (2, 6, 432), (3, 10, 688), (4, 15, 1008)])
def test_bytes_per_triangle(p, nphi, expect):
    # x, r, q, d read and written (8 passes of N_phi words) + 32 B geometry + 16 B neighbours
    assert bench.step_bytes_per_tri(nphi) == expect
    assert bench.step_bytes_per_tri(nphi, 4) == 32 * nphi + 48


def test_flops_per_triangle():
    # 2 [3 N^2 + 3 (4 (p+1) N + 2 (p+1)^2 + 2 N (p+1) + 16 (p+1)) + 16 N] at p = 3, N = 10
    n, ne = 10, 4
    assert bench.step_flops_per_tri(3) == 2 * (3 * n * n + 3 * (4 * ne * n + 2 * ne * ne +
                                                               2 * n * ne + 16 * ne) + 16 * n)
    assert bench.step_flops_per_tri(3) == 2936
