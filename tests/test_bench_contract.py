"""bench.py's contract on the host: the one-GPU guard, and the algorithmic bytes and flops per
triangle that its roofline figures are computed from (the algorithmic ten vector passes plus
60 B of geometry, the fused kernel's own eight passes plus the geometry and neighbour table, and
the FMA count of one fused CG iteration), and the reader of the stored oracle samples."""
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


@pytest.mark.parametrize("p,nphi,expect", [(1, 3, 300), (2, 6, 540), (3, 10, 860), (4, 15, 1260)])
def test_algorithmic_bytes_per_triangle(p, nphi, expect):
    # the roofline's algorithmic bytes: ten vector passes + 60 B of geometry and connectivity
    # (80 N_phi + 60 in FP64, 40 N_phi + 60 in FP32)
    assert bench.alg_bytes_per_tri(nphi) == expect
    assert bench.alg_bytes_per_tri(nphi, 4) == 40 * nphi + 60


def test_golden_sample_reader_and_error():
    import numpy as np
    g = bench.read_golden("tgv128_p3")
    assert g is not None
    idx, val, maxabs = g
    assert len(idx) == len(val) == 512 and maxabs > 0
    p = np.zeros(int(idx.max()) + 1)
    p[idx] = val
    assert bench.err_vs_oracle(g, p) == 0.0
    p[idx[3]] += 1e-3 * maxabs
    assert abs(bench.err_vs_oracle(g, p) - 1e-3) < 1e-12


def test_flops_per_triangle():
    # 2 [3 N^2 + 3 (4 (p+1) N + 2 (p+1)^2 + 2 N (p+1) + 16 (p+1)) + 16 N] at p = 3, N = 10
    n, ne = 10, 4
    assert bench.step_flops_per_tri(3) == 2 * (3 * n * n + 3 * (4 * ne * n + 2 * ne * ne +
                                                               2 * n * ne + 16 * ne) + 16 * n)
    assert bench.step_flops_per_tri(3) == 2936
