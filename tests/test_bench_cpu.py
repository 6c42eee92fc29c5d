"""Host-side checks of bench.py: the one-GPU contract and the flop model (no GPU)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2407_14633_amd import workload as W  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_circulant_detection():
    dev = W.zigzag_cnt(9, 4)
    assert bench.lead_is_circulant(dev.left) and bench.lead_is_circulant(dev.right)
    rnd = W.random_device(3, 5, seed=2, period=2)
    assert not bench.lead_is_circulant(rnd.left)
    M = np.array([[1, 2, 3], [3, 1, 2], [2, 3, 1]], complex)
    N = M.copy()
    N[2, 0] += 1e-12
    assert bench.is_circulant(M) and not bench.is_circulant(N)


def test_flop_model_counts():
    """Recursion flops: 2 chains per node of (N-1) dense inverses (8 b^3 each; the sparse
    coupling products are not counted), plus the final inverse of the real-axis chains;
    with b, K, N small enough to count by hand."""
    p = W.small_problem()
    N, b = p.device.n_rings, p.device.b
    K = bench.ell_width(p.device)
    assert K == 2                                     # zigzag couplings t(I + S^T) and tI
    f = bench.algorithmic_flops(p, np.full((p.grid.n_c + p.grid.n_r, 2), 10))
    inv = 8.0 * b ** 3
    n_c, n_r = p.grid.n_c, p.grid.n_r
    assert f["recur"] == 2 * (n_c + n_r) * (N - 1) * inv + 2 * n_r * inv
    assert f["cdiag"] == n_c * N * inv
    # ring-mode decimation: 115 b flops per two-ring doubling step and mode, + per-node finish
    nodes = n_c + n_r
    assert f["decimate"] == 2 * (115.0 * b * 10 * nodes + (28.0 * b + 8.0 * b * b) * nodes)
