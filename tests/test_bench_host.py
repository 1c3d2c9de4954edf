"""CPU tests of bench.py's host logic: the exact sampled error of the
moduli sweep agrees with the oracle's exact scaled error, and runs for
more than one GPU are refused with a message."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import exact
from workloads import operand_pair

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("phi,shape,seed", [(0.5, (9, 7, 50), 1), (4.0, (6, 8, 300), 2)])
def test_exact_scaled_error_matches_oracle(phi, shape, seed):
    m, n, k = shape
    A, B = operand_pair(m, n, k, phi, seed)
    C = A @ B  # a product with rounding errors of its own
    C[1, 2] = np.nextafter(C[1, 2], np.inf)
    rows, cols = [0, 1, m - 1], [0, 2, n - 1]
    got = bench.exact_scaled_error(C, A, B, rows, cols)
    want = float(exact.scaled_errors(C[np.ix_(rows, cols)], A[rows], B[:, cols]).max())
    assert got == want and got > 0


def test_exact_scaled_error_zero_row():
    A, B = operand_pair(4, 3, 20, 0.5, 3)
    A[2] = 0.0
    C = A @ B
    assert bench.exact_scaled_error(C, A, B, [2], [0, 1, 2]) == 0.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
