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


@pytest.mark.parametrize("phi,shape,nm,seed,cap", [(0.5, (12, 10, 40), 10, 4, -30),
                                                   (4.0, (9, 11, 64), 12, 5, -24),
                                                   (0.5, (7, 6, 300), 16, 6, -50)])
def test_certified_bound_covers_exact_errors(phi, shape, nm, seed, cap):
    """bench.py's whole-matrix bound is an upper bound of the exact scaled
    error on every entry of the oracle's product, with the oracle's shifts,
    and stays within the entrywise bound of Sec. VIII-E's error analysis (it
    is not vacuous)."""
    torch = pytest.importorskip("torch")
    from oracle import moduli, scheme
    m, n, k = shape
    A, B = operand_pair(m, n, k, phi, seed)
    A[3] = 0.0
    B[:, 4] = 0.0
    ms = moduli.best_coprime_set(nm)
    ba, bb = scheme.kept_bits("W", moduli.product(ms), k)
    r = scheme.emulate(A, B, ms, "W")
    C = r["C"]
    bound, s, t = bench.certified_error_bound(torch.from_numpy(A), torch.from_numpy(B),
                                              torch.from_numpy(C), ba, bb)
    assert np.array_equal(s.numpy(), r["s"]) and np.array_equal(t.numpy(), r["t"])
    b = bound.numpy()
    err = exact.scaled_errors(C, A, B)
    assert np.all(np.isfinite(b)) and np.all(b >= err)
    assert np.all(b[3] == 0) and np.all(b[:, 4] == 0)
    # the a priori entrywise bound: truncation below 2^(1 - beta) of each
    # row's (column's) largest magnitude, plus the final rounding
    amax = np.abs(A).max(axis=1)[:, None]
    bmax = np.abs(B).max(axis=0)[None, :]
    den = np.abs(A) @ np.abs(B)
    pri = (2.0 ** (1 - ba) * amax * np.abs(B).sum(axis=0)[None, :] +
           2.0 ** (1 - bb) * bmax * np.abs(A).sum(axis=1)[:, None] +
           2.0 ** (2 - ba - bb) * k * amax * bmax + 2.0 ** -53 * np.abs(C))
    nz = den > 0
    assert np.all(b[nz] <= 1.001 * pri[nz] / den[nz])
    assert b[nz].max() < 2.0 ** cap


def test_certified_bound_misses_a_wrong_rounding():
    """The bound holds only for the correctly rounded product: a C two ulps
    away at one entry of a product with no truncation exceeds it there."""
    torch = pytest.importorskip("torch")
    from oracle import moduli, scheme
    rng = np.random.default_rng(7)
    A = rng.integers(-1000, 1000, (5, 9)).astype(np.float64)
    B = rng.integers(-1000, 1000, (9, 4)).astype(np.float64)
    ms = moduli.best_coprime_set(12)
    ba, bb = scheme.kept_bits("W", moduli.product(ms), 9)
    C = scheme.emulate(A, B, ms, "W")["C"]
    assert np.array_equal(C, A @ B)  # small integers: exact
    bound, _, _ = bench.certified_error_bound(torch.from_numpy(A), torch.from_numpy(B),
                                              torch.from_numpy(C), ba, bb)
    Cw = C.copy()
    Cw[2, 1] = np.nextafter(np.nextafter(C[2, 1], np.inf), np.inf)
    err = exact.scaled_errors(Cw, A, B)
    assert err[2, 1] > bound.numpy()[2, 1]
