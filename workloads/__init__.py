"""Seeded synthetic operands for the emulated-DGEMM workloads.

This module holds no arithmetic of the emulation method. It only draws
random FP64 operands with the shapes and value distributions of the
workloads, so that the CPU oracle and the GPU path can be fed identical
bytes.

Distributions
-------------
* ``phi_matrix``: entries ``(U(-1/2, 1/2)) * exp(phi * N(0, 1))``. ``phi``
  controls the dynamic range of each row and column (``phi = 0.5`` mild,
  ``phi = 4`` strongly skewed rows, which is the case the paper's error
  analysis of skewed rows warns about, Sec. VIII-E).
* ``row_exponent_matrix``: the paper's timing operands (Table "setup",
  Sec. VI): row ``i`` is ``N(0, 1) * 2**e_i`` with integer ``e_i`` drawn from
  ``[-20, 20)``.
* ``grouped_shapes``: the batched workload, 512 independent products with
  ``m, n ~ U[64, 2048]`` and ``k ~ U[64, 4096]``.
"""
from __future__ import annotations

import numpy as np

__all__ = ["phi_matrix", "row_exponent_matrix", "operand_pair", "grouped_shapes",
           "integer_matrix"]


def phi_matrix(rows: int, cols: int, phi: float, seed: int) -> np.ndarray:
    """FP64 ``rows x cols`` matrix, entries ``U(-1/2,1/2) * exp(phi * N(0,1))``."""
    rng = np.random.default_rng(seed)
    u = rng.random((rows, cols)) - 0.5
    g = rng.standard_normal((rows, cols))
    return np.ascontiguousarray(u * np.exp(phi * g), dtype=np.float64)


def row_exponent_matrix(rows: int, cols: int, seed: int, lo: int = -20,
                        hi: int = 20) -> np.ndarray:
    """FP64 matrix whose row ``i`` is ``N(0,1) * 2**e_i``, ``e_i`` in ``[lo, hi)``."""
    rng = np.random.default_rng(seed)
    e = rng.integers(lo, hi, size=rows)
    g = rng.standard_normal((rows, cols))
    return np.ascontiguousarray(np.ldexp(g, e[:, None]), dtype=np.float64)


def operand_pair(m: int, n: int, k: int, phi: float, seed: int):
    """A (m x k) from ``seed`` and B (k x n) from ``seed + 1``."""
    return phi_matrix(m, k, phi, seed), phi_matrix(k, n, phi, seed + 1)


def integer_matrix(rows: int, cols: int, bound: int, seed: int) -> np.ndarray:
    """FP64 matrix of integers drawn uniformly from ``[-bound, bound]``."""
    rng = np.random.default_rng(seed)
    return rng.integers(-bound, bound + 1, size=(rows, cols)).astype(np.float64)


def grouped_shapes(count: int = 512, seed: int = 0, mn_lo: int = 64,
                   mn_hi: int = 2048, k_lo: int = 64, k_hi: int = 4096):
    """List of ``(m, n, k)`` for the batched workload, bounds inclusive."""
    rng = np.random.default_rng(seed)
    m = rng.integers(mn_lo, mn_hi + 1, size=count)
    n = rng.integers(mn_lo, mn_hi + 1, size=count)
    k = rng.integers(k_lo, k_hi + 1, size=count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(m, n, k)]
