"""Exact integer and rational matrix products (oracle; test infrastructure).

Pins: ``tests/test_oracle_exact.py`` checks every function here against
brute-force Python-int loops and ``fractions.Fraction`` on small inputs,
against numpy int64 matmul where that is exact, and checks the rounding
helper against CPython's correctly rounded ``int / int``.

What is computed
----------------
* ``exact_int_matmul``: the exact product of two integer matrices of any
  magnitude. Each operand is split into non-negative limbs of ``w`` bits
  with a separate sign, so every int64 partial product sum is bounded by
  ``K * 2**(2w) < 2**63``; the limb products are recombined with Python ints.
* ``to_fixed``: a FP64 matrix as ``M * 2**E`` with integer ``M`` exactly.
* ``exact_product``: the exact product AB of FP64 matrices (the
  ``C_exact`` of the error metric), as integers times a power of two.
* ``scaled_error``: ``max_ij |C_ij - (AB)_ij| / (|A||B|)_ij``, every term
  exact, the final ratio converted to float once.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

__all__ = ["to_object_ints", "exact_int_matmul", "to_fixed", "exact_product",
           "round_ratio_to_double", "scaled_error", "scaled_errors"]


def to_object_ints(X) -> np.ndarray:
    """Integer-valued array (int64, float64 holding integers, or object) as
    a numpy object array of exact Python ints."""
    X = np.asarray(X)
    out = np.empty(X.shape, dtype=object)
    flat = X.ravel()
    res = out.ravel()
    for idx in range(flat.size):
        v = flat[idx]
        iv = int(v)
        if isinstance(v, (float, np.floating)) and float(iv) != float(v):
            raise ValueError("non-integer value in integer matrix")
        res[idx] = iv
    return out


def _split_limbs(X: np.ndarray, w: int):
    """|X| split into non-negative ``w``-bit limbs (least significant first),
    each as int64 with the sign of X applied, so ``X = sum_i L_i * 2**(w*i)``."""
    sign = np.empty(X.shape, dtype=np.int64)
    mag = np.empty(X.shape, dtype=object)
    fl_x, fl_s, fl_m = X.ravel(), sign.ravel(), mag.ravel()
    nbits = 0
    for idx in range(fl_x.size):
        v = int(fl_x[idx])
        fl_s[idx] = -1 if v < 0 else 1
        a = -v if v < 0 else v
        fl_m[idx] = a
        nbits = max(nbits, a.bit_length())
    nl = max(1, -(-nbits // w))
    mask = (1 << w) - 1
    limbs = []
    for i in range(nl):
        L = np.empty(X.shape, dtype=np.int64)
        fl_l = L.ravel()
        for idx in range(fl_m.size):
            fl_l[idx] = (fl_m[idx] >> (w * i)) & mask
        limbs.append(L * sign)
    return limbs


def exact_int_matmul(X, Y) -> np.ndarray:
    """Exact ``X @ Y`` for integer matrices of arbitrary magnitude.

    Returns an object array of Python ints. Limb width ``w`` is chosen so
    that ``K * 2**(2w) < 2**63``: each int64 matmul of two limb planes is
    then exact, and the planes are recombined with exact Python ints.
    """
    X = np.asarray(X)
    Y = np.asarray(Y)
    if X.ndim != 2 or Y.ndim != 2 or X.shape[1] != Y.shape[0]:
        raise ValueError("shape mismatch")
    K = X.shape[1]
    m, n = X.shape[0], Y.shape[1]
    out = np.zeros((m, n), dtype=object)
    out[...] = 0
    if K == 0 or m == 0 or n == 0:
        return out
    w = (62 - K.bit_length()) // 2
    if w < 1:
        raise ValueError("inner dimension too large for the limb split")
    LX = _split_limbs(X, w)
    LY = _split_limbs(Y, w)
    for i, a in enumerate(LX):
        for j, b in enumerate(LY):
            part = a @ b  # exact: |sum| <= K * (2**w - 1)**2 < 2**63
            out = out + part.astype(object) * (1 << (w * (i + j)))
    return out


def to_fixed(A: np.ndarray):
    """FP64 matrix A as ``(M, E)``: object array of ints M with A == M * 2**E.

    Every finite double is ``mant * 2**ex`` with an integer ``mant`` of at
    most 53 bits (``numpy.frexp`` gives ``A = f * 2**e``, ``f`` in [0.5, 1),
    and ``f * 2**53`` is an integer). ``E`` is the least ``ex`` over the
    nonzero entries, so every entry becomes an exact integer multiple.
    """
    A = np.asarray(A, dtype=np.float64)
    if not np.all(np.isfinite(A)):
        raise ValueError("non-finite entry")
    f, e = np.frexp(A)
    mant = (f * 2.0 ** 53).astype(np.int64)
    ex = e.astype(np.int64) - 53
    nz = mant != 0
    E = int(ex[nz].min()) if np.any(nz) else 0
    M = np.empty(A.shape, dtype=object)
    fl_m, fl_mant, fl_ex = M.ravel(), mant.ravel(), ex.ravel()
    for idx in range(fl_m.size):
        v = int(fl_mant[idx])
        fl_m[idx] = v << (int(fl_ex[idx]) - E) if v != 0 else 0
    return M, E


def exact_product(A: np.ndarray, B: np.ndarray):
    """Exact AB as ``(Mc, E)`` with AB == Mc * 2**E (Mc: object ints)."""
    MA, EA = to_fixed(A)
    MB, EB = to_fixed(B)
    return exact_int_matmul(MA, MB), EA + EB


def round_ratio_to_double(num: int, shift: int) -> float:
    """RN(num * 2**(-shift)) into FP64, one rounding, ties to even.

    CPython's ``int / int`` is correctly rounded, subnormals included, and
    ``float(int)`` rounds to nearest even. A result beyond the largest
    double rounds to an infinity of the right sign.
    """
    try:
        if shift >= 0:
            return num / (1 << shift)
        return float(num << (-shift))
    except OverflowError:
        return float("inf") if num > 0 else float("-inf")


def scaled_errors(C: np.ndarray, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Elementwise ``|C - AB| / (|A||B|)`` as float64, each ratio exact
    before its final conversion. Entries with ``(|A||B|)_ij = 0`` get 0 if
    C_ij is 0, else inf."""
    MA, EA = to_fixed(A)
    MB, EB = to_fixed(B)
    Cex = exact_int_matmul(MA, MB)
    absA = np.vectorize(abs, otypes=[object])(MA)
    absB = np.vectorize(abs, otypes=[object])(MB)
    den = exact_int_matmul(absA, absB)
    E = EA + EB
    out = np.empty(C.shape, dtype=np.float64)
    scale = Fraction(2) ** E
    for i in range(C.shape[0]):
        for j in range(C.shape[1]):
            diff = abs(Fraction(float(C[i, j])) - Fraction(Cex[i, j]) * scale)
            d = den[i, j]
            if d == 0:
                out[i, j] = 0.0 if diff == 0 else float("inf")
            else:
                out[i, j] = float(diff / (Fraction(d) * scale))
    return out


def scaled_error(C: np.ndarray, A: np.ndarray, B: np.ndarray) -> float:
    """``max_ij |C_ij - (AB)_ij| / (|A||B|)_ij`` (0 for an empty product)."""
    if C.size == 0:
        return 0.0
    return float(np.max(scaled_errors(C, A, B)))
