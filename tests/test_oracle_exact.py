"""Pins for oracle/exact.py: brute force with Python ints and Fractions."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact


def _rand_ints(rng, shape, bits):
    out = np.empty(shape, dtype=object)
    for idx in np.ndindex(shape):
        v = int(rng.integers(0, 2 ** 30)) << int(rng.integers(0, max(1, bits - 30)))
        v ^= int(rng.integers(0, 2 ** 30))
        out[idx] = -v if rng.random() < 0.5 else v
    return out


@pytest.mark.parametrize("bits", [8, 40, 70, 130])
def test_exact_int_matmul_matches_brute_force(bits):
    rng = np.random.default_rng(bits)
    X = _rand_ints(rng, (5, 7), bits)
    Y = _rand_ints(rng, (7, 4), bits)
    got = exact.exact_int_matmul(X, Y)
    for i in range(5):
        for j in range(4):
            assert got[i, j] == sum(X[i, h] * Y[h, j] for h in range(7))


def test_exact_int_matmul_empty_inner():
    got = exact.exact_int_matmul(np.zeros((3, 0), dtype=object), np.zeros((0, 2), dtype=object))
    assert got.shape == (3, 2) and all(v == 0 for v in got.ravel())


def test_to_fixed_is_exact():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((6, 5)) * np.exp(8 * rng.standard_normal((6, 5)))
    A[0, 0] = 0.0
    A[1, 1] = 5e-324  # smallest subnormal
    A[2, 2] = -1.7e308
    M, E = exact.to_fixed(A)
    for idx in np.ndindex(A.shape):
        assert Fraction(M[idx]) * Fraction(2) ** E == Fraction(float(A[idx]))


def test_exact_product_against_fractions():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((4, 6)) * np.exp(3 * rng.standard_normal((4, 6)))
    B = rng.standard_normal((6, 3)) * np.exp(3 * rng.standard_normal((6, 3)))
    Mc, E = exact.exact_product(A, B)
    for i in range(4):
        for j in range(3):
            ref = sum(Fraction(float(A[i, h])) * Fraction(float(B[h, j])) for h in range(6))
            assert Fraction(Mc[i, j]) * Fraction(2) ** E == ref


@pytest.mark.parametrize("num,shift,expect", [
    (2 ** 53 + 1, 0, 2.0 ** 53),             # tie -> even
    (2 ** 53 + 3, 0, 2.0 ** 53 + 4),         # tie -> even (upwards)
    (-(2 ** 53 + 1), 0, -(2.0 ** 53)),
    (3, 1, 1.5),
    (1, 1075, 0.0),                          # half the least subnormal: tie -> 0
    (3, 1076, 5e-324),                       # 0.75 of the least subnormal
    (1, 1074, 5e-324),
    (2 ** 1024, 0, float("inf")),
    (-(2 ** 1100), 2, float("-inf")),
    (5, -3, 40.0),
])
def test_round_ratio_to_double(num, shift, expect):
    got = exact.round_ratio_to_double(num, shift)
    assert got == expect and np.signbit(got) == np.signbit(expect)


def test_round_ratio_matches_fraction_rounding():
    # Independent rounding: pick the nearer of the two neighbouring doubles
    # of the exact value (ties to the even significand) with Fractions.
    rng = np.random.default_rng(3)
    for _ in range(300):
        num = int(rng.integers(1, 2 ** 62)) * int(rng.integers(1, 2 ** 40)) + int(rng.integers(0, 2))
        shift = int(rng.integers(-20, 200))
        exact_v = Fraction(num) / Fraction(2) ** shift
        got = exact.round_ratio_to_double(num, shift)
        lo = float(np.nextafter(got, 0.0))
        hi = float(np.nextafter(got, np.inf))
        d = abs(Fraction(got) - exact_v)
        assert d <= abs(Fraction(lo) - exact_v) and d <= abs(Fraction(hi) - exact_v)


def test_scaled_error_zero_on_exact_and_detects_one_ulp():
    A = np.array([[1.0, 2.0], [3.0, -4.0]])
    B = np.array([[0.5, 0.25], [-1.0, 8.0]])
    C = A @ B  # exact: small dyadic values
    assert exact.scaled_error(C, A, B) == 0.0
    C2 = C.copy()
    C2[1, 1] = np.nextafter(C2[1, 1], np.inf)
    e = exact.scaled_errors(C2, A, B)
    ulp = float(np.spacing(C[1, 1]))
    assert e[1, 1] == pytest.approx(ulp / (3 * 0.25 + 4 * 8.0))
    assert e[0, 0] == 0.0
