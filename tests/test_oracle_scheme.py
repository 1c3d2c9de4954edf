"""Pins for oracle/scheme.py: brute force, CRT round trips, the plain
definition, invariance over modulus sets, integer special cases and the
entrywise error bound of Sec. VIII-E."""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import exact, scheme
from oracle import moduli as md
from workloads import operand_pair, integer_matrix, row_exponent_matrix


def test_frexp_exponents_bracket_row_max():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((20, 9)) * np.exp(6 * rng.standard_normal((20, 9)))
    A[3] = 0.0
    A[4, 2] = 5e-324
    A[4, [0, 1, 3, 4, 5, 6, 7, 8]] = 0.0
    e, nz, fin = scheme.frexp_exponents(A, 1)
    for i in range(20):
        mx = max(abs(Fraction(float(x))) for x in A[i])
        if mx == 0:
            assert not nz[i]
            continue
        assert Fraction(2) ** (int(e[i]) - 1) <= mx < Fraction(2) ** int(e[i])
    assert e[4] == -1073
    eB, nzB, _ = scheme.frexp_exponents(A.T, 0)
    assert np.array_equal(e, eB) and np.array_equal(nz, nzB)


def test_kept_bits_window_is_tight():
    for n in (10, 14, 16, 20):
        P = md.product(md.best_coprime_set(n))
        for K in (1, 256, 8192, 16384):
            bA, bB = scheme.kept_bits("W", P, K)
            assert bA - bB in (0, 1)
            assert P > 2 * K * (2 ** bA - 1) * (2 ** bB - 1)
            # one more bit on the smaller side would break K * 2**w <= (P-1)/2
            assert K * 2 ** (bA + bB + 1) > (P - 1) // 2


def test_truncate_against_fractions():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((6, 7)) * np.exp(5 * rng.standard_normal((6, 7)))
    e, nz, _ = scheme.frexp_exponents(A, 1)
    for beta in (20, 53, 70, 127):
        s = scheme.shifts_from_bits(e, nz, beta)
        T = scheme.truncate(A, s, 1)
        for idx in np.ndindex(A.shape):
            v = Fraction(float(A[idx])) * Fraction(2) ** int(s[idx[0]])
            ref = math.floor(v) if v >= 0 else math.ceil(v)
            assert T[idx] == ref and abs(ref) < 2 ** beta


@pytest.mark.parametrize("m", [2, 3, 199, 239, 255, 256])
def test_balanced_residues_brute_force(m):
    vals = np.array([[-(2 ** 70) - 5, -129, -128, -1, 0, 1, 127, 128, 2 ** 64 + 3, 255, 256]],
                    dtype=object)
    r = scheme.balanced_residues(vals, m)
    for v, x in zip(vals.ravel(), r.ravel()):
        assert (int(x) - v) % m == 0
        assert -(m // 2) <= x <= (m + 1) // 2 - 1
    if m == 256:
        assert r[0, 2] == -128 and r[0, 7] == -128


def test_residue_gemm_brute_force():
    rng = np.random.default_rng(2)
    RA = rng.integers(-128, 128, (4, 33))
    RB = rng.integers(-128, 128, (33, 5))
    for blas in (False, True):
        W, Z = scheme.residue_gemm(RA, RB, 251, blas=blas)
        for i in range(4):
            for j in range(5):
                w = sum(int(RA[i, h]) * int(RB[h, j]) for h in range(33))
                assert W[i, j] == w and Z[i, j] == w % 251


@pytest.mark.parametrize("n", [2, 10, 16, 20])
def test_crt_round_trip_and_window_edges(n):
    ms = md.best_coprime_set(n)
    P = md.product(ms)
    half = (P - 1) // 2
    rng = np.random.default_rng(n)
    xs = [half, -half, 0, 1, -1] + [int(rng.integers(-2 ** 62, 2 ** 62)) * (P // 2 ** 70 + 1) % half
                                    for _ in range(20)]
    X = np.array([xs], dtype=object)
    Z = np.stack([np.vectorize(lambda v, m=m: v % m, otypes=[np.int64])(X) for m in ms])
    back = scheme.crt_balanced(Z, ms)
    assert all(int(a) == int(b) for a, b in zip(back.ravel(), X.ravel()))


@pytest.mark.parametrize("mode,n", [("W", 14), ("W", 10), ("F53", 16), ("G", 14), ("G", 12)])
def test_scheme_equals_definition(mode, n):
    A, B = operand_pair(21, 13, 37, 1.0, 5)
    A[2, :] = 0.0
    B[:, 3] = 0.0
    ms = md.best_coprime_set(n)
    r = scheme.emulate(A, B, ms, mode)
    C = scheme.definition_product(A, B, ms, mode)
    assert np.array_equal(r["C"], C)
    assert np.all(r["C"][2, :] == 0) and np.all(r["C"][:, 3] == 0)


def test_result_independent_of_moduli_at_fixed_bits():
    A, B = operand_pair(9, 11, 64, 0.5, 7)
    s1 = md.best_coprime_set(16, 256)
    s2 = list(md.PAPER_INT8_239_SET)
    c1 = scheme.emulate(A, B, s1, "F53")["C"]
    c2 = scheme.emulate(A, B, s2, "F53")["C"]
    assert np.array_equal(c1, c2)


def test_integer_operands_give_the_exact_product():
    A = integer_matrix(12, 40, 1000, 3)
    B = integer_matrix(40, 10, 1000, 4)
    ref = A.astype(np.int64) @ B.astype(np.int64)
    for mode, n in (("W", 14), ("F53", 16), ("G", 14)):
        C = scheme.emulate(A, B, md.best_coprime_set(n), mode)["C"]
        assert np.array_equal(C, ref.astype(np.float64))


def _error_bound(A, B, bA, bB):
    """Entrywise bound on |C - AB| (generalising Sec. VIII-E to beta bits):
    2**(1-bA) a_max sum|b| + 2**(1-bB) b_max sum|a| + 2**(2-bA-bB) K a_max b_max
    + 2**-53 |C|; computed with a small safety factor for FP64 evaluation."""
    K = A.shape[1]
    amax = np.max(np.abs(A), axis=1)[:, None]
    bmax = np.max(np.abs(B), axis=0)[None, :]
    s1 = 2.0 ** (1 - bA) * amax * np.sum(np.abs(B), axis=0)[None, :]
    s2 = 2.0 ** (1 - bB) * bmax * np.sum(np.abs(A), axis=1)[:, None]
    s3 = 2.0 ** (2 - bA - bB) * K * amax * bmax
    return s1, s2, s3


@pytest.mark.parametrize("phi,mode,n", [(0.5, "W", 12), (4.0, "W", 16), (1.0, "F53", 16)])
def test_entrywise_error_bound(phi, mode, n):
    A, B = operand_pair(10, 8, 50, phi, 11)
    ms = md.best_coprime_set(n)
    r = scheme.emulate(A, B, ms, mode)
    bA, bB = r["bits"]
    s1, s2, s3 = _error_bound(A, B, bA, bB)
    Mc, E = exact.exact_product(A, B)
    for i in range(10):
        for j in range(8):
            err = abs(Fraction(float(r["C"][i, j])) - Fraction(Mc[i, j]) * Fraction(2) ** E)
            bound = (Fraction(float(s1[i, j])) + Fraction(float(s2[i, j])) + Fraction(float(s3[i, j]))) \
                * Fraction(1 + 2 ** -40) + abs(Fraction(float(r["C"][i, j]))) * Fraction(2) ** -53
            assert err <= bound


def test_mode_g_window_holds_entrywise():
    A = row_exponent_matrix(12, 30, 1)
    B = row_exponent_matrix(30, 9, 2)
    ms = md.best_coprime_set(12)
    P = md.product(ms)
    r = scheme.emulate(A, B, ms, "G")
    absA = np.vectorize(abs, otypes=[object])(r["Aint"])
    absB = np.vectorize(abs, otypes=[object])(r["Bint"])
    S = exact.exact_int_matmul(absA, absB)
    assert all(v <= (P - 1) // 2 for v in S.ravel())


def test_non_finite_rows_and_columns_give_nan():
    A, B = operand_pair(5, 4, 6, 0.5, 9)
    A[1, 2] = np.inf
    B[3, 0] = np.nan
    r = scheme.emulate(A, B, md.best_coprime_set(14), "W")
    C = r["C"]
    assert np.all(np.isnan(C[1, :])) and np.all(np.isnan(C[:, 0]))
    mask = np.ones_like(C, dtype=bool)
    mask[1, :] = False
    mask[:, 0] = False
    assert np.all(np.isfinite(C[mask]))


def test_config1_accuracy_modes():
    """256 cubed, phi = 0.5, fourteen moduli: mode W keeps 50/51 bits and
    misses 2**-50; mode G meets it (expected from the scaled-error
    analysis; the full exact metric over every entry)."""
    A, B = operand_pair(256, 256, 256, 0.5, 0)
    ms = md.best_coprime_set(14)
    rW = scheme.emulate(A, B, ms, "W", keep=False)
    rG = scheme.emulate(A, B, ms, "G", keep=False)
    assert rW["bits"] == (51, 50)
    eW = exact.scaled_error(rW["C"], A, B)
    eG = exact.scaled_error(rG["C"], A, B)
    assert eW > 2.0 ** -50 and eG <= 2.0 ** -50
