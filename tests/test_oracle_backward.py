"""Pins for oracle/backward.py: the residue path against an exact integer
product of the same truncated operands, exact integer gradients for small
integer operands, the entrywise truncation error bound against the exact
gradient products, window tightness of the backward kept bits, and
non-finite propagation."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import backward as bw
from oracle import exact
from oracle import moduli as md
from workloads import integer_matrix, operand_pair, phi_matrix


def _triple(m, n, k, phi, seed):
    X, W = operand_pair(m, n, k, phi, seed)
    dY = phi_matrix(m, n, phi, seed + 7)
    return X, W, dY


@pytest.mark.parametrize("mode,nm,shape,phi", [
    ("W", 10, (9, 7, 5), 0.5), ("W", 14, (6, 11, 13), 2.0), ("F53", 16, (5, 8, 6), 1.0),
    ("W", 20, (7, 5, 9), 4.0)])
def test_residue_path_equals_definition(mode, nm, shape, phi):
    m, n, k = shape
    X, W, dY = _triple(m, n, k, phi, 3)
    c = bw.forward_cached(X, W, md.best_coprime_set(nm), mode)
    assert np.array_equal(bw.backward_dx(dY, c), bw.backward_dx(dY, c, residues=False))
    assert np.array_equal(bw.backward_dw(dY, c), bw.backward_dw(dY, c, residues=False))


@pytest.mark.parametrize("nm", [8, 14])
def test_integer_operands_give_exact_gradients(nm):
    m, n, k = 12, 9, 7
    X = integer_matrix(m, k, 200, 1)
    W = integer_matrix(k, n, 200, 2)
    dY = integer_matrix(m, n, 200, 3)
    c = bw.forward_cached(X, W, md.best_coprime_set(nm), "W")
    ref_y = X.astype(np.int64) @ W.astype(np.int64)
    ref_dx = dY.astype(np.int64) @ W.astype(np.int64).T
    ref_dw = X.astype(np.int64).T @ dY.astype(np.int64)
    assert np.array_equal(c["Y"], ref_y.astype(np.float64))
    assert np.array_equal(bw.backward_dx(dY, c), ref_dx.astype(np.float64))
    assert np.array_equal(bw.backward_dw(dY, c), ref_dw.astype(np.float64))


def _check_bound(G, A, B, fold_terms, trunc_scale):
    """|G - AB| <= fold_terms + trunc_scale + 2**-53 |G| entrywise, with
    both terms given as FP64 arrays (slack 2**-40 for their evaluation)."""
    Mc, E = exact.exact_product(A, B)
    for i in range(G.shape[0]):
        for j in range(G.shape[1]):
            err = abs(Fraction(float(G[i, j])) - Fraction(Mc[i, j]) * Fraction(2) ** E)
            bound = (Fraction(float(fold_terms[i, j])) + Fraction(float(trunc_scale[i, j]))) \
                * Fraction(1 + 2 ** -40) + abs(Fraction(float(G[i, j]))) * Fraction(2) ** -53
            assert err <= bound, (i, j)


@pytest.mark.parametrize("mode,nm,phi", [("W", 12, 0.5), ("W", 16, 4.0), ("F53", 16, 1.0)])
def test_entrywise_error_bound(mode, nm, phi):
    """With a_j = dY_ij 2**(s''_i - t_j) and b_j = W_hj 2**t_j, truncation
    toward zero gives |a_j b_j - D_ij W'_hj| < |a_j| + |b_j| (|b_j| only
    where column j of W is nonzero), so
    |dX_ih - (dY W^T)_ih| <= sum_j |dY_ij| 2**-t_j [W_:j != 0]
                             + 2**-s''_i sum_j |W_hj| 2**t_j + 2**-53 |dX_ih|;
    the same with the roles swapped for dW."""
    m, n, k = 8, 6, 5
    X, W, dY = _triple(m, n, k, phi, 5)
    ms = md.best_coprime_set(nm)
    c = bw.forward_cached(X, W, ms, mode)
    P = md.product(ms)
    t = c["t"].astype(np.float64)
    s = c["s"].astype(np.float64)
    # dX
    dX = bw.backward_dx(dY, c)
    beta = bw.backward_bits(mode, P, n, c["bits"][1])
    s2, _ = bw.fold_shifts(dY, c["t"], beta, 1)
    wnz = np.any(W != 0, axis=0)
    t1 = (np.abs(dY) * np.where(wnz, 2.0 ** -t, 0.0)[None, :]).sum(axis=1)[:, None] * np.ones((1, k))
    t2 = 2.0 ** -s2.astype(np.float64)[:, None] * (np.abs(W) * 2.0 ** t[None, :]).sum(axis=1)[None, :]
    _check_bound(dX, dY, np.ascontiguousarray(W.T), t1, t2)
    # dW
    dW = bw.backward_dw(dY, c)
    beta = bw.backward_bits(mode, P, m, c["bits"][0])
    t3, _ = bw.fold_shifts(dY, c["s"], beta, 0)
    xnz = np.any(X != 0, axis=1)
    u1 = np.ones((k, 1)) * (np.abs(dY) * np.where(xnz, 2.0 ** -s, 0.0)[:, None]).sum(axis=0)[None, :]
    u2 = (np.abs(X) * 2.0 ** s[:, None]).sum(axis=0)[:, None] * 2.0 ** -t3.astype(np.float64)[None, :]
    _check_bound(dW, np.ascontiguousarray(X.T), dY, u1, u2)


@pytest.mark.parametrize("nm,shape", [(12, (8, 300, 40)), (16, (500, 6, 30)), (9, (3, 4, 5)),
                                      (14, (8, 3000, 4)), (14, (5000, 7, 3))])
def test_backward_bits_fill_the_window(nm, shape):
    """inner (2**beta - 1)(2**cached - 1) <= (P-1)/2 holds, one more bit of
    dY would break inner 2**(beta + cached) <= (P-1)/2, and since the cache
    splits the bits at the largest inner dimension, the fresh operand never
    keeps fewer bits than the cached one (up to the odd bit X keeps)."""
    m, n, k = shape
    ms = md.best_coprime_set(nm)
    P = md.product(ms)
    bx, bwb = bw.cache_bits("W", P, m, n, k)
    for inner, cached, slack in ((n, bwb, 0), (m, bx, 1)):
        beta = bw.backward_bits("W", P, inner, cached)
        assert beta >= 1
        assert inner * (2 ** beta - 1) * (2 ** cached - 1) <= (P - 1) // 2
        assert inner * 2 ** (beta + 1 + cached) > (P - 1) // 2
        assert beta >= cached - slack
    assert k * (2 ** bx - 1) * (2 ** bwb - 1) <= (P - 1) // 2


def test_zero_rows_and_non_finite_propagation():
    m, n, k = 6, 5, 4
    X, W, dY = _triple(m, n, k, 0.5, 8)
    dY[2, :] = 0.0
    dY[4, 1] = np.nan
    ms = md.best_coprime_set(14)
    c = bw.forward_cached(X, W, ms, "W")
    dX = bw.backward_dx(dY, c)
    dW = bw.backward_dw(dY, c)
    assert np.all(dX[2] == 0.0)
    assert np.all(np.isnan(dX[4])) and np.all(np.isfinite(np.delete(dX, 4, axis=0)))
    assert np.all(np.isnan(dW[:, 1])) and np.all(np.isfinite(np.delete(dW, 1, axis=1)))
    # a non-finite column of W in the forward poisons every row of dX only
    W2 = W.copy()
    W2[1, 3] = np.inf
    c2 = bw.forward_cached(X, W2, ms, "W")
    dY2 = phi_matrix(m, n, 0.5, 9)
    assert np.all(np.isnan(bw.backward_dx(dY2, c2)))
    assert np.all(np.isfinite(bw.backward_dw(dY2, c2)))
