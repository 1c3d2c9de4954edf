"""Backward products of an emulated Y = X W that reuse the forward's
cached shifts and residue planes (autograd through the emulation).

Oracle; test infrastructure only. The paper treats a single product; this
module writes out the reading used for training, where the two backward
products dX = dY W^T and dW = X^T dY are emulated with the same scheme and
the forward's truncated operands X', W' (equivalently their residues) are
reused instead of being scaled and reduced again. Pins
(``tests/test_oracle_backward.py``): the residue path equals the exact
integer product of the same truncated operands; small-integer operands give
the exact integer gradients (so a dropped fold, a sign error in a shift or
a transposed operand fails); the entrywise truncation error bound against
the exact product dY W^T (and X^T dY); a finite-difference check of a
one-layer loss; non-finite propagation.

Forward (shapes: X m x k, W k x n, Y m x n)
-------------------------------------------
Kept bits are chosen at K* = max(m, n, k), the largest inner dimension of
the three products, so the cached bits of X' and W' fit both backward
windows: beta_X = ceil(w(K*)/2), beta_W = floor(w(K*)/2) with
w(K) = floor(log2((P-1)/(2K))) (reading "W"), or 53 and 53 (reading "F53",
valid when the window holds at K*). s_i = beta_X - e_i (rows of X),
t_j = beta_W - f_j (columns of W), X' = trunc(X 2**s), W' = trunc(W 2**t),
Y = RN(X'W' 2**-(s+t)) as in ``scheme.emulate``.

dX = dY W^T (inner dimension n)
-------------------------------
W = W' diag(2**-t) up to truncation, so dY W^T ~ (dY diag(2**-t)) W'^T.
The fold dY'' = dY diag(2**-t) is a power-of-two scaling per column, kept
exact (never rounded to a double): the row exponent of dY'' is
e''_i = max_j (e(dY_ij) - t_j) over nonzero entries. dY'' keeps
beta'' = w(n) - beta_W bits ("W"; 53 for "F53"), so that
n (2**beta'' - 1)(2**beta_W - 1) < (P-1)/2: s''_i = beta'' - e''_i and
D_ij = trunc(dY_ij 2**(s''_i - t_j)). Then dX_ih = RN((D W'^T)_ih 2**-s''_i),
the integer product formed from residues of D and the cached residues of
W' (transposed) and reconstructed by the CRT.

dW = X^T dY (inner dimension m)
-------------------------------
Symmetric: the fold dY''' = diag(2**-s) dY per row; column exponents
f'''_j = max_i (e(dY_ij) - s_i); beta''' = w(m) - beta_X;
t'''_j = beta''' - f'''_j; E_ij = trunc(dY_ij 2**(t'''_j - s_i));
dW_hj = RN((X'^T E)_hj 2**-t'''_j).

Non-finite values (reading): a row of dY holding a NaN or an infinity, or
any column of W that held one in the forward (a NaN column of dY''), makes
the rows of dX it touches NaN (all rows in the second case); likewise a
column of dY, or any row of X that held one, for the columns of dW.
"""
from __future__ import annotations

import numpy as np

from . import exact, scheme
from .moduli import product

__all__ = ["cache_bits", "forward_cached", "backward_bits", "fold_shifts",
           "fold_truncate", "backward_dx", "backward_dw"]


def cache_bits(mode: str, P: int, m: int, n: int, k: int, kstar=None):
    """(beta_X, beta_W) of the cached forward: kept bits at K* = max(m, n, k)
    (``kstar`` gives K* of a whole problem when rows or columns of it are
    sampled)."""
    kstar = max(m, n, k, 1) if kstar is None else kstar
    bx, bw = scheme.kept_bits(mode, P, kstar)
    if mode == "F53" and 2 * kstar * (2 ** bx - 1) * (2 ** bw - 1) >= P:
        raise ValueError("max(m, n, k) exceeds kappa_rec for this modulus set")
    return bx, bw


def backward_bits(mode: str, P: int, inner: int, cached_bits: int) -> int:
    """Kept bits of the fresh operand dY of a backward product with inner
    dimension ``inner`` against cached bits ``cached_bits``."""
    if mode == "F53":
        return 53
    inner = max(inner, 1)
    q = (P - 1) // (2 * inner)
    w = q.bit_length() - 1
    beta = min(scheme.BETA_CAP, w - cached_bits)
    if beta < 1:
        raise ValueError("no bits left for dY at this inner dimension")
    return beta


def forward_cached(X, W, moduli, mode: str = "W", kstar=None, blas: bool = False):
    """Forward with kept bits at max(m, n, k); returns the cache the
    backward needs: shifts s, t, truncated X', W', their residue planes
    (RX[l]: m x k, RW[l]: k x n), the finite masks, the bits and Y.

    Rows of X and columns of W are scaled independently, so a sample of
    rows of X (columns of W) with ``kstar`` set to the whole problem's K*
    gives exactly those rows (columns) of the whole problem's cache and Y.
    ``blas`` forms the residue products through FP64 BLAS (exact, see
    ``scheme.residue_gemm``)."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    m, k = X.shape
    n = W.shape[1]
    P = product(moduli)
    bx, bw = cache_bits(mode, P, m, n, k, kstar)
    finX = np.all(np.isfinite(X), axis=1)
    finW = np.all(np.isfinite(W), axis=0)
    X0 = np.where(finX[:, None], X, 0.0)
    W0 = np.where(finW[None, :], W, 0.0)
    eX, nzX, _ = scheme.frexp_exponents(X0, 1)
    eW, nzW, _ = scheme.frexp_exponents(W0, 0)
    s = scheme.shifts_from_bits(eX, nzX, bx)
    t = scheme.shifts_from_bits(eW, nzW, bw)
    Xi = scheme.truncate(X0, s, 1)
    Wi = scheme.truncate(W0, t, 0)
    RX = [scheme.balanced_residues(Xi, int(mm)) for mm in moduli]
    RW = [scheme.balanced_residues(Wi, int(mm)) for mm in moduli]
    Z = np.zeros((len(moduli), m, n), dtype=np.int64)
    for l, mm in enumerate(moduli):
        _, Z[l] = scheme.residue_gemm(RX[l], RW[l], int(mm), blas=blas)
    Y = scheme.round_scaled(scheme.crt_balanced(Z, moduli), s, t)
    Y[(~finX)[:, None] | (~finW)[None, :]] = np.nan
    return {"s": s, "t": t, "bits": (bx, bw), "Xint": Xi, "Wint": Wi, "RX": RX,
            "RW": RW, "finX": finX, "finW": finW, "Y": Y, "mode": mode,
            "moduli": list(moduli), "shape": (m, n, k), "blas": blas}


def fold_shifts(D, fold, beta: int, axis: int):
    """Shifts of D 2**-fold (fold along the inner index) keeping ``beta``
    bits: per row (axis=1, fold per column) or per column (axis=0, fold
    per row). Returns (shift, nonzero). The exponent of d 2**-f is
    e(d) - f exactly, and the exponent of a maximum is the maximum of the
    exponents."""
    D = np.asarray(D, dtype=np.float64)
    _, e = np.frexp(D)
    f = fold[None, :] if axis == 1 else fold[:, None]
    ee = np.where(D != 0, e.astype(np.int64) - f, np.iinfo(np.int64).min)
    emax = ee.max(axis=axis) if D.shape[axis] else \
        np.full(D.shape[1 - axis], np.iinfo(np.int64).min)
    nonzero = emax != np.iinfo(np.int64).min
    return scheme.shifts_from_bits(np.where(nonzero, emax, 0), nonzero, beta), nonzero


def fold_truncate(D, shift, fold, axis: int):
    """trunc(D_ij 2**(shift - fold)) exactly, shift per row and fold per
    column (axis=1) or the transpose roles (axis=0). The scaled values lie
    below 2**beta, and ``numpy.ldexp`` is exact short of underflow, where
    the value is below 1 and truncates to 0 either way."""
    D = np.asarray(D, dtype=np.float64)
    if axis == 1:
        sh = shift[:, None] - fold[None, :]
    else:
        sh = shift[None, :] - fold[:, None]
    T = np.trunc(np.ldexp(D, sh))
    if T.size == 0 or np.max(np.abs(T)) < 2.0 ** 62:
        return T.astype(np.int64)
    return exact.to_object_ints(T)


def _crt_round(Zs, moduli, s_rows, t_cols):
    return scheme.round_scaled(scheme.crt_balanced(Zs, moduli), s_rows, t_cols)


def backward_dx(dY, cache, residues: bool = True):
    """dX = dY W^T through the cached W' (module header). ``residues``
    False forms D W'^T by an exact integer product instead of residues and
    the CRT (the definition the residue path must reproduce). Rows of dX
    depend only on the same rows of dY, so a cache of sampled rows of X
    takes the same rows of dY."""
    dY = np.asarray(dY, dtype=np.float64)
    m, n, k = cache["shape"]
    moduli = cache["moduli"]
    P = product(moduli)
    bad_rows = ~np.all(np.isfinite(dY), axis=1) | (not np.all(cache["finW"]))
    D0 = np.where(bad_rows[:, None], 0.0, np.where(np.isfinite(dY), dY, 0.0))
    beta = backward_bits(cache["mode"], P, n, cache["bits"][1])
    s2, _ = fold_shifts(D0, cache["t"], beta, 1)
    D = fold_truncate(D0, s2, cache["t"], 1)
    zero = np.zeros(k, dtype=np.int64)
    if residues:
        Z = np.zeros((len(moduli), m, k), dtype=np.int64)
        for l, mm in enumerate(moduli):
            rd = scheme.balanced_residues(D, int(mm))
            _, Z[l] = scheme.residue_gemm(rd, cache["RW"][l].T, int(mm), blas=cache["blas"])
        dX = _crt_round(Z, moduli, s2, zero)
    else:
        Xp = exact.exact_int_matmul(D, np.ascontiguousarray(cache["Wint"].T))
        dX = scheme.round_scaled(Xp, s2, zero)
    dX[bad_rows, :] = np.nan
    return dX


def backward_dw(dY, cache, residues: bool = True):
    """dW = X^T dY through the cached X' (module header). Columns of dW
    depend only on the same columns of dY, so a cache of sampled columns
    of W takes the same columns of dY."""
    dY = np.asarray(dY, dtype=np.float64)
    m, n, k = cache["shape"]
    moduli = cache["moduli"]
    P = product(moduli)
    bad_cols = ~np.all(np.isfinite(dY), axis=0) | (not np.all(cache["finX"]))
    E0 = np.where(bad_cols[None, :], 0.0, np.where(np.isfinite(dY), dY, 0.0))
    beta = backward_bits(cache["mode"], P, m, cache["bits"][0])
    t3, _ = fold_shifts(E0, cache["s"], beta, 0)
    E = fold_truncate(E0, t3, cache["s"], 0)
    zero = np.zeros(k, dtype=np.int64)
    if residues:
        Z = np.zeros((len(moduli), k, n), dtype=np.int64)
        for l, mm in enumerate(moduli):
            re = scheme.balanced_residues(E, int(mm))
            _, Z[l] = scheme.residue_gemm(np.ascontiguousarray(cache["RX"][l].T), re, int(mm),
                                          blas=cache["blas"])
        dW = _crt_round(Z, moduli, zero, t3)
    else:
        Xp = exact.exact_int_matmul(np.ascontiguousarray(cache["Xint"].T), E)
        dW = scheme.round_scaled(Xp, zero, t3)
    dW[:, bad_cols] = np.nan
    return dW
