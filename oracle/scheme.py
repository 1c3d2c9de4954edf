"""The residue (Ozaki II) scheme with INT8 channels, step by step.

Oracle; test infrastructure only. Pins (``tests/test_oracle_scheme.py``):
brute-force residues and Python ``%``; CRT round trips at the window edges
+-(P-1)/2 and at random points; bitwise equality of the CRT path with the
plain definition RN(A'B' 2**-(s+t)) computed by an exact integer product
that never touches a residue; independence of C from the modulus set at
fixed kept bits (Sec. II-A: accuracy is the same however the exact integer
product is formed); exact integer products returned unchanged when the
operands are small integers; the entrywise error bound of Sec. VIII-E.

Steps (Sec. II-A eq. "convert", Sec. II-B, Sec. III-C, Sec. V-A)
----------------------------------------------------------------
1. Exponents: e_i with 2**(e_i - 1) <= max_h |a_ih| < 2**e_i per row of A
   (f_j per column of B); a row or column of zeros is marked and its
   shift is 0 (the paper's mu = 1).
2. Kept bits beta_A, beta_B. The paper keeps 53 bits ("F53": mu is the
   largest power of two with every scaled entry below 2**53). Reading for
   the moduli-count knob ("W", the style the paper attributes to prior
   variants, Sec. VIII-C): w = floor(log2((P-1)/(2K))), beta_A = ceil(w/2),
   beta_B = floor(w/2), so K (2**beta_A - 1)(2**beta_B - 1) < K 2**w
   <= (P-1)/2 and the CRT window holds for any data. Reading "G"
   (bound-adaptive, one extra INT8 product): see ``bound_shifts``.
3. Truncation: A' = trunc(a * 2**s_i) with s_i = beta_A - e_i (eq.
   "convert"); |A'| < 2**beta_A.
4. Balanced residues modulo m, nearest zero, ties to -m/2 so that m = 256
   fits INT8 (Sec. II-B; Sec. V-D stores them in two's complement).
5. Residue GEMM W = R_A R_B exact (|W| <= K r_A r_B <= 2**31 - 1), and
   Z = W mod m in [0, m) (Sec. III-A: sum_k lambda_k W_k == A'B' mod m).
6. CRT: X == Z_l mod m_l, X in [0, P), balanced to X - P when X > (P-1)/2
   (Sec. II-B; the window is strict so the tie is unreachable).
7. One rounding: C_ij = RN(X_ij * 2**-(s_i + t_j)) (Sec. II-A, Sec. V-D).

Non-finite input (the paper is silent): every entry of C in a row of A or
column of B holding a NaN or an infinity is NaN; those rows and columns
are otherwise treated as zero rows and columns (shift 0, zero residues, and
no contribution to the bound product of reading "G").
"""
from __future__ import annotations

import numpy as np

from . import exact
from .moduli import product

__all__ = ["frexp_exponents", "kept_bits", "shifts_from_bits", "truncate",
           "balanced_residues", "residue_gemm", "crt_balanced",
           "round_scaled", "emulate", "definition_product", "bound_planes",
           "bound_shifts", "BETA_CAP"]

BETA_CAP = 127


def frexp_exponents(X: np.ndarray, axis: int):
    """(e, nonzero, finite): frexp exponent of the largest magnitude along
    ``axis`` (axis=1: rows of A; axis=0: columns of B)."""
    X = np.asarray(X, dtype=np.float64)
    finite = np.all(np.isfinite(X), axis=axis)
    Xf = np.where(np.isfinite(X), X, 0.0)
    amax = np.max(np.abs(Xf), axis=axis) if X.shape[axis] > 0 else \
        np.zeros(X.shape[1 - axis])
    _, e = np.frexp(amax)
    return e.astype(np.int64), amax > 0, finite


def kept_bits(mode: str, P: int, K: int):
    """(beta_A, beta_B) for modes "F53" and "W" (module header, step 2)."""
    if mode == "F53":
        return 53, 53
    if mode == "W":
        if K < 1:
            K = 1
        q = (P - 1) // (2 * K)
        if q < 1:
            raise ValueError("modulus product too small for K")
        w = q.bit_length() - 1  # floor(log2((P-1)/(2K)))
        return min(BETA_CAP, (w + 1) // 2), min(BETA_CAP, w // 2)
    raise ValueError("unknown mode " + repr(mode))


def shifts_from_bits(e: np.ndarray, nonzero: np.ndarray, beta) -> np.ndarray:
    """s = beta - e for a nonzero row or column, 0 for a zero one."""
    beta = np.broadcast_to(np.asarray(beta, dtype=np.int64), e.shape)
    return np.where(nonzero, beta - e, 0).astype(np.int64)


def truncate(X: np.ndarray, s: np.ndarray, axis: int):
    """trunc(X * 2**s) elementwise, s per row (axis=1) or column (axis=0).

    ``numpy.ldexp`` scales by a power of two exactly (the result lies below
    2**beta <= 2**127, far from overflow, and a result that underflows is
    below 1 and truncates to 0 either way), and ``numpy.trunc`` rounds
    toward zero. The integers are returned as an object array of Python
    ints (exact for any beta), or as int64 when every value is below 2**62.
    """
    X = np.where(np.isfinite(X), X, 0.0)
    sh = s[:, None] if axis == 1 else s[None, :]
    T = np.trunc(np.ldexp(X, sh))
    if T.size == 0 or np.max(np.abs(T)) < 2.0 ** 62:
        return T.astype(np.int64)  # every value is an integer below 2**62
    return exact.to_object_ints(T)


def balanced_residues(Xint: np.ndarray, m: int) -> np.ndarray:
    """Residues of integer matrix Xint modulo m in [-floor(m/2), ceil(m/2)-1],
    as int64. Python's % returns values in [0, m) for m > 0."""
    if Xint.dtype == np.int64:
        r = np.mod(Xint, m)
    else:
        r = np.vectorize(lambda v: int(v) % m, otypes=[np.int64])(Xint) \
            if Xint.size else np.zeros(Xint.shape, dtype=np.int64)
    half = (m + 1) // 2
    return np.where(r >= half, r - m, r).astype(np.int64)


def residue_gemm(RA: np.ndarray, RB: np.ndarray, m: int, blas: bool = False):
    """(W, Z): the exact product of residue planes and Z = W mod m.

    int64 matmul is exact for |W| < 2**63; with ``blas`` the product goes
    through FP64 BLAS, exact because every partial sum is an integer of
    magnitude at most K (m/2)**2 < 2**53 (checked)."""
    K = RA.shape[1]
    if K * (m // 2) ** 2 >= 2 ** 53:
        raise ValueError("FP64 sums would not be exact")
    if blas:
        W = (RA.astype(np.float64) @ RB.astype(np.float64)).astype(np.int64)
    else:
        W = RA.astype(np.int64) @ RB.astype(np.int64)
    return W, np.mod(W, m).astype(np.int64)


def crt_balanced(Z: np.ndarray, moduli) -> np.ndarray:
    """X with X == Z[l] (mod m_l) for every l, balanced into
    [-(P-1)/2, (P-1)/2] (textbook CRT: X = sum_l ((Z_l y_l) mod m_l) M_l
    mod P with M_l = P / m_l and y_l = M_l**-1 mod m_l)."""
    P = product(moduli)
    shape = Z.shape[1:]
    X = np.zeros(shape, dtype=object)
    X[...] = 0
    for l, m in enumerate(moduli):
        m = int(m)
        Ml = P // m
        yl = pow(Ml % m, -1, m)
        zl = Z[l].astype(object)
        X = X + ((zl * yl) % m) * Ml
    X = X % P
    half = (P - 1) // 2
    return np.where(X > half, X - P, X)


def round_scaled(X: np.ndarray, s: np.ndarray, t: np.ndarray) -> np.ndarray:
    """C_ij = RN(X_ij * 2**-(s_i + t_j)), one rounding."""
    C = np.empty(X.shape, dtype=np.float64)
    for i in range(X.shape[0]):
        for j in range(X.shape[1]):
            C[i, j] = exact.round_ratio_to_double(int(X[i, j]), int(s[i]) + int(t[j]))
    return C


def bound_planes(X: np.ndarray, e: np.ndarray, axis: int) -> np.ndarray:
    """Reading "G", first step: abar = ceil(|x| * 2**(6 - e)) per row
    (axis=1) or column (axis=0), an integer in [0, 64] because
    |x| < 2**e. Non-finite entries count as zero. ``numpy.ldexp`` is exact
    unless its result underflows to 0, which only happens for a nonzero x
    whose exact scaled value lies in (0, 1): its ceiling is 1."""
    X = np.where(np.isfinite(X), X, 0.0)
    sh = (6 - e)[:, None] if axis == 1 else (6 - e)[None, :]
    V = np.ldexp(np.abs(X), sh)
    out = np.ceil(V).astype(np.int64)
    out[(V == 0) & (X != 0)] = 1
    return out


def bound_shifts(A, B, P: int):
    """Reading "G" (bound-adaptive kept bits; the paper only mentions a
    scaling set from the modulus product and one more INT8 product, in its
    comparison with GEMMul8, Sec. VI-D).

    Gbar = abar @ bbar is exact (entries <= K * 2**12). With L =
    floor(log2((P-1)/2)) and c(g) = ceil(log2 g):
        sigma_i = floor((L + 12 - c(max_j Gbar_ij)) / 2),
        tau_j   = floor((L + 12 - c(max_i Gbar_ij)) / 2),
    each capped at BETA_CAP (also when the maximum is 0). Then
    sum_h |A'_ih||B'_hj| <= 2**(sigma_i + tau_j - 12) Gbar_ij <= 2**L, so
    the CRT window holds entry by entry. Returns
    (sigma, tau, abar, bbar, Gbar)."""
    eA, nzA, _ = frexp_exponents(A, 1)
    eB, nzB, _ = frexp_exponents(B, 0)
    abar = bound_planes(A, eA, 1)
    bbar = bound_planes(B, eB, 0)
    G = abar @ bbar
    L = ((P - 1) // 2).bit_length() - 1

    def side(gmax):
        out = np.empty(gmax.shape, dtype=np.int64)
        for idx, g in enumerate(gmax):
            g = int(g)
            if g <= 0:
                out[idx] = BETA_CAP
            else:
                c = (g - 1).bit_length()  # ceil(log2 g)
                out[idx] = min(BETA_CAP, (L + 12 - c) // 2)
        return out

    gmax_r = G.max(axis=1) if G.shape[1] else np.zeros(G.shape[0], np.int64)
    gmax_c = G.max(axis=0) if G.shape[0] else np.zeros(G.shape[1], np.int64)
    return side(gmax_r), side(gmax_c), abar, bbar, G


def _finite_parts(A, B):
    """(A0, B0, finA, finB): rows of A and columns of B holding a NaN or an
    infinity replaced by zeros (the reading for non-finite input)."""
    finA = np.all(np.isfinite(A), axis=1)
    finB = np.all(np.isfinite(B), axis=0)
    A0 = np.where(finA[:, None], A, 0.0)
    B0 = np.where(finB[None, :], B, 0.0)
    return A0, B0, finA, finB


def _shifts(A, B, moduli, mode):
    K = A.shape[1]
    P = product(moduli)
    A, B, finA, finB = _finite_parts(A, B)
    eA, nzA, _ = frexp_exponents(A, 1)
    eB, nzB, _ = frexp_exponents(B, 0)
    if mode == "G":
        sig, tau, _, _, _ = bound_shifts(A, B, P)
        s = shifts_from_bits(eA, nzA, sig)
        t = shifts_from_bits(eB, nzB, tau)
        bits = (sig, tau)
    else:
        bA, bB = kept_bits(mode, P, K)
        if mode == "F53" and 2 * K * (2 ** bA - 1) * (2 ** bB - 1) >= P:
            raise ValueError("K exceeds kappa_rec for this modulus set")
        s = shifts_from_bits(eA, nzA, bA)
        t = shifts_from_bits(eB, nzB, bB)
        bits = (bA, bB)
    return s, t, finA, finB, bits


def emulate(A: np.ndarray, B: np.ndarray, moduli, mode: str = "W",
            blas: bool = False, keep: bool = True):
    """Emulated C = A B through INT8 residue channels.

    Returns a dict with the intermediates: ``s``, ``t`` (shifts), ``bits``,
    ``RA``/``RB`` (residue planes, lists of int64 arrays, RB as k x n),
    ``Z`` (uint8 or int64 residues of A'B'), ``X`` (balanced CRT result)
    and ``C``."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    M, K = A.shape
    N = B.shape[1]
    s, t, finA, finB, bits = _shifts(A, B, moduli, mode)
    A, B, _, _ = _finite_parts(A, B)
    Ai = truncate(A, s, 1)
    Bi = truncate(B, t, 0)
    RA, RB, Z = [], [], np.zeros((len(moduli), M, N), dtype=np.int64)
    for l, m in enumerate(moduli):
        ra = balanced_residues(Ai, int(m))
        rb = balanced_residues(Bi, int(m))
        _, Z[l] = residue_gemm(ra, rb, int(m), blas=blas)
        if keep:
            RA.append(ra)
            RB.append(rb)
    X = crt_balanced(Z, moduli)
    C = round_scaled(X, s, t)
    bad = (~finA)[:, None] | (~finB)[None, :]
    C[bad] = np.nan
    return {"s": s, "t": t, "bits": bits, "RA": RA, "RB": RB, "Z": Z, "X": X,
            "C": C, "Aint": Ai, "Bint": Bi}


def definition_product(A: np.ndarray, B: np.ndarray, moduli, mode: str = "W"):
    """The plain definition C = RN(A'B' 2**-(s+t)) with A'B' formed by an
    exact integer product (no residues, no CRT). Used to pin ``emulate``."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    s, t, finA, finB, _ = _shifts(A, B, moduli, mode)
    A, B, _, _ = _finite_parts(A, B)
    X = exact.exact_int_matmul(truncate(A, s, 1), truncate(B, t, 0))
    C = round_scaled(X, s, t)
    bad = (~finA)[:, None] | (~finB)[None, :]
    C[bad] = np.nan
    return C
