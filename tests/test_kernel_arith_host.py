"""CPU checks of the integer and rounding identities that the HIP kernels
rely on, restated in exact integer arithmetic (no GPU, no kernel code):

* Reduce: the balanced residue t - m floor(t/m + 1/2) of t < 2^19 is the
  low byte of t - m (low 24 bits of the FP32 word fma(t, r, 1.5 2^23)),
  r = 1/m rounded strictly up to FP32, for every m <= 256 and every t.
* GEMM epilogue: for an INT32 accumulator w, q from fma(w, 1/m, 1.5 2^52)
  in FP64 (the low 32 bits of the result), the 24-bit multiply-add
  w + q24 (2^16 - m) and two packed 16-bit unsigned-min corrections give
  w mod m in [0, m), for every m <= 256 on the INT32 extremes, exact ties
  and a random sample of w.
* Reconstruct: rounding |X| = sum_k d_k 2^(40 k) (or 2^(30 k)) to FP64
  from its leading digits with a Fast2Sum remainder equals the correctly
  rounded value whenever the fast path accepts it (no exact tie of the
  53-bit rounding, result at or above 2^-1021)."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

C_MAGIC = 12582912  # 1.5 2^23


def _f32_parts(x):
    """(M, E) with x = M 2^E exactly, M a 24-bit integer (FP32 x > 0)."""
    fr, ex = math.frexp(float(np.float32(x)))
    return int(fr * 2 ** 24), ex - 24


def _rne_shift(num, s):
    """Round num / 2^s to the nearest integer, ties to even (numpy int64)."""
    q = num >> s
    rem = num - (q << s)
    half = np.int64(1) << (s - 1)
    up = (rem > half) | ((rem == half) & ((q & 1) == 1))
    return q + up


def _mul24(a, b):
    """v_mul_i32_i24: signed low 24 bits of each, low 32 bits of the product."""
    a24 = ((a & 0xFFFFFF) ^ 0x800000) - 0x800000
    b24 = ((b & 0xFFFFFF) ^ 0x800000) - 0x800000
    return (a24 * b24) & 0xFFFFFFFF


def _rcp_up(m):
    r = np.float32(1.0) / np.float32(m)
    if float(r) * m <= 1.0:
        r = np.nextafter(r, np.float32(1.0))
    return r


def test_reduce_residue_from_magic_fma_every_m_and_t():
    t = np.arange(1 << 19, dtype=np.int64)
    for m in range(2, 257):
        M, E = _f32_parts(_rcp_up(m))
        q = _rne_shift(t * M, -E)  # fma(t, r, 1.5 2^23) - 1.5 2^23, exactly
        low24 = (0x400000 + q) & 0xFFFFFF
        r32 = (t + _mul24(low24, -m)) & 0xFFFFFFFF
        want = t - m * ((2 * t + m) // (2 * m))
        assert np.array_equal(r32 & 0xFF, want & 0xFF), m
        assert want.min() >= -(m // 2) and want.max() <= (m + 1) // 2 - 1


def test_gemm_epilogue_mod_every_m_sampled_w():
    rng = np.random.default_rng(3)
    ws = [-2 ** 31, -2 ** 31 + 1, -1, 0, 1, 2 ** 31 - 1, -65536, 65535, 65536, -65537]
    ws += [int(v) for v in rng.integers(-2 ** 31, 2 ** 31, 400)]
    for m in range(2, 257):
        rcp64 = Fraction(1.0 / m)  # FP64 1/m, exactly
        # exact ties w / m = k + 1/2 in both signs
        wm = ws + [k * m + m // 2 for k in (-(2 ** 31) // m + 1, -3, 0, 5, (2 ** 31 - 1) // m - 1)
                   if m % 2 == 0]
        for w in wm:
            q = round(w * rcp64)  # fma(w, rcp64, 1.5 2^52) - 1.5 2^52: one rounding, ties to even
            q32 = q & 0xFFFFFFFF
            r = ((q32 & 0xFFFFFF) * (65536 - m) + (w & 0xFFFFFFFF)) & 0xFFFF
            v = min(r, (r + m) & 0xFFFF)
            v = min(v, (v - m) & 0xFFFF)
            assert v == w % m, (m, w)


def _exact_rn(X, sc):
    try:
        return float(Fraction(X) / Fraction(2) ** sc)
    except OverflowError:
        return math.inf


def _fast_round(X, sc, CB, KC):
    dg = [float((X >> (CB * k)) & ((1 << CB) - 1)) for k in range(KC)]
    a = b = c = 0.0
    j = -1
    for k in range(KC):
        if dg[k] != 0.0:
            j, a = k, dg[k]
            b = dg[k - 1] if k >= 1 else 0.0
            c = dg[k - 2] if k >= 2 else 0.0
    if j < 0:
        return None
    unit_f = float(1 << CB)
    low = a < 2.0 ** (53 - CB)
    top = a * unit_f + b if low else a
    nxt = c if low else b
    unit = CB * (j - 2 if low else j - 1)
    big = top * unit_f
    hi = big + nxt
    e1 = nxt - (hi - big)
    assert Fraction(big) + Fraction(nxt) - Fraction(hi) == Fraction(e1)  # Fast2Sum is exact
    eh = math.frexp(hi)[1]
    if abs(e1) == math.ldexp(1.0, eh - 54) or eh + unit - sc < -1020:
        return None
    try:
        return math.ldexp(hi, unit - sc)
    except OverflowError:
        return math.inf


@pytest.mark.parametrize("CB,KC,bits", [(40, 4, 137), (30, 7, 200)])
def test_reconstruct_fast_rounding_is_correct_rounding(CB, KC, bits):
    rnd = random.Random(CB)
    taken = 0
    for _ in range(20000):
        L = rnd.randint(1, bits)
        X = rnd.getrandbits(L) | (1 << (L - 1))
        kind = rnd.random()
        if L > 60 and kind < 0.3:  # exact ties and their neighbours
            p = L - 54
            X = (X >> (p + 1) << (p + 1)) | (1 << p)
            X += rnd.choice([0, 1, -1])
        sc = rnd.choice([rnd.randint(-200, 200), rnd.randint(L - 1100, L - 1000), 0])
        got = _fast_round(X, sc, CB, KC)
        if got is not None:
            taken += 1
            assert got == _exact_rn(X, sc), (X, sc)
    assert taken > 10000


def _to_mid(v, sh, neg):
    """The exact-form kernels' 96-bit signed digits of A' = +-v 2^sh:
    (A' + 0x80...80 mod 2^96) with each byte's top bit flipped."""
    M64, M32 = (1 << 64) - 1, (1 << 32) - 1
    lo = (v << sh) & M64
    hi = (v >> (64 - sh)) & M32 if sh > 0 else 0
    nlo = (-lo) & M64 if neg else lo
    nhi = ((~hi) + (1 if lo == 0 else 0)) & M32 if neg else hi
    y0 = (nlo + 0x8080808080808080) & M64
    y1 = (nhi + 0x80808080 + (1 if y0 < nlo else 0)) & M32
    words = [(y0 & M32) ^ 0x80808080, (y0 >> 32) ^ 0x80808080, y1 ^ 0x80808080]
    return [((w >> (8 * i)) & 0xFF) - 256 * (((w >> (8 * i)) & 0xFF) >= 128)
            for w in words for i in range(4)]


def test_reduce_96_bit_signed_digits_and_residue():
    """Twelve signed digits rebuild +-v 2^sh exactly for |A'| < 2^94, and
    three signed dot products on top of 2 km stay in [0, 2^19) and give the
    balanced residue through the magic-constant FMA, for every m <= 256."""
    rnd = random.Random(9)
    cases = [(1, 0, False), (1, 0, True), ((1 << 53) - 1, 41, False), ((1 << 53) - 1, 41, True),
             (1 << 52, 12, True), ((1 << 53) - 1, 11, True), (12345, 0, True)]
    cases += [(rnd.getrandbits(rnd.randint(1, 53)), rnd.randint(0, 41), rnd.random() < 0.5)
              for _ in range(300)]
    for m in range(2, 257):
        km = m * -(-(1 << 17) // m)
        wts = []
        for j in range(12):
            w = pow(2, 8 * j, m)
            wts.append(w - m if w >= (m + 1) // 2 else w)
        M, E = _f32_parts(_rcp_up(m))
        for v, sh, neg in cases:
            a = (-1 if neg else 1) * (v << sh)
            d = _to_mid(v, sh, neg)
            assert all(-128 <= x <= 127 for x in d)
            assert sum(x << (8 * i) for i, x in enumerate(d)) == a
            t = 2 * km + sum(x * w for x, w in zip(d, wts))
            assert 0 <= t < (1 << 19)
            q = int(_rne_shift(np.array([t * M], dtype=np.int64), -E)[0])
            r = (t + int(_mul24(np.array([(0x400000 + q) & 0xFFFFFF]), np.array([-m]))[0])) & 0xFF
            want = a - m * ((2 * a + m) // (2 * m))  # balanced residue of A'
            assert r == want & 0xFF, (m, v, sh, neg)
