"""Integer alphabets of low-precision float formats (Sec. III-A).

Oracle; test infrastructure only. Pins (``tests/test_oracle_forms.py``):
E2M1 is {0, +-1, +-2, +-3, +-4, +-6, +-8, +-12} at e_S = 1 (Sec. III-A);
|S.S| = 37 over E2M1 (Example "decoders"); E2M3 and E4M3 hold 49 values
within radius 32 and E3M2 and E5M2 hold 33 (Sec. IV-A); E4M3 agrees with
E2M3 up to 60 and E5M2 with E3M2 up to 448 (Example "equivalence"); INT8
has 256 values.

A format's alphabet is its set of finite values times the least power of
two 2**e_S that makes them all integers. Values are enumerated from the
bit fields of each encoding: exponent width ``E``, mantissa width ``M``,
bias ``2**(E-1) - 1``; a zero exponent field is subnormal,
``(mant / 2**M) * 2**(1 - bias)``; otherwise ``(1 + mant / 2**M) *
2**(exp - bias)``. The encodings that are not finite numbers are dropped:
E4M3 (the "FN" variant) uses only exponent 15 with mantissa 7 as NaN and has
no infinities; E5M2 keeps IEEE infinities and NaNs at exponent 31; E2M3,
E3M2 and E2M1 have none.
"""
from __future__ import annotations

from fractions import Fraction

__all__ = ["FORMATS", "format_values", "alphabet", "alphabet_scale"]

# name: (exponent bits, mantissa bits, rule for non-finite encodings)
FORMATS = {
    "E4M3": (4, 3, "fn"),
    "E5M2": (5, 2, "ieee"),
    "E2M3": (2, 3, "none"),
    "E3M2": (3, 2, "none"),
    "E2M1": (2, 1, "none"),
}


def format_values(name: str):
    """Sorted list of the distinct finite values (Fractions) of a format."""
    if name == "INT8":
        return [Fraction(v) for v in range(-128, 128)]
    E, M, rule = FORMATS[name]
    bias = 2 ** (E - 1) - 1
    vals = set()
    for exp in range(2 ** E):
        for mant in range(2 ** M):
            if rule == "ieee" and exp == 2 ** E - 1:
                continue
            if rule == "fn" and exp == 2 ** E - 1 and mant == 2 ** M - 1:
                continue
            if exp == 0:
                mag = Fraction(mant, 2 ** M) * Fraction(2) ** (1 - bias)
            else:
                mag = (1 + Fraction(mant, 2 ** M)) * Fraction(2) ** (exp - bias)
            vals.add(mag)
            vals.add(-mag)
    return sorted(vals)


def alphabet_scale(name: str) -> int:
    """e_S: the least e with every finite value times 2**e an integer."""
    if name == "INT8":
        return 0
    e = 0
    while any((v * 2 ** e).denominator != 1 for v in format_values(name)):
        e += 1
    return e


def alphabet(name: str):
    """The integer alphabet S (sorted list of ints)."""
    e = alphabet_scale(name)
    return [int(v * 2 ** e) for v in format_values(name)]
