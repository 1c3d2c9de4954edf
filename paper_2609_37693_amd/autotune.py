"""Choice of the moduli count per problem for grouped products.

The accuracy of an emulated product in mode W is set by the bits each row
of A and column of B keeps, min(beta_A, beta_B), which grows with the
modulus product P and shrinks with K (w = floor(log2((P - 1) / (2K)))).
The scaled error max |C - AB| / (|A||B|) measured with the oracle on
U(-1/2, 1/2) exp(N(0, 1)) operands is about 2^(3.5 - min(beta_A, beta_B))
for K from 64 to 4096, so the default target of 55 kept bits meets
2^-50 with margin. For each problem the smallest count whose kept bits at
the problem's K reach the target is taken; plans are shared between
problems with the same count. The kept bits come from the library's own
plan (ozemu_plan_kept_bits), so the rule is the one the kernels apply.
"""
from __future__ import annotations

from . import Plan

__all__ = ["DEFAULT_TARGET_BITS", "moduli_for", "plans_for"]

DEFAULT_TARGET_BITS = 55
_PLANS = {}


def _plan(n: int, scaling: str = "W") -> Plan:
    key = (n, scaling)
    if key not in _PLANS:
        _PLANS[key] = Plan(num_moduli=n, scaling=scaling)
    return _PLANS[key]


def moduli_for(k: int, target_bits: int = DEFAULT_TARGET_BITS, lo: int = 2, hi: int = 32) -> int:
    """Smallest moduli count in [lo, hi] whose mode-W kept bits at inner
    dimension k are both at least target_bits (hi if none reaches it)."""
    k = max(int(k), 1)
    for n in range(lo, hi + 1):
        pl = _plan(n)
        try:
            ba, bb = pl.kept_bits(k)
        except Exception:  # k beyond this count's caps
            continue
        if min(ba, bb) >= target_bits:
            return n
    return hi


def plans_for(shapes, moduli: int | None = None, target_bits: int = DEFAULT_TARGET_BITS):
    """One plan per (m, n, k): the given moduli count for all, or the
    smallest count that meets target_bits at each problem's K."""
    if moduli is not None:
        pl = _plan(int(moduli))
        return [pl] * len(shapes)
    cache = {}
    out = []
    for _, _, k in shapes:
        if k not in cache:
            cache[k] = _plan(moduli_for(k, target_bits))
        out.append(cache[k])
    return out
