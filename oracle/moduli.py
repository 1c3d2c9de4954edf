"""Modulus sets, CRT window and exactness caps (oracle; test infrastructure).

Pins (``tests/test_oracle_moduli.py``): brute-force search over all subsets
on small limits for ``best_coprime_set``; the paper's printed values
r_max(1) = 362 under INT32 and 32 under FP32 at K = 2**14 (Sec. IV-C,
Example "equivalence"), K_max = 151,647 for sixteen moduli up to 239 and
131,071 for moduli up to 256 (Sec. IV-C), and the counting bound Q >= 16
for INT8 at K = 2**14 (Example "INT8", Sec. III-F).

Definitions
-----------
* A configuration's moduli are pairwise coprime (Sec. III-A); P is their
  product.
* CRT window (Sec. III-C, eq. "ov-crtgen"): P > 2 K B_A B_B, where B_A and
  B_B bound the magnitudes of the integer operands.
* Accumulator exactness (eq. "ov-accgen"): K * sum_G rho_A rho_B <= Lambda,
  Lambda = 2**31 - 1 for INT32 and 2**24 for FP32 (Sec. III-C).
* Caps (eq. "caps"): kappa_rec = (P - 1) / (2 B_A B_B),
  kappa_acc = Lambda / max accumulator sum; K_max = min of their floors.
* r_max(l) = floor(sqrt(Lambda / (l K))) (eq. "rmax").
* Counting bound (Sec. III-F): Q >= log2(2 K B_A B_B + 1) / log2 |S|.
"""
from __future__ import annotations

import math
from math import gcd, isqrt

__all__ = ["LAMBDA_INT32", "LAMBDA_FP32", "product", "pairwise_coprime",
           "best_coprime_set", "crt_window_ok", "kappa_rec", "kappa_acc_int8",
           "k_max_int8", "r_max", "counting_bound", "balanced_radius",
           "PAPER_INT8_239_SET", "log2_product"]

LAMBDA_INT32 = 2 ** 31 - 1
LAMBDA_FP32 = 2 ** 24

# A sixteen-modulus INT8 set with every modulus at most 239 (Sec. IV-C keeps
# its moduli up to 239 for a radius of 119). The paper does not print its
# set; this one is the largest-product pairwise-coprime set of sixteen
# moduli in [2, 239], the output of ``best_coprime_set(16, 239)``, written
# out so tests can pin that search against it.
PAPER_INT8_239_SET = (239, 237, 236, 235, 233, 229, 227, 223, 221, 217, 211,
                      209, 199, 197, 193, 191)


def product(ms) -> int:
    p = 1
    for m in ms:
        p *= int(m)
    return p


def pairwise_coprime(ms) -> bool:
    ms = [int(m) for m in ms]
    return all(gcd(a, b) == 1 for i, a in enumerate(ms) for b in ms[i + 1:])


def _prime_factors(n: int):
    out, p = [], 2
    while p * p <= n:
        if n % p == 0:
            out.append(p)
            while n % p == 0:
                n //= p
        p += 1
    if n > 1:
        out.append(n)
    return out


def best_coprime_set(count: int, limit: int = 256, lower: int = 2):
    """Pairwise-coprime set of ``count`` integers in ``[lower, limit]`` with
    the largest product; ties go to the set whose descending tuple is
    lexicographically largest. Returned sorted descending.

    Every integer up to ``limit`` has at most one prime factor above
    ``sqrt(limit)``. A dynamic program therefore tracks which small primes
    (at most ``sqrt(limit)``) are used, as a bit mask, and the number of
    members, and takes at most one member per large prime. Comparisons are
    on exact integer products.
    """
    if count < 0:
        raise ValueError("count must be non-negative")
    small = [p for p in range(2, isqrt(limit) + 1) if all(p % q for q in range(2, p))]
    bit = {p: 1 << i for i, p in enumerate(small)}
    groups = {}  # key: large prime (or None for small-smooth) -> list of (m, mask)
    for m in range(max(2, lower), limit + 1):
        mask, large = 0, None
        for p in _prime_factors(m):
            if p in bit:
                mask |= bit[p]
            else:
                large = p
        groups.setdefault(large, []).append((m, mask))
    # state: (mask, size) -> (product, members tuple sorted descending)
    best = {(0, 0): (1, ())}

    def better(a, b):
        return b is None or (a[0], a[1]) > (b[0], b[1])

    def add(state_map, key, val):
        if better(val, state_map.get(key)):
            state_map[key] = val

    # members without a large prime may be combined freely if their masks
    # are disjoint: each is its own 0/1 item.
    items = [[it] for it in groups.get(None, [])]
    # members sharing a large prime: at most one of them.
    items += [groups[k] for k in sorted(k for k in groups if k is not None)]
    for group in items:
        nxt = dict(best)
        for (mask, size), (prod, mem) in best.items():
            if size >= count:
                continue
            for m, mm in group:
                if mask & mm:
                    continue
                val = (prod * m, tuple(sorted(mem + (m,), reverse=True)))
                add(nxt, (mask | mm, size + 1), val)
        best = nxt
    cands = [v for (mask, size), v in best.items() if size == count]
    if not cands:
        raise ValueError("no pairwise-coprime set of that size")
    winner = None
    for v in cands:
        if better(v, winner):
            winner = v
    return list(winner[1])


def crt_window_ok(P: int, K: int, BA: int, BB: int) -> bool:
    """CRT window (eq. "ov-crtgen"): P > 2 K B_A B_B."""
    return P > 2 * K * BA * BB


def kappa_rec(P: int, BA: int, BB: int) -> int:
    """floor((P - 1) / (2 B_A B_B)) (eq. "caps")."""
    return (P - 1) // (2 * BA * BB)


def balanced_radius(m: int) -> int:
    """Largest magnitude of a residue modulo m taken nearest zero: the
    representatives are [-floor(m/2), ceil(m/2) - 1], so the radius is
    floor(m/2)."""
    return m // 2


def kappa_acc_int8(moduli) -> int:
    """floor(Lambda / max_m r_m**2) with one INT8 GEMM per modulus and
    Lambda = 2**31 - 1 (eqs. "ov-accgen", "caps")."""
    r = max(balanced_radius(int(m)) for m in moduli)
    return LAMBDA_INT32 // (r * r)


def k_max_int8(moduli, BA: int = 2 ** 53 - 1, BB: int = 2 ** 53 - 1) -> int:
    """K_max = min(floor(kappa_rec), floor(kappa_acc)) (Sec. III-C)."""
    return min(kappa_rec(product(moduli), BA, BB), kappa_acc_int8(moduli))


def r_max(lam: int, limbs: int, K: int) -> int:
    """r_max(l) = floor(sqrt(Lambda / (l K))) (eq. "rmax"), exactly."""
    return isqrt(lam // (limbs * K))


def counting_bound(K: int, BA: int, BB: int, alphabet_size: int) -> int:
    """Least integer Q with Q >= log2(2 K B_A B_B + 1) / log2|S| (Sec. III-F),
    decided exactly: the least Q with |S|**Q >= 2 K B_A B_B + 1."""
    need = 2 * K * BA * BB + 1
    q, acc = 0, 1
    while acc < need:
        acc *= alphabet_size
        q += 1
    return q


def log2_product(ms) -> float:
    return sum(math.log2(int(m)) for m in ms)
