"""Configurations of limb channels for float alphabets: the pool of
admissible channels and the least-GEMM-count coprime selection.

Oracle; test infrastructure only. Pins (``tests/test_oracle_fp.py``): the
least GEMM counts Sec. IV prints in Table "moduli" for E4M3 at K = 2**12
(29) and 2**14 (30), and Sec. IV-A's account of the 2**14 configuration,
15 one-limb channels at one GEMM and 5 two-limb channels at three; E2M3
taking E4M3's configuration at 2**14 (Example "equivalence"); brute force
over all subsets of small pools; every channel's table checked against the
form identity (eq. "ov-form") and the caps.

Pool (Sec. III-D, reduced to two candidate forms)
-------------------------------------------------
Under FP32 accumulation (Lambda = 2**24) at slab length K_t, every stored
value must lie within r1 = floor(sqrt(Lambda / K_t)) (eq. "rmax" at one
product per accumulator), so the usable alphabet is S_r = S within r1. A
modulus m enters the pool with
* the one-limb form (rank 1) if S_r meets every class modulo m, else
* the two-limb Toom form at points {0, 1, inf} (rank 3) at the least base b
  in [2, 4 r1 + 1] for which the values c0 + b c1 with c0, c1 and c0 + c1
  all in S_r meet every class modulo m, and the reduce-then-combine
  epilogue bound max{2m, (m - 1) sum_k lbar_k} <= Lambda holds (eq.
  "ov-comrtc").
The paper's pool also holds schoolbook forms, Toom forms of three limbs,
the subset form and searched forms; this pool is a subset, so its least
counts can only be larger (equal at E4M3 for K = 2**12 and 2**14).

Selection (Sec. III-E, program "ov-reduced")
--------------------------------------------
Pairwise-coprime members of least total rank Q whose product exceeds the
target, or (for a given budget) of largest product within Q. Every member
is at most M, so it has at most one prime factor above tau = isqrt(M): a
dynamic program tracks the primes up to tau used (bit mask) and the rank
spent, and takes at most one member per prime above tau (the grouping of
the paper's steps 1-3, without its step-5 repair, which the grouping makes
unnecessary). Products are compared through L(m) = floor(2**32 log2 m),
computed by fixed-point squaring; a strictly larger sum replaces a state, so
ties keep the first member in the order: members without a large prime by
increasing m, then groups by increasing large prime, members inside a group
by increasing m; ranks by increasing value. The target test is exact (the
integer product against K * 2**107 or the requested bound).
"""
from __future__ import annotations

from math import gcd, isqrt

from . import alphabets
from . import forms

__all__ = ["LAMBDA_FP32", "fixed_log2", "radius_bound", "usable_alphabet", "pool",
           "select", "configuration", "Member"]

LAMBDA_FP32 = 2 ** 24
FRAC = 32  # fractional bits of L(m)


def fixed_log2(m: int) -> int:
    """L(m): log2(m) with 32 fraction bits by repeated squaring in 62-bit
    fixed point, truncating after each square (a definition both sides of
    the library compute identically; it is within a few units of the last
    place of floor(2**32 log2 m), far finer than the gaps between the
    logarithms of distinct products compared here). x holds m / 2**e in
    [1, 2) times 2**62; each square that reaches 2 contributes a 1 bit and
    is halved."""
    if m < 1:
        raise ValueError("m >= 1")
    e = m.bit_length() - 1
    x = (m << 62) >> e
    out = e
    for _ in range(FRAC):
        x = (x * x) >> 62
        out <<= 1
        if x >= (2 << 62):
            x >>= 1
            out |= 1
    return out


class Member(tuple):
    """(m, rank, base): base 0 for the one-limb form."""
    __slots__ = ()

    def __new__(cls, m, rank, base):
        return tuple.__new__(cls, (int(m), int(rank), int(base)))

    m = property(lambda s: s[0])
    rank = property(lambda s: s[1])
    base = property(lambda s: s[2])


def radius_bound(k_slab: int, lam: int = LAMBDA_FP32) -> int:
    return isqrt(lam // max(int(k_slab), 1))


def usable_alphabet(fmt: str, k_slab: int):
    r1 = radius_bound(k_slab)
    return [v for v in alphabets.alphabet(fmt) if abs(v) <= r1]


def _covers(values, m: int) -> bool:
    import numpy as np
    return np.unique(np.asarray(values, dtype=np.int64) % m).size == m


def pool(fmt: str, k_slab: int):
    """Admissible members (m, rank, base) by increasing m (module header)."""
    Sr = usable_alphabet(fmt, k_slab)
    Sset = set(Sr)
    r1 = radius_bound(k_slab)
    toom_vals = {}
    for b in range(2, 4 * r1 + 2):
        toom_vals[b] = sorted({c0 + b * c1 for c0 in Sr for c1 in Sr if (c0 + c1) in Sset})
    mmax = max(len(v) for v in toom_vals.values())
    out = []
    for m in range(2, mmax + 1):
        if _covers(Sr, m):
            out.append(Member(m, 1, 0))
            continue
        for b in range(2, 4 * r1 + 2):
            vals = toom_vals[b]
            if len(vals) < m or not _covers(vals, m):
                continue
            lbar = sum(l % m for l in forms.toom2_form(b).lam)
            if max(2 * m, (m - 1) * lbar) <= LAMBDA_FP32:
                out.append(Member(m, 3, b))
                break
    return out


def _factors(n: int):
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


def select(members, q_max: int, target: int | None = None):
    """Least-Q selection (target given: the product must exceed it) or the
    largest product within rank q_max (target None). Returns the chosen
    members sorted by decreasing m, or None if the target is not reached
    within q_max.

    State (q, mask): rank spent and small primes used; value: the largest
    sum of L(m) reaching it (numpy int64 arrays, one row per q). Items are
    processed in the order of the module header; an item's update reads the
    states before its group and replaces a state only by a strictly larger
    value, so inside a group the first member wins a tie."""
    import numpy as np
    if not members:
        return None
    M = max(mb.m for mb in members)
    tau = isqrt(M)
    small = [p for p in range(2, tau + 1) if all(p % d for d in range(2, isqrt(p) + 1))]
    bit = {p: 1 << i for i, p in enumerate(small)}
    free, groups = [], {}
    for mb in sorted(members, key=lambda x: x.m):
        mask, large = 0, None
        for f in _factors(mb.m):
            if f in bit:
                mask |= bit[f]
            else:
                large = f
        if large is None:
            free.append([(mb, mask)])
        else:
            groups.setdefault(large, []).append((mb, mask))
    items = free + [groups[p] for p in sorted(groups)]
    NM = 1 << len(small)
    NEG = np.iinfo(np.int64).min // 4
    best = np.full((q_max + 1, NM), NEG, dtype=np.int64)
    best[0, 0] = 0
    masks = np.arange(NM, dtype=np.int64)
    trail = []  # per item group: (group, choice), choice[q, mask] = gi << 20 | src, or -1
    for grp in items:
        new = best.copy()
        choice = np.full((q_max + 1, NM), -1, dtype=np.int32)
        for gi, (mb, mk) in enumerate(grp):
            L = fixed_log2(mb.m)
            src = masks[(masks & mk) == 0]
            dst = src | mk
            for q in range(0, q_max + 1 - mb.rank):
                v = best[q, src]
                cand = v + L
                upd = (v > NEG) & (cand > new[q + mb.rank, dst])
                if upd.any():
                    new[q + mb.rank, dst[upd]] = cand[upd]
                    choice[q + mb.rank, dst[upd]] = (gi << 20) | src[upd]
        trail.append((grp, choice))
        best = new

    def rebuild(q, mask):
        chosen = []
        for grp, choice in reversed(trail):
            hit = int(choice[q, mask])
            if hit >= 0:
                mb = grp[hit >> 20][0]
                chosen.append(mb)
                q -= mb.rank
                mask = hit & ((1 << 20) - 1)
        return sorted(chosen, key=lambda x: -x.m)

    def prod(ch):
        p = 1
        for mb in ch:
            p *= mb.m
        return p

    if target is None:
        flat = best.reshape(-1)
        idx = int(np.argmax(flat))  # first maximum: least q, then least mask
        return rebuild(idx // NM, idx % NM)
    lt = fixed_log2(target) if target >= 1 else 0
    slack = 64 * (len(members) + 1)
    for q in range(q_max + 1):
        row = best[q]
        order = sorted(np.nonzero(row >= lt - slack)[0].tolist(), key=lambda mk: (-int(row[mk]), mk))
        for mk in order:
            ch = rebuild(q, mk)
            if prod(ch) > target:
                return ch
    return None


def configuration(fmt: str, k_slab: int, q: int | None = None, window_k: int | None = None):
    """Channels for a format at slab length k_slab: the least-Q set with
    P > window_k * 2**107 (the F53 window, eq. "ov-crt") when window_k is
    given, else the largest-product set within q GEMMs."""
    mem = pool(fmt, k_slab)
    if window_k is not None:
        return select(mem, q if q is not None else 96, target=int(window_k) * 2 ** 107)
    return select(mem, q)


def pairwise_coprime(members) -> bool:
    ms = [mb.m for mb in members]
    return all(gcd(a, b) == 1 for i, a in enumerate(ms) for b in ms[i + 1:])
