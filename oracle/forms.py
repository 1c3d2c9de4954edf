"""Limb channels, forms, encoding tables and the R>C epilogue.

Oracle; test infrastructure only. Pins (``tests/test_oracle_forms.py``):
Example 1 of Sec. III-B over E2M1 at base 13 (one limb covers [-4, 4], two
cover [-56, 56]; 58, 60, 64 reachable past the run and 57, 59, 61-63, 65
not; 5 = -8 + 13; class 57 modulo 115 stored as (-6, -4); radius 8; 13
values within radius 8 so m <= 169; gamma = 8 modulo 13, Fig. 2); the
schoolbook rank q(169, 13, 2) = 3 of eq. "qm" and OzII-FP4's 18 * 4 + 3 =
75 GEMMs (Sec. IV-B); the form identity of eq. "ov-form" checked over every
pair of classes for every form built here; the R>C epilogue against the
product reduced directly.

Definitions (Sec. III-A, III-B, III-C)
--------------------------------------
* A form of rank r modulo m: tables alpha_k, beta_k from classes to S and
  integer weights lambda_k with sum_k lambda_k alpha_k(t) beta_k(u) == t u
  (mod m) for all classes t, u (eq. "ov-form").
* A limb channel (m, b, l) stores a class as a tuple c of l limbs in S
  representing sum_i b**i c_i. Linear forms take plane k as a fixed integer
  combination p_k of the limbs (A side) and q_k (B side) with
  sum_k lambda_k p_k q_k^T == w w^T (mod m), w = (1, b, .., b**(l-1))
  (eq. "ov-linear").
* One-limb form (complete alphabet): p = q = (1), lambda = 1, rank 1.
* Toom form at two limbs, points {0, 1, inf}: p = q = (1, 0), (1, 1),
  (0, 1); since A(x)B(x) = T0 + T1 x + T2 x**2 with W0 = T0,
  W1 = T0 + T1 + T2, Winf = T2, the represented product
  T0 + b T1 + b**2 T2 equals (1 - b) W0 + b W1 + (b**2 - b) Winf.
* Schoolbook form: every limb pair (i, j) at weight b**(i+j); groups whose
  weight m divides are dropped, rank l**2 - sum n_g (eq. "qm").
* Encoding: each class is stored as a representing tuple whose plane
  values all lie in S, the one whose largest plane magnitude is least.
  The paper does not break ties; the reading used here takes, among those,
  the least sum of |limbs|, then the lexicographically least tuple
  (c_{l-1}, ..., c_0). The radius r_m is the largest plane magnitude over
  the m stored tuples.
* Epilogue, reduce-then-combine (eq. "ov-comrtc"): Z = (sum_k lbar_k
  (W_k mod m)) mod m, lbar_k = lambda_k mod m; exact in FP32 where
  max{2m, (m-1) sum lbar} <= 2**24. Slabs add residues: Z <- (Z + Z_s) mod m.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import product as iproduct

import numpy as np

__all__ = ["LinearForm", "one_limb_form", "toom2_form", "schoolbook_form",
           "schoolbook_rank", "encode_table", "channel_radius", "reach",
           "check_form_identity", "rtc_epilogue", "Channel", "make_channel",
           "channel_planes", "channel_residue"]


@dataclass
class LinearForm:
    """p[k], q[k]: integer limb combinations of plane k; lam[k]: weights."""
    limbs: int
    base: int
    p: list
    q: list
    lam: list
    kind: str = ""

    @property
    def rank(self) -> int:
        return len(self.lam)


def one_limb_form() -> LinearForm:
    return LinearForm(1, 1, [(1,)], [(1,)], [1], "one-limb")


def toom2_form(b: int) -> LinearForm:
    pts = [(1, 0), (1, 1), (0, 1)]
    return LinearForm(2, b, pts, pts, [1 - b, b, b * b - b], "toom2")


def schoolbook_form(m: int, b: int, limbs: int) -> LinearForm:
    p, q, lam = [], [], []
    for i in range(limbs):
        for j in range(limbs):
            if pow(b, i + j, m) == 0:
                continue  # group weight divisible by m: vanishes modulo m
            p.append(tuple(1 if x == i else 0 for x in range(limbs)))
            q.append(tuple(1 if x == j else 0 for x in range(limbs)))
            lam.append(b ** (i + j))
    return LinearForm(limbs, b, p, q, lam, "schoolbook")


def schoolbook_rank(m: int, b: int, limbs: int) -> int:
    """q(m, b, l) = l**2 - sum_{g : m | b**g} n_g (eq. "qm")."""
    n_g = {}
    for i in range(limbs):
        for j in range(limbs):
            n_g[i + j] = n_g.get(i + j, 0) + 1
    return limbs * limbs - sum(n for g, n in n_g.items() if pow(b, g, m) == 0)


def _planes_of(form: LinearForm, c, side="p"):
    combos = form.p if side == "p" else form.q
    return tuple(sum(pi * ci for pi, ci in zip(pk, c)) for pk in combos)


def encode_table(m: int, form: LinearForm, S, limb_radii=None):
    """Stored tuple for every class t in [0, m), or None if a class has no
    tuple whose A-side and B-side plane values all lie in S (the channel is
    then not admissible). Reading of the tie-break in the module header."""
    Sset = set(S)
    radii = limb_radii or [max(abs(v) for v in S)] * form.limbs
    limb_vals = [[v for v in S if abs(v) <= radii[i]] for i in range(form.limbs)]
    best = [None] * m
    for c in iproduct(*limb_vals):
        pa = _planes_of(form, c, "p")
        pb = _planes_of(form, c, "q")
        if not all(v in Sset for v in pa + pb):
            continue
        val = sum(ci * form.base ** i for i, ci in enumerate(c))
        cls = val % m
        key = (max(abs(v) for v in pa + pb), sum(abs(x) for x in c), tuple(reversed(c)))
        if best[cls] is None or key < best[cls][0]:
            best[cls] = (key, c)
    if any(b is None for b in best):
        return None
    return [b[1] for b in best]


def channel_radius(table, form: LinearForm) -> int:
    return max(max(abs(v) for v in _planes_of(form, c, "p") + _planes_of(form, c, "q"))
               for c in table)


def reach(S, b: int, limbs: int):
    """Set of integers sum_i b**i c_i with every c_i in S."""
    vals = {0}
    for i in range(limbs):
        vals = {v + (b ** i) * s for v in vals for s in S}
    return vals


def check_form_identity(m: int, form: LinearForm, table) -> bool:
    """eq. "ov-form" over every pair of classes (t, u)."""
    for t in range(m):
        ct = table[t]
        pa = _planes_of(form, ct, "p")
        for u in range(m):
            cu = table[u]
            pb = _planes_of(form, cu, "q")
            s = sum(l * x * y for l, x, y in zip(form.lam, pa, pb))
            if (s - t * u) % m:
                return False
    return True


def rtc_epilogue(Ws, lam, m: int) -> np.ndarray:
    """Z = (sum_k lbar_k (W_k mod m)) mod m (reduce-then-combine)."""
    Z = np.zeros(np.shape(Ws[0]), dtype=np.int64)
    for W, l in zip(Ws, lam):
        Z = Z + (l % m) * np.mod(np.asarray(W, dtype=np.int64), m)
    return np.mod(Z, m)


@dataclass
class Channel:
    m: int
    form: LinearForm
    table: list = field(repr=False)
    radius: int = 0


def make_channel(m: int, form: LinearForm, S):
    tab = encode_table(m, form, S)
    if tab is None:
        return None
    return Channel(m, form, tab, channel_radius(tab, form))


def channel_planes(Xint_mod_m: np.ndarray, ch: Channel, side: str = "p"):
    """Planes alpha_k(X) (side "p") or beta_k(X) (side "q") for classes in
    [0, m) given as an int64 array; returns a list of int64 arrays."""
    vals = np.array([_planes_of(ch.form, c, side) for c in ch.table], dtype=np.int64)
    return [vals[Xint_mod_m, k] for k in range(ch.form.rank)]


def channel_residue(Aclass, Bclass, ch: Channel, slab: int = 0):
    """Z = A'B' mod m through the channel's planes, exact products and the
    R>C epilogue, with the inner dimension in slabs of ``slab`` terms
    (0: one slab). Aclass (M x K), Bclass (K x N): classes in [0, m)."""
    K = Aclass.shape[1]
    slab = slab or max(K, 1)
    UA = channel_planes(Aclass, ch, "p")
    VB = channel_planes(Bclass, ch, "q")
    Z = np.zeros((Aclass.shape[0], Bclass.shape[1]), dtype=np.int64)
    for k0 in range(0, max(K, 1), slab):
        Ws = [U[:, k0:k0 + slab] @ V[k0:k0 + slab, :] for U, V in zip(UA, VB)]
        Z = np.mod(Z + rtc_epilogue(Ws, ch.form.lam, ch.m), ch.m)
    return Z
