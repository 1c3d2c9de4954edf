"""The residue scheme through limb channels of a float alphabet (FP8/FP6/FP4
matrix units with FP32 accumulation), step by step.

Oracle; test infrastructure only. Pins (``tests/test_oracle_fp.py``): the
result is bitwise the plain definition RN(A'B' 2**-(s+t)) at the same kept
bits (``scheme.definition_product``), whatever the channels, forms and slab
length (Sec. II-A: every exact configuration returns the same product);
slab lengths give identical residues; a configuration at the accumulator
bound K_t rho**2 = 2**24 stays exact.

Steps (Sec. V-A phases, Sec. III-A/III-C)
-----------------------------------------
1-3. Scale and truncate as in ``scheme`` (kept bits from the modulus product
     P of the channels: reading "W", or 53 bits, reading "F53").
4.   For each channel (m, form, base): classes A' mod m, B' mod m in
     [0, m); plane k of A holds alpha_k(class) and of B beta_k(class), read
     from the channel's table (``forms.encode_table`` over the alphabet
     within radius r1 = floor(sqrt(2**24 / K_t))).
5.   Per slab of K_t terms: W_k = U_k V_k, exact (|W_k| <= K_t r1**2 <=
     2**24, eq. "ov-accgen"); the slab's residue (sum_k lbar_k (W_k mod m))
     mod m (reduce-then-combine, eq. "ov-comrtc"); slabs add residues
     modulo m (Sec. V-B).
6-7. CRT over the channel moduli, balanced, one rounding (as ``scheme``).
"""
from __future__ import annotations

import numpy as np

from . import forms, scheme
from .fp_config import usable_alphabet

__all__ = ["channels", "residues", "emulate_fp"]


def channels(fmt: str, k_slab: int, config):
    """forms.Channel for every member (m, rank, base) of a configuration."""
    Sr = usable_alphabet(fmt, k_slab)
    out = []
    for mb in config:
        form = forms.one_limb_form() if mb.rank == 1 else forms.toom2_form(mb.base)
        ch = forms.make_channel(mb.m, form, Sr)
        if ch is None:
            raise ValueError("member %r has no table over this alphabet" % (tuple(mb),))
        out.append(ch)
    return out


def _classes(Xint, m: int) -> np.ndarray:
    if Xint.dtype == np.int64:
        return np.mod(Xint, m).astype(np.int64)
    return np.vectorize(lambda v: int(v) % m, otypes=[np.int64])(Xint) if Xint.size else \
        np.zeros(Xint.shape, dtype=np.int64)


def residues(Ai, Bi, chans, k_slab: int) -> np.ndarray:
    """Z[c] = A'B' mod m_c through each channel's planes, in slabs."""
    M, N = Ai.shape[0], Bi.shape[1]
    Z = np.zeros((len(chans), M, N), dtype=np.int64)
    for c, ch in enumerate(chans):
        Z[c] = forms.channel_residue(_classes(Ai, ch.m), _classes(Bi, ch.m), ch, slab=k_slab)
    return Z


def emulate_fp(A, B, fmt: str, config, k_slab: int, mode: str = "W", keep: bool = False):
    """C = A B through the channels of ``config`` (list of fp_config.Member)
    with slabs of ``k_slab`` terms. Returns a dict with s, t, bits, Z, X, C
    (and the channels when ``keep``)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    moduli = [mb.m for mb in config]
    s, t, finA, finB, bits = scheme._shifts(A, B, moduli, mode)
    A0, B0, _, _ = scheme._finite_parts(A, B)
    Ai = scheme.truncate(A0, s, 1)
    Bi = scheme.truncate(B0, t, 0)
    chans = channels(fmt, k_slab, config)
    Z = residues(Ai, Bi, chans, k_slab)
    X = scheme.crt_balanced(Z, moduli)
    C = scheme.round_scaled(X, s, t)
    C[(~finA)[:, None] | (~finB)[None, :]] = np.nan
    out = {"s": s, "t": t, "bits": bits, "Z": Z, "X": X, "C": C}
    if keep:
        out["channels"] = chans
        out["Aint"], out["Bint"] = Ai, Bi
    return out
