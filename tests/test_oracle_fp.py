"""Pins for oracle/fp_config.py and oracle/fp_scheme.py: the least GEMM
counts of Table "moduli" (E4M3: 29 at K = 2**12, 30 at 2**14 as 15 one-limb
and 5 two-limb channels, Sec. IV-A; E2M3 sharing E4M3's configuration at
2**14, Example "equivalence"), brute force over small pools, the form
identity of every table checked, and the float-channel scheme equal to the
plain definition at the same kept bits, for any slab length."""
from math import gcd, log2

import numpy as np
import pytest

from oracle import forms, scheme
from oracle import fp_config as fc
from oracle import fp_scheme as fs
from workloads import operand_pair


@pytest.fixture(scope="module")
def e4m3_14():
    return fc.configuration("E4M3", 2 ** 14, window_k=2 ** 14)


def test_fixed_log2_matches_floor_log2():
    for m in list(range(1, 300)) + [1153, 1201, 2401, 65521]:
        v = fc.fixed_log2(m)
        assert abs(v - int(np.floor(log2(m) * 2 ** 32))) <= 2
    assert fc.fixed_log2(1024) == 10 << 32


def test_e4m3_least_q_at_2_14_matches_paper(e4m3_14):
    cfg = e4m3_14
    assert sum(mb.rank for mb in cfg) == 30
    assert sum(1 for mb in cfg if mb.rank == 1) == 15
    assert sum(1 for mb in cfg if mb.rank == 3) == 5
    assert fc.pairwise_coprime(cfg)
    P = 1
    for mb in cfg:
        P *= mb.m
    assert P > 2 ** 14 * 2 ** 107


@pytest.mark.slow
def test_e4m3_least_q_at_2_12_matches_paper():
    cfg = fc.configuration("E4M3", 2 ** 12, window_k=2 ** 12)
    assert sum(mb.rank for mb in cfg) == 29


def test_e2m1_least_q_at_2_14_between_paper_and_ozii_fp4():
    """With one-limb and two-limb Toom forms only, E2M1 reaches the window
    at K = 2**14 in 62 GEMMs: no fewer than the paper's 59 over its larger
    pool, fewer than OzII-FP4's 75 (Table "moduli")."""
    cfg = fc.configuration("E2M1", 2 ** 14, window_k=2 ** 14)
    q = sum(mb.rank for mb in cfg)
    assert q == 62 and 59 <= q < 75
    assert fc.pairwise_coprime(cfg)


def test_e2m3_takes_e4m3_configuration_at_2_14(e4m3_14):
    assert fc.configuration("E2M3", 2 ** 14, window_k=2 ** 14) == e4m3_14


def test_pool_members_are_admissible():
    K = 2 ** 14
    r1 = fc.radius_bound(K)
    assert r1 == 32  # r_max(1) under FP32 at 2**14, Sec. IV (Example "equivalence")
    Sr = fc.usable_alphabet("E4M3", K)
    assert len(Sr) == 49  # 49 values within radius 32
    pool = fc.pool("E4M3", K)
    ones = [mb.m for mb in pool if mb.rank == 1]
    assert max(ones) == 49 and 50 not in ones
    for mb in pool[:: max(1, len(pool) // 12)]:
        form = forms.one_limb_form() if mb.rank == 1 else forms.toom2_form(mb.base)
        ch = forms.make_channel(mb.m, form, Sr)
        assert ch is not None and K * ch.radius ** 2 <= 2 ** 24
        if mb.rank == 3:
            lbar = sum(l % mb.m for l in form.lam)
            assert (mb.m - 1) * lbar <= 2 ** 24


def _least_q_brute(pool, target):
    """Least total rank over every pairwise-coprime subset with product >
    target (recursive enumeration, coprimality pruned as it goes)."""
    best = [None]

    def rec(i, prod, q, used):
        if prod > target:
            best[0] = q if best[0] is None else min(best[0], q)
            return
        if best[0] is not None and q >= best[0]:
            return
        for j in range(i, len(pool)):
            mb = pool[j]
            if all(gcd(mb.m, u) == 1 for u in used):
                rec(j + 1, prod * mb.m, q + mb.rank, used + [mb.m])
    rec(0, 1, 0, [])
    return best[0]


def test_selection_against_brute_force():
    """Least Q over all coprime subsets of a small pool for several targets."""
    pool = [mb for mb in fc.pool("E2M1", 2 ** 14) if mb.m <= 30]
    for target_bits in (12, 20, 28, 34):
        target = 2 ** target_bits
        want = _least_q_brute(pool, target)
        got = fc.select(pool, 40, target=target)
        assert got is not None and fc.pairwise_coprime(got)
        assert sum(mb.rank for mb in got) == want
        P = 1
        for mb in got:
            P *= mb.m
        assert P > target


def test_tables_satisfy_the_form_identity(e4m3_14):
    Sr = fc.usable_alphabet("E4M3", 2 ** 14)
    chans = fs.channels("E4M3", 2 ** 14, e4m3_14)
    small_toom = min((c for c in chans if c.form.rank == 3), key=lambda c: c.m)
    for ch in [c for c in chans if c.form.rank == 1][:6] + [small_toom]:
        assert forms.check_form_identity(ch.m, ch.form, ch.table)
        assert all(all(v in Sr for v in forms._planes_of(ch.form, c, "p")) for c in ch.table)


@pytest.mark.parametrize("mode", ["W", "F53"])
@pytest.mark.parametrize("shape", [(6, 5, 40), (9, 3, 130)])
def test_e4m3_scheme_equals_definition(e4m3_14, mode, shape):
    m, n, k = shape
    A, B = operand_pair(m, n, k, 1.0, 3)
    r = fs.emulate_fp(A, B, "E4M3", e4m3_14, 2 ** 14, mode)
    ref = scheme.definition_product(A, B, [mb.m for mb in e4m3_14], mode)
    assert np.array_equal(r["C"], ref)


def test_e2m1_scheme_equals_definition_and_slabs_agree():
    cfg = fc.configuration("E2M1", 2 ** 14, q=40)
    A, B = operand_pair(7, 6, 90, 2.0, 5)
    ref = scheme.definition_product(A, B, [mb.m for mb in cfg], "W")
    Z0 = None
    for slab in (2 ** 14, 64, 7):
        r = fs.emulate_fp(A, B, "E2M1", cfg, slab, "W")
        assert np.array_equal(r["C"], ref)
        Z0 = r["Z"] if Z0 is None else Z0
        assert np.array_equal(r["Z"], Z0)


def test_accumulator_at_lambda_is_exact(e4m3_14):
    """Every entry of A' and B' congruent to 32 modulo 49, whose one-limb
    table value is 32 = r1: each product's accumulator sums K * 32 * 32 =
    2**24 at K = 2**14, the largest value the bound allows."""
    ch = [c for c in fs.channels("E4M3", 2 ** 14, e4m3_14) if c.m == 49][0]
    assert ch.table[32] == (32,)
    K = 2 ** 14
    Acls = np.full((2, K), 32, dtype=np.int64)
    Bcls = np.full((K, 3), 32, dtype=np.int64)
    U = forms.channel_planes(Acls, ch, "p")[0]
    V = forms.channel_planes(Bcls, ch, "q")[0]
    W = U @ V
    assert (W == 2 ** 24).all()
    assert (forms.channel_residue(Acls, Bcls, ch) == (32 * 32 * K) % 49).all()
