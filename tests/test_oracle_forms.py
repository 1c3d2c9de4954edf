"""Pins for oracle/alphabets.py and oracle/forms.py against the paper's
worked examples (values in tests/golden/paper_values.json)."""
import json
import os

import numpy as np
import pytest

from oracle import alphabets as al
from oracle import forms as fo

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _run(vals):
    x = 0
    while (x + 1) in vals and -(x + 1) in vals:
        x += 1
    return x


def test_e2m1_alphabet():
    g = GOLD["e2m1_alphabet"]
    assert al.alphabet("E2M1") == g["value"] and al.alphabet_scale("E2M1") == g["e_S"]


def test_int8_alphabet():
    assert al.alphabet("INT8") == list(range(-128, 128))


def test_example1_reach_and_encoding():
    g = GOLD["example1"]
    S = al.alphabet("E2M1")
    b = g["base"]
    assert _run(fo.reach(S, b, 1)) == g["one_limb_run"]
    r2 = fo.reach(S, b, 2)
    assert _run(r2) == g["two_limb_run"]
    assert all(v in r2 for v in g["reachable_past_run"])
    assert not any(v in r2 for v in g["unreachable_past_run"])
    c0, c1 = g["five"]
    assert c0 + b * c1 == 5 and 5 not in S and c0 in S and c1 in S
    sb = fo.schoolbook_form(115, b, 2)
    tab = fo.encode_table(115, sb, S)
    assert list(tab[57]) == g["class57_mod115"]
    assert tab[57][0] + b * tab[57][1] == g["class57_value"]
    assert fo.channel_radius(tab, sb) == g["radius_115"]
    within = [v for v in S if abs(v) <= g["radius_115"]]
    assert len(within) == g["values_within_8"]
    assert len(within) ** 2 == g["max_modulus_two_limbs_radius8"]
    assert fo.encode_table(169, fo.schoolbook_form(169, b, 2), within) is not None
    gamma = max(min(abs(s) for s in S if (s - c) % b == 0) for c in range(b))
    assert gamma == g["gamma_mod13"]


def test_product_set_size_e2m1():
    S = al.alphabet("E2M1")
    assert len({a * b for a in S for b in S}) == GOLD["e2m1_product_set_size"]["value"]


def test_values_within_radius_32():
    for name, cnt in GOLD["within_radius_32"].items():
        if name.startswith("cite"):
            continue
        assert len([v for v in al.alphabet(name) if abs(v) <= 32]) == cnt


def test_partner_agreement():
    g = GOLD["partner_agreement"]
    for pair, lim in (("E4M3_E2M3", g["E4M3_E2M3"]), ("E5M2_E3M2", g["E5M2_E3M2"])):
        big, small = pair.split("_")
        A, B = set(al.alphabet(big)), set(al.alphabet(small))
        assert max(B) == lim
        assert {v for v in A if abs(v) <= lim} == {v for v in B if abs(v) <= lim}
        assert any(v in A for v in range(lim + 1, 2 * lim + 1))


def test_schoolbook_rank_and_ozii_fp4_count():
    g = GOLD["schoolbook_169_13_2_rank"]
    assert fo.schoolbook_rank(169, 13, 2) == g["value"]
    assert fo.schoolbook_form(169, 13, 2).rank == g["value"]
    assert fo.schoolbook_rank(115, 13, 2) == 4
    assert (g["channels"] - 1) * 4 + fo.schoolbook_rank(169, 13, 2) == g["ozii_fp4_Q"]


def test_search_figure_count_arithmetic():
    g = GOLD["search_figure_Q"]
    assert sum(a * b for a, b in g["terms"]) == g["value"]


@pytest.mark.parametrize("fmt,m,b", [("E2M1", 115, 13), ("E2M1", 97, 11), ("E2M3", 601, 29),
                                     ("E2M1", 13, 1)])
def test_form_identity_every_class_pair(fmt, m, b):
    S = al.alphabet(fmt)
    forms = [fo.toom2_form(b), fo.schoolbook_form(m, b, 2)] if b > 1 else [fo.one_limb_form()]
    for f in forms:
        tab = fo.encode_table(m, f, S)
        if tab is None:
            continue
        assert fo.check_form_identity(m, f, tab)


def test_toom2_weights_reproduce_product():
    rng = np.random.default_rng(0)
    b = 17
    f = fo.toom2_form(b)
    for _ in range(200):
        a0, a1, c0, c1 = (int(x) for x in rng.integers(-40, 41, 4))
        W0, W1, Wi = a0 * c0, (a0 + a1) * (c0 + c1), a1 * c1
        assert f.lam[0] * W0 + f.lam[1] * W1 + f.lam[2] * Wi == (a0 + b * a1) * (c0 + b * c1)


def test_channel_residue_matches_direct_product_with_slabs():
    S = al.alphabet("E2M1")
    rng = np.random.default_rng(4)
    for m, b in ((115, 13), (97, 11)):
        for f in (fo.toom2_form(b), fo.schoolbook_form(m, b, 2)):
            ch = fo.make_channel(m, f, S)
            if ch is None:
                continue
            A = rng.integers(-10 ** 6, 10 ** 6, (7, 45))
            B = rng.integers(-10 ** 6, 10 ** 6, (45, 6))
            ref = np.mod(A @ B, m)
            for slab in (0, 8, 45, 44):
                assert np.array_equal(fo.channel_residue(np.mod(A, m), np.mod(B, m), ch, slab), ref)


def test_rtc_epilogue_reduces_each_term():
    W = [np.array([[-5, 10 ** 6]]), np.array([[7, -3]])]
    Z = fo.rtc_epilogue(W, [-12, 13], 11)
    assert np.array_equal(Z, np.mod(-12 * W[0] + 13 * W[1], 11))
