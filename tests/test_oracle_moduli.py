"""Pins for oracle/moduli.py against the paper's printed caps and brute force."""
import json
import os
from itertools import combinations

import pytest

from oracle import moduli as md

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("limit", [20, 36, 49])
@pytest.mark.parametrize("count", [1, 2, 3, 4, 5])
def test_best_coprime_set_brute_force(limit, count):
    best = None
    for c in combinations(range(2, limit + 1), count):
        if md.pairwise_coprime(c):
            key = (md.product(c), tuple(sorted(c, reverse=True)))
            if best is None or key > best:
                best = key
    assert tuple(md.best_coprime_set(count, limit)) == best[1]


def test_sets_are_pairwise_coprime_and_bounded():
    for n in range(1, 25):
        s = md.best_coprime_set(n, 256)
        assert len(s) == n and md.pairwise_coprime(s) and max(s) <= 256 and min(s) >= 2


def test_paper_int8_k_max():
    g = GOLD["int8_k_max"]
    s239 = md.best_coprime_set(g["count"], 239)
    assert tuple(s239) == md.PAPER_INT8_239_SET
    assert max(md.balanced_radius(m) for m in s239) == g["radius_239"]
    assert md.k_max_int8(s239) == g["moduli_le_239"]
    assert md.k_max_int8(md.best_coprime_set(g["count"], 256)) == g["moduli_le_256"]


def test_r_max_values():
    g = GOLD["r_max_1"]
    assert md.r_max(md.LAMBDA_INT32, 1, 2 ** 14) == g["int32_K16384"]
    assert md.r_max(md.LAMBDA_FP32, 1, 2 ** 14) == g["fp32_K16384"]
    assert md.LAMBDA_FP32 // 2 ** 14 == g["lambda_over_K_fp32_K16384"]


def test_counting_bound_int8():
    B = 2 ** 53 - 1
    assert md.counting_bound(2 ** 14, B, B, 256) == GOLD["int8_counting_bound_K16384"]["value"]


def test_window_and_kappa_rec_consistent():
    s = md.best_coprime_set(16, 256)
    P = md.product(s)
    B = 2 ** 53 - 1
    kr = md.kappa_rec(P, B, B)
    assert md.crt_window_ok(P, kr, B, B) and not md.crt_window_ok(P, kr + 1, B, B)
    # fourteen moduli do not reach the FP64 window of eq. "ov-crt" at K = 2**11
    assert not md.crt_window_ok(md.product(md.best_coprime_set(14, 256)), 2048, B, B)
