"""CPU tests of the moduli-count choice for grouped products: the chosen
count reaches the kept-bit target and one modulus fewer does not; the kept
bits agree with the oracle's mode-W rule for the library's modulus sets."""
import pytest

from oracle import moduli as md
from oracle import scheme

oz = pytest.importorskip("paper_2609_37693_amd")
from paper_2609_37693_amd import autotune  # noqa: E402


@pytest.mark.parametrize("k", [1, 64, 128, 129, 1000, 4096, 8192, 65536])
@pytest.mark.parametrize("target", [40, 55])
def test_smallest_count_meeting_target(k, target):
    n = autotune.moduli_for(k, target)
    P = md.product(md.best_coprime_set(n))
    assert min(scheme.kept_bits("W", P, k)) >= target
    if n > 2:
        Pm = md.product(md.best_coprime_set(n - 1))
        try:
            bits = scheme.kept_bits("W", Pm, k)
        except ValueError:
            return
        assert min(bits) < target


def test_plans_shared_and_fixed_count():
    shapes = [(10, 10, 64), (5, 7, 64), (3, 3, 5000)]
    ps = autotune.plans_for(shapes)
    assert ps[0] is ps[1] and len(ps[2].moduli()) >= len(ps[0].moduli())
    fixed = autotune.plans_for(shapes, moduli=14)
    assert all(len(p.moduli()) == 14 for p in fixed)
