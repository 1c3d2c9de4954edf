"""GPU parity of the blocked call (Sec. V-B, "Slabs"): the inner dimension
in slabs, each slab's residues added into a running residue mod m. The
result is bitwise the oracle's emulated product over the whole inner
dimension (same kept bits), for slabs of any length, ragged last slabs,
and an inner dimension beyond the INT32 accumulation cap that the
unblocked call refuses."""
import numpy as np
import pytest

from oracle import scheme
from tests.gpu_util import cuda_ok, dev, host
from workloads import operand_pair

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a HIP device")]

oz = pytest.importorskip("paper_2609_37693_amd")


@pytest.mark.parametrize("mode,nmod", [("W", 16), ("F53", 16), ("W", 20)])
@pytest.mark.parametrize("shape,k_slab", [((300, 257, 1000), 64), ((300, 257, 1000), 100),
                                          ((300, 257, 1000), 999), ((300, 257, 1000), 4096),
                                          ((1, 1, 1), 1), ((513, 70, 130), 65)])
def test_blocked_matches_oracle(mode, nmod, shape, k_slab):
    import torch
    m, n, k = shape
    A, B = operand_pair(m, n, k, 0.5, 3)
    plan = oz.Plan(num_moduli=nmod, scaling=mode)
    print("blocked", mode, nmod, shape, k_slab, flush=True)
    C = host(oz.dgemm_blocked(dev(A), dev(B), plan, k_slab))
    torch.cuda.synchronize()
    ref = scheme.emulate(A, B, plan.moduli(), mode, blas=True, keep=False)["C"]
    assert np.array_equal(C, ref)


def test_blocked_beyond_the_accumulation_cap():
    """k = 140000 > 131071: the unblocked call refuses it; two and three
    slabs give the oracle's product bitwise, non-finite rows and columns
    give NaN."""
    import torch
    plan = oz.Plan(num_moduli=16, scaling="W")
    cap = plan.k_max()
    m, n, k = 5, 6, 140000
    assert k > cap
    A, B = operand_pair(m, n, k, 0.5, 4)
    A[2, 777] = np.nan
    B[99999, 4] = np.inf
    with pytest.raises(oz.OzemuError):
        oz.dgemm(dev(A), dev(B), plan)
    ref = scheme.emulate(A, B, plan.moduli(), "W", blas=True, keep=False)["C"]
    assert np.isnan(ref[2]).all() and np.isnan(ref[:, 4]).all()
    for k_slab in (cap, 50000):
        print("blocked beyond cap", k_slab, flush=True)
        C = host(oz.dgemm_blocked(dev(A), dev(B), plan, k_slab))
        torch.cuda.synchronize()
        assert np.array_equal(C, ref, equal_nan=True), k_slab


def test_blocked_single_slab_equals_unblocked_call():
    """With k_slab >= k the blocked call is the unblocked call, and reusing
    one workspace across calls of different slab counts keeps results."""
    import torch
    m, n, k = 600, 520, 2048
    A, B = operand_pair(m, n, k, 1.0, 5)
    plan = oz.Plan(num_moduli=16, scaling="W")
    dA, dB = dev(A), dev(B)
    nbytes = max(oz.blocked_workspace_size(plan, m, n, k, 256),
                 oz.blocked_workspace_size(plan, m, n, k, k))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    full = host(oz.dgemm(dA, dB, plan))
    one = host(oz.dgemm_blocked(dA, dB, plan, k, workspace=ws))
    eight = host(oz.dgemm_blocked(dA, dB, plan, 256, workspace=ws))
    again = host(oz.dgemm_blocked(dA, dB, plan, k, workspace=ws))
    torch.cuda.synchronize()
    assert np.array_equal(one, full) and np.array_equal(eight, full) and np.array_equal(again, full)


def test_blocked_with_leading_dimensions():
    """Operands that are column slices of wider matrices (lda > k, ldb > n)
    and C written into a wider buffer: each slab's columns of A and rows of
    B are found through the leading dimensions."""
    import torch
    m, n, k = 130, 90, 700
    A, B = operand_pair(m, n, k, 1.0, 8)
    plan = oz.Plan(num_moduli=16, scaling="W")
    wideA = torch.zeros((m, k + 37), dtype=torch.float64, device="cuda")
    wideB = torch.zeros((k, n + 5), dtype=torch.float64, device="cuda")
    wideA[:, 3:3 + k] = dev(A)
    wideB[:, 1:1 + n] = dev(B)
    wideC = torch.full((m, n + 11), 7.0, dtype=torch.float64, device="cuda")
    dA, dB = wideA[:, 3:3 + k], wideB[:, 1:1 + n]
    assert dA.stride(0) == k + 37 and dB.stride(0) == n + 5
    oz.dgemm_blocked(dA, dB, plan, 256, out=wideC[:, 2:2 + n])
    torch.cuda.synchronize()
    Cw = host(wideC)
    ref = scheme.emulate(A, B, plan.moduli(), "W", blas=True, keep=False)["C"]
    assert np.array_equal(Cw[:, 2:2 + n], ref)
    assert (Cw[:, :2] == 7.0).all() and (Cw[:, 2 + n:] == 7.0).all()
