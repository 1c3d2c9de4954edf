"""GPU parity of the float-channel path (FP8 E4M3, FP6 E2M3 and FP4 E2M1
matrix cores, FP32 accumulation) against oracle/fp_scheme.py, bitwise, through
the C-ABI: ragged shapes, several channel sets, slabs, an accumulator
driven to exactly 2**24, and sampled entries of the 16384-cubed workload."""
import numpy as np
import pytest

from oracle import exact, scheme
from oracle import fp_config as fc
from oracle import fp_scheme as fs
from tests.gpu_util import cuda_ok, dev, host
from workloads import operand_pair

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a HIP device")]

oz = pytest.importorskip("paper_2609_37693_amd")

_CFG = {}


def _config(fmt, gemms, k_slab):
    key = (fmt, gemms, k_slab)
    if key not in _CFG:
        if gemms == 0:
            _CFG[key] = fc.configuration(fmt, k_slab, window_k=k_slab)
        else:
            _CFG[key] = fc.configuration(fmt, k_slab, q=gemms)
    return _CFG[key]


CASES = [("E4M3", 30, "W"), ("E4M3", 0, "F53"), ("E4M3", 0, "W"), ("E2M1", 40, "W"),
         ("E2M1", 24, "W"), ("E2M3", 0, "W"), ("E2M3", 36, "F53"), ("E2M3", 22, "W")]
SHAPES = [(256, 256, 256), (300, 257, 129), (5, 700, 3), (513, 260, 1100), (1, 1, 1)]


@pytest.mark.parametrize("fmt,gemms,mode", CASES)
@pytest.mark.parametrize("shape", SHAPES)
def test_fp_dgemm_matches_oracle(fmt, gemms, mode, shape):
    import torch
    m, n, k = shape
    A, B = operand_pair(m, n, k, 1.0, 17)
    plan = oz.Plan(format=fmt, gemms=gemms, k_slab=16384, scaling=mode)
    cfg = _config(fmt, gemms, 16384)
    assert plan.channels() == [tuple(mb) for mb in cfg]
    C = oz.dgemm(dev(A), dev(B), plan)
    torch.cuda.synchronize()
    ref = fs.emulate_fp(A, B, fmt, cfg, 16384, mode)["C"]
    assert np.array_equal(host(C), ref)


@pytest.mark.parametrize("fmt,gemms", [("E4M3", 30), ("E2M1", 40), ("E2M3", 30)])
def test_fp_slabs_and_special_values(fmt, gemms):
    """K = 20000 runs in two slabs of 16384 terms whose residues add
    modulo m; a NaN row, a zero column and an infinite column as in the
    INT8 path."""
    import torch
    m, n, k = 70, 90, 20000
    A, B = operand_pair(m, n, k, 2.0, 23)
    A[5, 17] = np.nan
    B[:, 3] = 0.0
    B[100, 8] = -np.inf
    plan = oz.Plan(format=fmt, gemms=gemms, k_slab=16384)
    cfg = _config(fmt, gemms, 16384)
    C = oz.dgemm(dev(A), dev(B), plan)
    torch.cuda.synchronize()
    ref = fs.emulate_fp(A, B, fmt, cfg, 16384, "W")["C"]
    assert np.array_equal(host(C), ref, equal_nan=True)
    assert np.isnan(host(C)[5]).all() and np.isnan(host(C)[:, 8]).all()


def _value_for_class(target, beta, m):
    """Smallest integer a in [1, 2**20] with a * 2**(beta - e(a)) == target
    (mod m), e(a) the bit length of a: a row of equal entries a keeps
    exactly that integer after scaling to beta bits."""
    for a in range(1, 1 << 20):
        e = a.bit_length()
        if (a * pow(2, beta - e, m)) % m == target % m if beta >= e else False:
            return a
    raise AssertionError("no value")


@pytest.mark.parametrize("fmt", ["E4M3", "E2M3"])
def test_accumulator_at_lambda_is_exact(fmt):
    """Every entry of A' and B' congruent to 32 modulo 49, whose one-limb
    plane value is 32 = floor(sqrt(2**24 / 2**14)): each accumulator of
    that channel sums 2**14 products 32 * 32 = 2**24 exactly on the FP8
    (or FP6) unit; the whole product must equal the oracle bitwise."""
    import torch
    plan = oz.Plan(format=fmt, gemms=0, k_slab=16384)
    cfg = _config(fmt, 0, 16384)
    assert 49 in [mb.m for mb in cfg]
    K = 16384
    ba, bb = plan.kept_bits(K)
    a = _value_for_class(32, ba, 49)
    b = _value_for_class(32, bb, 49)
    A = np.full((64, K), float(a))
    B = np.full((K, 64), float(b))
    A[1::2] *= -1.0  # signs vary by row, magnitudes stay at the radius
    C = oz.dgemm(dev(A), dev(B), plan)
    torch.cuda.synchronize()
    ref = fs.emulate_fp(A, B, fmt, cfg, 16384, "W")["C"]
    assert np.array_equal(host(C), ref)
    assert np.array_equal(host(C), A @ B)  # small integers: the exact product


@pytest.mark.parametrize("fmt,gemms", [("E4M3", 0), ("E2M1", 0), ("E2M3", 0)])
def test_fp_16384_sampled_parity_and_error(fmt, gemms):
    """The float workload, m = n = k = 16384, phi = 1, at the window
    configurations (Q = 30 for E4M3 and E2M3, 62 for E2M1): sampled rows x columns
    bitwise equal to the oracle (kept bits depend on K and the modulus
    product only); the exact scaled error is reported and bounded by 2**-46
    (53/54 kept bits at this K; 2**-50 takes a few more GEMMs)."""
    import torch
    N = 16384
    A, B = operand_pair(N, N, N, 1.0, 0)
    plan = oz.Plan(format=fmt, gemms=gemms, k_slab=16384)
    cfg = _config(fmt, gemms, 16384)
    C = oz.dgemm(dev(A), dev(B), plan)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(N, 8, replace=False))
    cols = np.sort(rng.choice(N, 8, replace=False))
    As = np.ascontiguousarray(A[rows])
    Bs = np.ascontiguousarray(B[:, cols])
    got = host(C)[np.ix_(rows, cols)]
    ref = fs.emulate_fp(As, Bs, fmt, cfg, 16384, "W")["C"]
    assert np.array_equal(got, ref)
    err = exact.scaled_error(got, As, Bs)
    print("%s scaled error over the sample: 2^%.2f" % (fmt, np.log2(err) if err > 0 else -99))
    assert err <= 2.0 ** -46
