"""GPU parity: every phase of the HIP path against the CPU oracle on the
same seeded inputs, bit for bit (integer work and the correctly rounded
result alike), through the C-ABI."""
import numpy as np
import pytest

from oracle import exact, scheme
from oracle import moduli as md
from tests.gpu_util import (cuda_ok, dev, host, oracle_shifts, oracle_planes, default_moduli,
                            to_blocked, from_blocked, plane_offsets)
from workloads import operand_pair, row_exponent_matrix

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a HIP device")]

oz = pytest.importorskip("paper_2609_37693_amd")

SHAPES = [(256, 256, 256), (300, 257, 129), (1, 1, 1), (5, 700, 3), (513, 260, 520)]


def _inputs(m, n, k, phi=0.5, seed=0):
    A, B = operand_pair(m, n, k, phi, seed)
    return A, B


@pytest.mark.parametrize("mode,nmod", [("W", 14), ("F53", 16), ("G", 14), ("W", 20), ("G", 20)])
@pytest.mark.parametrize("shape", SHAPES)
def test_scale_matches_oracle(mode, nmod, shape):
    m, n, k = shape
    A, B = _inputs(m, n, k, 1.0, 3)
    if m > 2:
        A[1, :] = 0.0
    plan = oz.Plan(num_moduli=nmod, scaling=mode)
    ms = plan.moduli()
    sa, sb = oz.scale(dev(A), dev(B), plan)
    s, t = oracle_shifts(A, B, ms, mode)
    assert np.array_equal(host(sa).astype(np.int64), s)
    assert np.array_equal(host(sb).astype(np.int64), t)


@pytest.mark.parametrize("mode,nmod", [("W", 14), ("W", 20), ("G", 16), ("F53", 16)])
@pytest.mark.parametrize("shape", [(256, 256, 256), (300, 257, 129), (5, 700, 3)])
def test_reduce_planes_match_oracle(mode, nmod, shape):
    m, n, k = shape
    A, B = _inputs(m, n, k, 4.0, 5)
    plan = oz.Plan(num_moduli=nmod, scaling=mode)
    ms = plan.moduli()
    sa, sb = oz.scale(dev(A), dev(B), plan)
    pa, pb = oz.reduce(dev(A), dev(B), sa, sb, plan)
    PA, PB = oracle_planes(A, B, ms, mode, plan.plane_dims(m, n, k))
    assert np.array_equal(from_blocked(host(pa)), PA)
    assert np.array_equal(from_blocked(host(pb)), PB)


@pytest.mark.parametrize("shape", [(256, 256, 256), (300, 257, 129), (512, 768, 320),
                                   (513, 260, 1100)])
def test_residue_gemm_matches_oracle(shape):
    m, n, k = shape
    rng = np.random.default_rng(7)
    plan = oz.Plan(num_moduli=16, scaling="W")
    ms = plan.moduli()
    mp, np_, kp = plan.plane_dims(m, n, k)
    PA = np.zeros((16, mp, kp), np.int8)
    PB = np.zeros((16, np_, kp), np.int8)
    for l, mm in enumerate(ms):
        lo, hi = -(mm // 2), (mm + 1) // 2 - 1
        PA[l, :m, :k] = rng.integers(lo, hi + 1, (m, k))
        PB[l, :n, :k] = rng.integers(lo, hi + 1, (n, k))
    z = host(oz.residue_gemm(dev(to_blocked(PA)), dev(to_blocked(PB)), m, n, k, plan))
    for l, mm in enumerate(ms):
        _, Z = scheme.residue_gemm(PA[l, :m, :k].astype(np.int64), PB[l, :n, :k].T.astype(np.int64),
                                   int(mm))
        assert np.array_equal(z[l, :m, :n], Z), "modulus %d" % mm


def test_residue_gemm_extreme_accumulators():
    """Planes at the largest magnitudes with one sign per column block, so
    every INT32 accumulator reaches -k 128 127 or k 128**2 (2**27 at
    k = 8192): exact sums in both signs."""
    m = n = 256
    k = 8192
    plan = oz.Plan(num_moduli=16, scaling="W")
    ms = plan.moduli()
    mp, np_, kp = plan.plane_dims(m, n, k)
    PA = np.full((16, mp, kp), -128, np.int8)
    PB = np.full((16, np_, kp), -128, np.int8)
    PB[:, : n // 2, :] = 127
    z = host(oz.residue_gemm(dev(to_blocked(PA)), dev(to_blocked(PB)), m, n, k, plan))
    for l, mm in enumerate(ms):
        assert np.all(z[l, :, : n // 2] == (k * -128 * 127) % mm)
        assert np.all(z[l, :, n // 2:] == (k * 128 * 128) % mm)


@pytest.mark.parametrize("mode,nmod", [("W", 14), ("G", 14), ("W", 20), ("W", 10), ("F53", 16)])
@pytest.mark.parametrize("shape", [(256, 256, 256), (300, 257, 129), (1, 1, 1), (7, 300, 1000),
                                   (520, 770, 2000)])
def test_dgemm_bitwise_matches_oracle(mode, nmod, shape):
    m, n, k = shape
    A, B = _inputs(m, n, k, 0.5, 0)
    plan = oz.Plan(num_moduli=nmod, scaling=mode)
    C = host(oz.dgemm(dev(A), dev(B), plan))
    ref = scheme.emulate(A, B, plan.moduli(), mode, keep=False)["C"]
    assert np.array_equal(C, ref)


def test_phases_compose_to_dgemm():
    m, n, k = 300, 257, 129
    A, B = _inputs(m, n, k, 1.0, 2)
    plan = oz.Plan(num_moduli=16, scaling="W")
    dA, dB = dev(A), dev(B)
    sa, sb = oz.scale(dA, dB, plan)
    pa, pb = oz.reduce(dA, dB, sa, sb, plan)
    z = oz.residue_gemm(pa, pb, m, n, k, plan)
    C1 = host(oz.reconstruct(z, sa, sb, m, n, k, plan))
    C2 = host(oz.dgemm(dA, dB, plan))
    assert np.array_equal(C1, C2)
    r = scheme.emulate(A, B, plan.moduli(), "W")
    mp, np_, kp = plan.plane_dims(m, n, k)
    assert np.array_equal(host(z)[:, :m, :n], r["Z"])


def test_config1_accuracy():
    """256 cubed, phi = 0.5, fourteen moduli (the small workload): bitwise
    equal to the oracle, and mode G within 2**-50 scaled error."""
    A, B = _inputs(256, 256, 256, 0.5, 0)
    for mode in ("W", "G"):
        plan = oz.Plan(num_moduli=14, scaling=mode)
        C = host(oz.dgemm(dev(A), dev(B), plan))
        assert np.array_equal(C, scheme.emulate(A, B, plan.moduli(), mode, keep=False)["C"])
        if mode == "G":
            assert exact.scaled_error(C, A, B) <= 2.0 ** -50


def test_special_values():
    m, n, k = 70, 66, 90
    A, B = _inputs(m, n, k, 2.0, 4)
    A[0, :] = 0.0
    B[:, 1] = 0.0
    A[2, 5] = np.inf
    A[3, 7] = np.nan
    B[4, 9] = -np.inf
    A[5, :] = A[5, :] * 1e-300
    A[6, :] = 5e-324 * np.arange(k)  # subnormals
    A[7, :] = A[7, :] * 1e300
    B[:, 10] = B[:, 10] * 1e300  # products overflow to infinity
    A[8, 3] = 1e300
    A[8, 4] = 1e-300  # row spanning 2**1993
    for mode in ("W", "G", "F53"):
        nm = 16
        plan = oz.Plan(num_moduli=nm, scaling=mode)
        C = host(oz.dgemm(dev(A), dev(B), plan))
        ref = scheme.emulate(A, B, plan.moduli(), mode, keep=False)["C"]
        assert np.array_equal(C, ref, equal_nan=True), mode


def test_integer_operands_exact():
    from workloads import integer_matrix
    A = integer_matrix(200, 300, 2 ** 20, 1)
    B = integer_matrix(300, 150, 2 ** 20, 2)
    plan = oz.Plan(num_moduli=14, scaling="W")
    C = host(oz.dgemm(dev(A), dev(B), plan))
    assert np.array_equal(C, (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))


def test_empty_and_degenerate_shapes():
    import torch
    plan = oz.Plan(num_moduli=12, scaling="W")
    A = torch.zeros((0, 5), dtype=torch.float64, device="cuda")
    B = torch.zeros((5, 3), dtype=torch.float64, device="cuda")
    assert oz.dgemm(A, B, plan).shape == (0, 3)
    A = torch.randn((4, 0), dtype=torch.float64, device="cuda")
    B = torch.randn((0, 3), dtype=torch.float64, device="cuda")
    C = oz.dgemm(A, B, plan)
    assert C.shape == (4, 3) and bool(torch.all(C == 0))


def test_moduli_set_does_not_change_f53_result():
    A, B = _inputs(200, 180, 400, 1.0, 9)
    c1 = host(oz.dgemm(dev(A), dev(B), oz.Plan(num_moduli=16, scaling="F53")))
    c2 = host(oz.dgemm(dev(A), dev(B), oz.Plan(moduli=list(md.PAPER_INT8_239_SET), scaling="F53")))
    assert np.array_equal(c1, c2)


def test_strided_operands():
    import torch
    A, B = _inputs(130, 140, 150, 1.0, 11)
    plan = oz.Plan(num_moduli=14, scaling="W")
    bigA = torch.zeros((130, 200), dtype=torch.float64, device="cuda")
    bigA[:, :150] = dev(A)
    bigB = torch.zeros((150, 171), dtype=torch.float64, device="cuda")
    bigB[:, :140] = dev(B)
    C = host(oz.dgemm(bigA[:, :150], bigB[:, :140], plan))
    assert np.array_equal(C, scheme.emulate(A, B, plan.moduli(), "W", keep=False)["C"])


def test_row_exponent_operands():
    A = row_exponent_matrix(128, 96, 3)
    B = row_exponent_matrix(96, 160, 4)
    for mode in ("W", "G"):
        plan = oz.Plan(num_moduli=16, scaling=mode)
        C = host(oz.dgemm(dev(A), dev(B), plan))
        assert np.array_equal(C, scheme.emulate(A, B, plan.moduli(), mode, keep=False)["C"])


def test_repeated_calls_are_bitwise_stable():
    """Regression: every call must give the same bits. Bound-adaptive scaling
    once varied between runs (its ceiling was computed through a 64-bit
    integer sequence); the bound planes are now formed with an exact FP64
    ldexp and ceiling."""
    import torch
    m, n, k = 513, 260, 520
    A, B = _inputs(m, n, k, 1.0, 3)
    A[1, :] = 0.0
    dA, dB = dev(A), dev(B)
    for mode, nmod in (("G", 20), ("W", 16)):
        plan = oz.Plan(num_moduli=nmod, scaling=mode)
        s, t = oracle_shifts(A, B, plan.moduli(), mode)
        ref = scheme.emulate(A, B, plan.moduli(), mode, keep=False)["C"]
        for rep in range(8):
            ws = torch.randint(0, 256, (plan.workspace_size(m, n, k),), dtype=torch.uint8,
                               device="cuda")
            sa, sb = oz.scale(dA, dB, plan, workspace=ws)
            assert np.array_equal(host(sa).astype(np.int64), s), (mode, rep)
            assert np.array_equal(host(sb).astype(np.int64), t), (mode, rep)
            C = host(oz.dgemm(dA, dB, plan, workspace=ws))
            assert np.array_equal(C, ref), (mode, rep)


def test_full_size_sampled_parity_and_error():
    """The bench workload (8192 cubed, phi = 0.5, sixteen moduli, mode W):
    C on 48 sampled rows x 48 sampled columns is bitwise equal to the oracle
    (in mode W a row's shift depends only on that row and K), and the exact
    scaled error max |C - AB| / (|A||B|) over the sample is at most 2**-50."""
    import torch
    n = 8192
    A, B = operand_pair(n, n, n, 0.5, 0)
    plan = oz.Plan(num_moduli=16, scaling="W")
    C = oz.dgemm(dev(A), dev(B), plan)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(n, 48, replace=False))
    cols = np.sort(rng.choice(n, 48, replace=False))
    Cs = host(C)[np.ix_(rows, cols)]
    As = np.ascontiguousarray(A[rows])
    Bs = np.ascontiguousarray(B[:, cols])
    ref = scheme.emulate(As, Bs, plan.moduli(), "W", blas=True, keep=False)["C"]
    assert np.array_equal(Cs, ref)
    err = exact.scaled_error(Cs, As, Bs)
    assert err <= 2.0 ** -50, err


def test_full_size_certified_bound():
    """The bench workload over the whole matrix: the Scale phase's shifts
    equal the definition's (frexp exponents of every row and column maximum)
    and the certified bound (|dA||B| + |Ahat||dB| + 2^-53 |C|) / (|A||B|),
    valid for the correctly rounded product that the sampled and small-size
    parity tests check bit for bit, is at most 2**-50 on every entry."""
    import os
    import sys
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    n = 8192
    A, B = operand_pair(n, n, n, 0.5, 0)
    plan = oz.Plan(num_moduli=16, scaling="W")
    dA, dB = dev(A), dev(B)
    del A, B
    C = oz.dgemm(dA, dB, plan)
    sa, sb = oz.scale(dA, dB, plan)
    ba, bb = plan.kept_bits(n)
    bound, s, t = bench.certified_error_bound(dA, dB, C, ba, bb)
    assert torch.equal(s, sa.to(torch.int64)) and torch.equal(t, sb.to(torch.int64))
    worst = float(bound.max())
    assert worst <= 2.0 ** -50, worst


@pytest.mark.parametrize("shape,mode,nmod", [((4100, 300, 200), "W", 14), ((6000, 50, 70), "G", 16),
                                             ((4352, 257, 129), "F53", 16)])
def test_tall_products_match_oracle(shape, mode, nmod):
    """Tall products (more than 4096 rows, a ragged last tile row) in modes
    W, G and F53: bitwise equal to the oracle, and repeated calls agree."""
    import torch
    m, n, k = shape
    A, B = _inputs(m, n, k, 1.0, 31)
    plan = oz.Plan(num_moduli=nmod, scaling=mode)
    C1 = oz.dgemm(dev(A), dev(B), plan)
    C2 = oz.dgemm(dev(A), dev(B), plan)
    torch.cuda.synchronize()
    ref = scheme.emulate(A, B, plan.moduli(), mode, blas=True, keep=False)["C"]
    assert np.array_equal(host(C1), ref)
    assert np.array_equal(host(C2), ref)


_ODD16 = [251, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191, 181, 179, 173, 167]


@pytest.mark.parametrize("moduli", [None, _ODD16])
def test_reconstruct_crt_edge_values(moduli):
    """Reconstruct alone, on the residues of chosen X: 0, +-1, the ends of
    the balanced range +-(P-1)/2 (where the estimate of the nearest multiple
    of P may be off by one), values next to P 2^-30 and P/2 - P 2^-30 (where
    the sign is or is not read from the estimate), rounding ties at 2^53,
    2^54, 2^64 and 2^100 and at bit positions around the 40-bit chunk
    boundaries (with their neighbours), and random values; row shifts that give normal,
    subnormal, zero and infinite results; a column with the non-finite
    marker gives NaN. Bitwise equal to the oracle's one rounding of
    X 2^-(s_i + t_j). The default set holds 256 (P even), the other only
    odd moduli."""
    import torch
    from oracle import exact
    plan = oz.Plan(num_moduli=16, scaling="W") if moduli is None else \
        oz.Plan(scaling="W", moduli=moduli)
    ms = plan.moduli()
    P = 1
    for mm in ms:
        P *= mm
    half = (P - 1) // 2
    e30, e31 = P >> 30, P >> 31
    xs = [0, 1, 2, 3, half, half - 1, half - 2 ** 20, e30, e30 - 1, e30 + 1, e31,
          half - e30, half - e30 - 1, half - e30 + 1, half - e31,
          2 ** 53 + 1, 2 ** 53 + 3, 2 ** 54 + 2, 2 ** 54 + 6, 2 ** 64 + 2 ** 11,
          2 ** 64 + 3 * 2 ** 11, 2 ** 100 + 2 ** 47, 2 ** 100 + 2 ** 47 + 1]
    # exact ties of the 53-bit rounding and their neighbours at bit
    # positions around the 40-bit chunk boundaries, and leading chunks just
    # below and above 2^13
    for pos in (1, 12, 13, 26, 27, 39, 40, 41, 52, 53, 66, 70):
        for t in (2 ** 52 + 5, 2 ** 52 + 4, 2 ** 53 - 1):
            x = t * 2 ** (pos + 1) + 2 ** pos
            xs += [x, x - 1, x + 1]
    xs += [2 ** 93 - 1, 2 ** 93, 2 ** 93 + 2 ** 40 + 1, 2 ** 52 + 1, 2 ** 53 - 1,
           2 ** 92 + 2 ** 39, 2 ** 120 + 2 ** 67 + 2 ** 66]
    xs = [x for x in xs if x <= half]
    xs = xs + [-x for x in xs if x]
    rng = np.random.default_rng(11)
    xs += [int(v) for v in rng.integers(-2 ** 62, 2 ** 62, 8)]
    xs += [int.from_bytes(rng.bytes(16), "little") % P - half for _ in range(12)]
    row_shifts = [0, 40, -40, 1000, 1060, 1100, 1150, 1200, 1300, -900, -1100]
    m, n, k = len(row_shifts), len(xs) + 1, 64
    mp, np_, _ = plan.plane_dims(m, n, k)
    Z = np.zeros((len(ms), mp, np_), dtype=np.uint8)
    X = np.zeros((m, n), dtype=object)
    for j, x in enumerate(xs):
        X[:, j] = x
    for l, mm in enumerate(ms):
        Z[l, :m, :n] = np.vectorize(lambda v: int(v) % mm, otypes=[np.int64])(X)
    sa = np.array(row_shifts, dtype=np.int32)
    sb = np.zeros(n, dtype=np.int32)
    sb[n - 1] = -(2 ** 31)  # the non-finite marker
    C = host(oz.reconstruct(dev(Z), dev(sa), dev(sb), m, n, k, plan))
    torch.cuda.synchronize()
    for i in range(m):
        for j in range(n - 1):
            want = exact.round_ratio_to_double(int(X[i, j]), int(sa[i]))
            got = C[i, j]
            assert got == want and np.signbit(got) == np.signbit(want), (i, j, xs[j], row_shifts[i])
    assert np.isnan(C[:, n - 1]).all()


@pytest.mark.parametrize("nmod,shape", [(17, (130, 90, 64)), (17, (70, 65, 100)),
                                        (17, (300, 257, 256)), (18, (65, 70, 8192))])
def test_kept_bits_at_the_reduce_threshold(nmod, shape):
    """Plans keeping 62 bits (signed-digit Reduce, |A'| up to 2^62 - 2^10
    here) and 63 bits (the exact form), with rows and columns at their
    largest magnitude of either sign: bitwise equal to the oracle."""
    m, n, k = shape
    plan = oz.Plan(num_moduli=nmod, scaling="W")
    A, B = _inputs(m, n, k, 0.5, 9)
    big = 1.0 - 2.0 ** -52
    A[0, :] = -big
    A[1, ::2] = big
    B[:, 0] = -big
    B[::3, 1] = big
    C = host(oz.dgemm(dev(A), dev(B), plan))
    ref = scheme.emulate(A, B, plan.moduli(), "W", keep=False)["C"]
    assert np.array_equal(C, ref)


@pytest.mark.parametrize("nmod", [24, 28, 32])
@pytest.mark.parametrize("phi", [0.5, 4.0])
def test_exact_form_of_reduce_both_paths(nmod, phi):
    """Kept bits above 62 (89, 102 and 116 per side here): workgroups whose
    entries all stay below 2^94 take the twelve-signed-digit form, the
    others the shift-table form; with phi = 4 one call holds both. The
    product is bitwise the oracle's."""
    import torch
    m, n, k = 200, 150, 300
    A, B = operand_pair(m, n, k, phi, 7)
    plan = oz.Plan(num_moduli=nmod, scaling="W")
    print("exact form", nmod, phi, plan.kept_bits(k), flush=True)
    C = host(oz.dgemm(dev(A), dev(B), plan))
    torch.cuda.synchronize()
    ref = scheme.emulate(A, B, plan.moduli(), "W", blas=True, keep=False)["C"]
    assert np.array_equal(C, ref)
    dA, dB = dev(A), dev(B)
    sa, sb = oz.scale(dA, dB, plan)
    pa, pb = oz.reduce(dA, dB, sa, sb, plan)
    PA, PB = oracle_planes(A, B, plan.moduli(), "W", plan.plane_dims(m, n, k))
    assert np.array_equal(from_blocked(host(pa)), PA)
    assert np.array_equal(from_blocked(host(pb)), PB)
