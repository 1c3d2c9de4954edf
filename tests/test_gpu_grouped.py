"""GPU parity of grouped products (ozemu_group_*): every problem bitwise
equal to the oracle (small groups with ragged, empty and mixed-plan
problems) and to the single-product path (the 512-problem workload, with
oracle samples and the exact scaled error), and HIP-graph replays equal to
the eager run."""
import numpy as np
import pytest

from oracle import exact, scheme
from tests.gpu_util import cuda_ok, dev, host
from workloads import grouped_shapes, operand_pair

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a HIP device")]

oz = pytest.importorskip("paper_2609_37693_amd")


def _problems(shapes, phi, seed):
    out = []
    for p, (m, n, k) in enumerate(shapes):
        out.append(operand_pair(m, n, k, phi, seed + 2 * p))
    return out


def test_small_group_matches_oracle_mixed_plans():
    import torch
    rng = np.random.default_rng(4)
    shapes = [(int(rng.integers(1, 300)), int(rng.integers(1, 300)), int(rng.integers(1, 700)))
              for _ in range(18)]
    shapes += [(0, 5, 7), (6, 0, 7), (6, 5, 0), (257, 256, 64), (1, 1, 1)]
    plans = {"W14": oz.Plan(14, "W"), "W20": oz.Plan(20, "W"), "F53": oz.Plan(16, "F53"),
             "W10": oz.Plan(10, "W")}
    keys = list(plans)
    which = [keys[p % len(keys)] for p in range(len(shapes))]
    ops = _problems(shapes, 1.0, 30)
    g = oz.Group([dev(a) for a, _ in ops], [dev(b) for _, b in ops], [plans[w] for w in which])
    outs = g.run()
    torch.cuda.synchronize()
    for p, ((A, B), w) in enumerate(zip(ops, which)):
        pl = plans[w]
        mode = "F53" if w == "F53" else "W"
        C = host(outs[p])
        assert C.shape == (A.shape[0], B.shape[1])
        if A.shape[1] == 0:
            assert not C.any()
            continue
        if C.size == 0:
            continue
        ref = scheme.emulate(A, B, pl.moduli(), mode, keep=False)["C"]
        assert np.array_equal(C, ref), (p, shapes[p], w)


def test_group_special_values_and_strides():
    import torch
    plan = oz.Plan(16, "W")
    A1, B1 = operand_pair(70, 90, 50, 1.0, 5)
    A1[3, 7] = np.nan
    B1[:, 4] = 0.0
    A2, B2 = operand_pair(40, 30, 300, 4.0, 6)
    big = torch.zeros((40, 400), dtype=torch.float64, device="cuda")
    big[:, 5:305] = dev(A2)
    A2v = big[:, 5:305]  # leading dimension 400
    g = oz.Group([dev(A1), A2v], [dev(B1), dev(B2)], plan)
    o1, o2 = g.run()
    torch.cuda.synchronize()
    ms = plan.moduli()
    assert np.array_equal(host(o1), scheme.emulate(A1, B1, ms, "W", keep=False)["C"],
                          equal_nan=True)
    assert np.array_equal(host(o2), scheme.emulate(A2, B2, ms, "W", keep=False)["C"])


def test_group_graph_replays_match_eager():
    """The run captured in a HIP graph (one table copy from pinned memory,
    then kernels; no memset nodes) replays to the eager result, with eager
    work and synchronization between replays."""
    import torch
    shapes = grouped_shapes(24, seed=3, mn_hi=600, k_hi=900)
    ops = _problems(shapes, 1.0, 70)
    plan = oz.Plan(16, "W")
    g = oz.Group([dev(a) for a, _ in ops], [dev(b) for _, b in ops], plan)
    eager = [host(c).copy() for c in g.run()]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        g.run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        g.run()
    for rep in range(3):
        for c in g.outs:
            c.fill_(-1.0)
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for p, c in enumerate(g.outs):
            assert np.array_equal(host(c), eager[p]), (rep, p)
        del junk


def test_workload_512_problems_matches_single_path_and_oracle():
    """The batched workload: 512 problems, m, n ~ U[64, 2048], k ~ U[64,
    4096], phi = 1, sixteen moduli. Every output equals the single-product
    path bitwise; sampled rows x columns of 6 problems equal the oracle
    bitwise and meet the exact scaled error 2**-50."""
    import torch
    shapes = grouped_shapes(512, seed=0)
    plan = oz.Plan(16, "W")
    rng = np.random.default_rng(0)
    As, Bs = [], []
    for p, (m, n, k) in enumerate(shapes):
        A, B = operand_pair(m, n, k, 1.0, 1000 + 2 * p)
        As.append(dev(A))
        Bs.append(dev(B))
    g = oz.Group(As, Bs, plan)
    outs = g.run()
    torch.cuda.synchronize()
    for p in range(len(shapes)):
        single = oz.dgemm(As[p], Bs[p], plan)
        assert torch.equal(outs[p], single), p
    for p in rng.choice(len(shapes), 6, replace=False):
        m, n, k = shapes[p]
        rows = np.sort(rng.choice(m, min(m, 8), replace=False))
        cols = np.sort(rng.choice(n, min(n, 8), replace=False))
        A = host(As[p])[rows]
        B = np.ascontiguousarray(host(Bs[p])[:, cols])
        ref = scheme.emulate(A, B, plan.moduli(), "W", blas=True, keep=False)["C"]
        got = host(outs[p])[np.ix_(rows, cols)]
        assert np.array_equal(got, ref), p
        assert exact.scaled_error(got, A, B) <= 2.0 ** -50
