"""Emulated-DGEMM throughput on one MI355X, next to native FP64 DGEMM.

Workload: C = A B with A, B FP64 8192 x 8192, entries U(-1/2, 1/2) *
exp(phi N(0, 1)) (phi = 0.5), emulated through INT8 residue channels
(one INT8 MFMA GEMM per modulus, INT32 accumulation). One step is one
whole emulated call: Scale, Reduce, the residue GEMMs with their fused
modular epilogue, and Reconstruct. Inputs are resident in HBM before the
timed region. Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--moduli N] [--scaling W|G|F53]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0      # MI355X dense INT8 MFMA, TOP/s
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 matrix, TFLOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--phi", type=float, default=0.5)
    ap.add_argument("--moduli", type=int, default=16)
    ap.add_argument("--scaling", default="W", choices=["W", "G", "F53"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=32,
                    help="rows of C in the CPU oracle's bounded sample")
    ap.add_argument("--no-native", action="store_true")
    ap.add_argument("--format", default="E4M3", choices=["E4M3", "E2M3", "E2M1"],
                    help="fp workload: float alphabet of the limb channels")
    ap.add_argument("--gemms-list", default="0",
                    help="fp workload: comma-separated GEMM counts (0: least count for the "
                         "window at K = 16384)")
    ap.add_argument("--workload", default="dgemm",
                    choices=["dgemm", "mlp", "grouped", "fp", "sweep", "blocked"],
                    help="dgemm: the 8192^3 emulated DGEMM (default); mlp: one training "
                         "step of a 4-layer tanh MLP through the cached-residue backward; "
                         "grouped: 512 uneven products as one grouped run in a HIP graph; "
                         "sweep: the 8192^3 DGEMM over moduli counts and phi, time and "
                         "exact scaled error on sampled entries; blocked: the blocked call "
                         "at an inner dimension beyond the INT32 accumulation cap")
    ap.add_argument("--moduli-list", default="10,11,12,13,14,15,16,17,18,19,20",
                    help="sweep: moduli counts")
    ap.add_argument("--phi-list", default="0.5,4", help="sweep: phi values")
    ap.add_argument("--sample", type=int, default=8,
                    help="sweep: rows and columns of C whose exact error is computed")
    ap.add_argument("--problems", type=int, default=512)
    ap.add_argument("--group-moduli", type=int, default=None,
                    help="grouped: one moduli count for every problem (default: chosen per "
                         "problem for 55 kept bits)")
    ap.add_argument("--blocked-mn", type=int, default=4096, help="blocked: m = n")
    ap.add_argument("--blocked-k", type=int, default=262144, help="blocked: inner dimension")
    ap.add_argument("--k-slab", type=int, default=0,
                    help="blocked: slab length (0: the fewest equal slabs within the "
                         "accumulation cap)")
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--width", type=int, default=4096)
    return ap.parse_args()


def time_stream(fn, iters, warmup):
    """Mean ms per call of fn() with HIP events on torch's current stream,
    the stream every library call is launched on."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(iters):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / iters


GEMM_SOURCES = ("paper_2609_37693_amd/csrc/gemm_i8.hip",
                "paper_2609_37693_amd/csrc/ozemu_internal.hpp")
TRAFFIC_PROFILE = os.path.join("profiles", "residue_gemm_8192x16.md")


def committed_traffic(n, num_moduli):
    """HBM bytes per residue-GEMM launch measured with rocprofv3 (FETCH_SIZE
    and WRITE_SIZE, calibrated on a streaming kernel of known size) and
    recorded in the profile summary; None when the workload differs or the
    kernel source changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, TRAFFIC_PROFILE)).read()
    except OSError:
        return None
    found = re.search(r"```json\n(\{.*?\})\n```", text, re.S)
    if not found:
        return None
    rec = json.loads(found.group(1))
    h = hashlib.sha256()
    for f in GEMM_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != rec.get("source_hash"):
        return None
    if rec.get("n") != n or rec.get("moduli") != num_moduli:
        return None
    return rec.get("traffic_bytes")


def cpu_baseline(A, B, moduli, mode, rows):
    """The CPU oracle, as it stands, on a bounded sample: rows [0, rows) of
    C at full K and N (every step of the scheme, B's scaling and residues
    over all of B included). Rate in emulated TFLOP/s over the sample."""
    from oracle import scheme
    t0 = time.perf_counter()
    scheme.emulate(A[:rows], B, moduli, mode, blas=True, keep=False)
    dt = time.perf_counter() - t0
    n, k = B.shape[1], B.shape[0]
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    # native FP64 DGEMM on the same host (numpy's BLAS), 1024 rows of C
    r2 = min(1024, A.shape[0])
    A2 = np.ascontiguousarray(A[:r2])
    A2 @ B
    t1 = time.perf_counter()
    A2 @ B
    dt2 = time.perf_counter() - t1
    return {"value": 2.0 * rows * n * k / dt / 1e12, "unit": "TFLOP/s", "cores": cores,
            "native_cpu_dgemm_tflops": 2.0 * r2 * n * k / dt2 / 1e12,
            "kind": "oracle",
            "sample": "rows 0..%d of C at %dx%dx%d (%s, %d moduli): %.1f s on %s; BLAS uses "
                      "all cores, the rest of the oracle one" % (rows, rows, n, k, mode,
                                                                 len(moduli), dt,
                                                                 platform.processor() or
                                                                 platform.machine())}


def _fixed_row(v):
    """Exact integers r and one exponent E with v[k] = r[k] 2^E (finite v)."""
    import math
    parts = [math.frexp(float(x)) for x in v]
    ints = [(int(fr * (1 << 53)), ex - 53) for fr, ex in parts]
    E = min(ex for m, ex in ints if m) if any(m for m, _ in ints) else 0
    return [m << (ex - E) if m else 0 for m, ex in ints], E


def exact_scaled_error(C, A, B, rows, cols):
    """max over the sampled entries of |C_ij - (AB)_ij| / (|A||B|)_ij, each
    ratio exact in integers before its final conversion (0/0 counts 0)."""
    from fractions import Fraction
    worst = 0.0
    Bc = {j: _fixed_row(B[:, j]) for j in cols}
    for i in rows:
        ra, Ea = _fixed_row(A[i])
        for j in cols:
            rb, Eb = Bc[j]
            ex = sum(x * y for x, y in zip(ra, rb))
            den = sum(abs(x) * abs(y) for x, y in zip(ra, rb))
            scale = Fraction(2) ** (Ea + Eb)
            diff = abs(Fraction(float(C[i, j])) - ex * scale)
            if den == 0:
                err = 0.0 if diff == 0 else float("inf")
            else:
                err = float(diff / (den * scale))
            worst = max(worst, err)
    return worst


def _ldexp_exact(X, e):
    """X * 2**e elementwise (e an integer tensor broadcasting against X), in
    two power-of-two steps so that neither factor leaves the FP64 range; exact
    whenever the intermediate and the result are normal or the result is the
    truncation of a representable value."""
    import torch
    h = torch.div(e, 2, rounding_mode="floor")
    return X * torch.pow(2.0, h.to(torch.float64)) * torch.pow(2.0, (e - h).to(torch.float64))


def certified_error_bound(A, B, C, beta_a, beta_b):
    """Certified per-entry bound on |C - AB| / (|A||B|) over the whole matrix.

    Valid for C = RN(A'B' 2^-(s_i+t_j)) with A' = trunc(A 2^s), B' =
    trunc(B 2^t) and the shifts of the definition: s_i = beta_a - e_i, e_i
    the frexp exponent of row i's largest magnitude (0 for a zero row),
    likewise t_j over the columns of B (Sec. V-A, phases 1 and 4). With
    Ahat = A' 2^-s and dA = A - Ahat (both exact in FP64, dA holds the bits
    of A below 2^-s_i), AB - Ahat Bhat = dA B + Ahat dB, so

        |C - AB| <= |dA||B| + |Ahat||dB| + 2^-53 |C|.

    The three products of nonnegative matrices are FP64 GEMMs with relative
    error at most gamma_k = k u / (1 - k u), u = 2^-53, whatever the
    summation order: numerators are raised by that factor and the
    denominator |A||B| lowered. Returns (bound tensor, s, t); entries whose
    row of A or column of B is zero get 0 when C is 0 there, inf otherwise.
    """
    import torch
    k = A.shape[1]
    u = 2.0 ** -53
    gam = k * u / (1.0 - k * u)
    ra = A.abs().amax(dim=1) if k else torch.zeros(A.shape[0], dtype=A.dtype, device=A.device)
    cb = B.abs().amax(dim=0) if k else torch.zeros(B.shape[1], dtype=B.dtype, device=B.device)
    s = torch.where(ra > 0, beta_a - torch.frexp(ra).exponent, 0).to(torch.int64)
    t = torch.where(cb > 0, beta_b - torch.frexp(cb).exponent, 0).to(torch.int64)
    Ah = _ldexp_exact(torch.trunc(_ldexp_exact(A, s[:, None])), -s[:, None])
    Bh = _ldexp_exact(torch.trunc(_ldexp_exact(B, t[None, :])), -t[None, :])
    num = (A - Ah).abs() @ B.abs()
    num += Ah.abs() @ (B - Bh).abs()
    num *= (1.0 + 2.0 * gam) * (1.0 + u)
    num += C.abs() * (u * (1.0 + u))
    den = (A.abs() @ B.abs()) * (1.0 - gam)
    pos = den > 0
    bound = torch.where(pos, num / torch.where(pos, den, 1.0),
                        torch.where(C == 0, 0.0, float("inf")))
    return bound, s, t


def sweep_main(args):
    """The 8192^3 emulated DGEMM for every moduli count and phi in the
    lists: whole-call time, the exact scaled error over sampled rows x
    columns of C, and native FP64 beside it. The headline per phi is the
    fastest count whose sampled error is within 2^-50."""
    import torch
    import paper_2609_37693_amd as oz
    from workloads import operand_pair

    n = args.size
    mods = [int(x) for x in args.moduli_list.split(",") if x]
    phis = [float(x) for x in args.phi_list.split(",") if x]
    rng = np.random.default_rng(args.seed + 99)
    rows = sorted(rng.choice(n, args.sample, replace=False).tolist())
    cols = sorted(rng.choice(n, args.sample, replace=False).tolist())
    flops = 2.0 * n * n * n
    curve, best = [], {}
    for phi in phis:
        A_h, B_h = operand_pair(n, n, n, phi, args.seed)
        A = torch.from_numpy(A_h).cuda()
        B = torch.from_numpy(B_h).cuda()
        C = torch.empty((n, n), dtype=torch.float64, device="cuda")
        ref = torch.empty_like(C)
        native_ms = time_stream(lambda: torch.matmul(A, B, out=ref), 5, 2)
        for nm in mods:
            plan = oz.Plan(num_moduli=nm, scaling=args.scaling)
            ws = torch.empty(plan.workspace_size(n, n, n), dtype=torch.uint8, device="cuda")
            ms = time_stream(lambda: oz.dgemm(A, B, plan, out=C, workspace=ws), args.steps,
                             args.warmup)
            torch.cuda.synchronize()
            Cs = C[rows][:, cols].cpu().numpy()
            sub = {(i, j): Cs[a, b] for a, i in enumerate(rows) for b, j in enumerate(cols)}
            err = exact_scaled_error(_SubC(sub), A_h, B_h, rows, cols)
            try:
                kept = list(plan.kept_bits(n))
            except oz.OzemuError:  # mode G: bits per row and column
                kept = None
            rec = {"phi": phi, "moduli": nm, "kept_bits": kept, "ms": ms,
                   "tflops": flops / (ms * 1e-3) / 1e12, "native_ms": native_ms,
                   "speedup_vs_native": native_ms / ms, "scaled_error_sample": err,
                   "log2_error": (float(np.log2(err)) if err > 0 else None)}
            curve.append(rec)
            print("phi %g moduli %d: %.3f ms, error 2^%s" % (phi, nm, ms, rec["log2_error"]),
                  file=sys.stderr, flush=True)
            if err <= 2.0 ** -50 and (phi not in best or ms < best[phi]["ms"]):
                best[phi] = rec
            del ws
    head = best.get(phis[0]) or curve[0]
    out = {
        "metric": "emulated DGEMM TFLOP/s vs native FP64 MFMA at 8192^3, at <=2^-50 scaled error",
        "value": head["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int8", "data": "synthetic",
        "config": {"workload": "emulated DGEMM m=n=k=%d over moduli counts %s and phi %s, "
                               "INT8 residue path, mode %s" % (n, args.moduli_list,
                                                               args.phi_list, args.scaling),
                   "m": n, "n": n, "k": n, "sample": "%d x %d entries of C" % (len(rows),
                                                                                len(cols))},
        "least_error_2^-50": {str(p): {"moduli": r["moduli"], "ms": r["ms"],
                                       "speedup_vs_native": r["speedup_vs_native"]}
                              for p, r in best.items()},
        "sweep": curve,
    }
    print(json.dumps(out), flush=True)


class _SubC:
    """C_ij lookup over the sampled entries only."""

    def __init__(self, d):
        self.d = d

    def __getitem__(self, ij):
        return self.d[ij]


def mlp_main(args):
    """One training step of a 4-layer FP64 MLP (no bias, tanh between
    layers, loss 1/2 ||H_4 - T||^2): forward through the cached-residue
    emulated product, backward dX = dY W^T and dW = X^T dY through the
    cached planes. Twelve products of batch x width x width per step."""
    import torch
    import paper_2609_37693_amd as oz
    from paper_2609_37693_amd.autograd import emulated_matmul
    from workloads import phi_matrix

    B, Wd = args.batch, args.width
    X = torch.from_numpy(phi_matrix(B, Wd, 1.0, args.seed)).cuda()
    T = torch.from_numpy(np.random.default_rng(args.seed + 5).standard_normal((B, Wd))).cuda()
    Ws = [torch.from_numpy(phi_matrix(Wd, Wd, 1.0, args.seed + 10 + i) * 2.0 ** -6).cuda()
          .requires_grad_() for i in range(4)]
    plan = oz.Plan(num_moduli=args.moduli, scaling="W")

    def step(emulated=True):
        for w in Ws:
            w.grad = None
        h = X
        for i, w in enumerate(Ws):
            h = emulated_matmul(h, w, plan) if emulated else h @ w
            if i < 3:
                h = torch.tanh(h)
        loss = 0.5 * ((h - T) ** 2).sum()
        loss.backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    flops = 12 * 2.0 * B * Wd * Wd
    g_emu = [w.grad.clone() for w in Ws]
    native_ms = time_stream(lambda: step(False), max(3, args.steps // 2), 1)
    step(False)
    torch.cuda.synchronize()
    rel = max(float(torch.linalg.norm(a - w.grad) / torch.linalg.norm(w.grad))
              for a, w in zip(g_emu, Ws))
    out = {
        "metric": "emulated FP64 MLP training step TFLOP/s (forward + cached-residue backward)",
        "value": flops / (ms * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "4-layer tanh MLP, batch %d, width %d, FP64, %d moduli, "
                               "cached-residue backward" % (B, Wd, args.moduli),
                   "batch": B, "width": Wd, "moduli": args.moduli},
        "native_fp64": {"ms": native_ms, "value": flops / (native_ms * 1e-3) / 1e12},
        "speedup_vs_native": native_ms / ms,
        "max_rel_frobenius_grad_vs_native": rel,
    }
    print(json.dumps(out), flush=True)


def grouped_main(args):
    """512 independent products, m, n ~ U[64, 2048], k ~ U[64, 4096], phi = 1
    entries, as one grouped run (persistent residue GEMM) captured in a HIP
    graph; native FP64 is the same products as torch.matmul calls, also
    captured in a graph."""
    import torch
    import paper_2609_37693_amd as oz
    from paper_2609_37693_amd import autotune
    from workloads import grouped_shapes, operand_pair

    shapes = grouped_shapes(args.problems, seed=args.seed)
    As, Bs = [], []
    for p, (m, n, k) in enumerate(shapes):
        A, B = operand_pair(m, n, k, 1.0, 1000 + 2 * p)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
    plans = autotune.plans_for(shapes, args.group_moduli)
    group = oz.Group(As, Bs, plans)
    flops = sum(2.0 * m * n * k for m, n, k in shapes)

    def graph_of(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        return g

    g_emu = graph_of(group.run)
    for _ in range(args.warmup):
        g_emu.replay()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        g_emu.replay()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    eager_ms = time_stream(group.run, max(2, args.steps // 4), 1)

    refs = [torch.empty_like(c) for c in group.outs]

    def native():
        for A, B, R in zip(As, Bs, refs):
            torch.matmul(A, B, out=R)
    g_nat = graph_of(native)
    native_ms = time_stream(g_nat.replay, max(3, args.steps // 2), 1)
    g_nat.replay()
    torch.cuda.synchronize()
    num = sum(float(torch.linalg.norm(c - r) ** 2) for c, r in zip(group.outs, refs))
    den = sum(float(torch.linalg.norm(r) ** 2) for r in refs)
    counts = {}
    for pl in plans:
        counts[len(pl.moduli())] = counts.get(len(pl.moduli()), 0) + 1
    out = {
        "metric": "emulated grouped DGEMM TFLOP/s (512 uneven FP64 products, one grouped run)",
        "value": flops / (ms * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "%d products, m, n ~ U[64, 2048], k ~ U[64, 4096], phi = 1, "
                               "HIP graph" % len(shapes), "problems": len(shapes),
                   "tflop": flops / 1e12, "moduli_per_problem": counts},
        "eager_ms": eager_ms,
        "native_fp64": {"ms": native_ms, "value": flops / (native_ms * 1e-3) / 1e12},
        "speedup_vs_native": native_ms / ms,
        "rel_frobenius_vs_native": (num / den) ** 0.5,
    }
    print(json.dumps(out), flush=True)


def fp_main(args):
    """FP64 products through FP8 E4M3 / FP4 E2M1 limb channels (FP32
    accumulation, slabs of 16384 terms) at m = n = k = size (16384 unless
    --size is given), phi = 1: one whole emulated call per step for every
    GEMM count in --gemms-list, with the exact scaled error on 64 sampled
    entries and the relative Frobenius difference from native FP64."""
    import torch
    import paper_2609_37693_amd as oz
    from oracle import exact
    from workloads import operand_pair

    n = args.size if args.size != 8192 else 16384
    A_h, B_h = operand_pair(n, n, n, 1.0, args.seed)
    A = torch.from_numpy(A_h).cuda()
    B = torch.from_numpy(B_h).cuda()
    ref = A @ B
    native_ms = time_stream(lambda: torch.matmul(A, B, out=ref), max(3, args.steps // 2), 1)
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(n, 8, replace=False))
    cols = np.sort(rng.choice(n, 8, replace=False))
    As = np.ascontiguousarray(A_h[rows])
    Bs = np.ascontiguousarray(B_h[:, cols])
    flops = 2.0 * n ** 3
    peak = 5000.0 if args.format == "E4M3" else 10100.0
    curve = []
    for g in [int(x) for x in args.gemms_list.split(",")]:
        plan = oz.Plan(format=args.format, gemms=g, k_slab=16384)
        C = torch.empty((n, n), dtype=torch.float64, device="cuda")
        ws = torch.empty(plan.workspace_size(n, n, n), dtype=torch.uint8, device="cuda")
        ms = time_stream(lambda: oz.dgemm(A, B, plan, out=C, workspace=ws), args.steps,
                         args.warmup)
        torch.cuda.synchronize()
        Q = plan.gemms()
        got = C[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()].cpu().numpy()
        err = exact.scaled_error(got, As, Bs)
        rel = float(torch.linalg.norm(C - ref) / torch.linalg.norm(ref))
        curve.append({"gemms": Q, "channels": len(plan.channels()),
                      "kept_bits": list(plan.kept_bits(n)), "ms": ms,
                      "tflops": flops / (ms * 1e-3) / 1e12,
                      "lowp_tflops": 2.0 * Q * n ** 3 / (ms * 1e-3) / 1e12,
                      "scaled_error_sample": err, "rel_frobenius_vs_native": rel,
                      "speedup_vs_native": native_ms / ms})
        del C, ws
        torch.cuda.empty_cache()
    head = curve[0]
    out = {
        "metric": "emulated DGEMM TFLOP/s through %s limb channels at %d^3" % (args.format, n),
        "value": head["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"E4M3": "fp8", "E2M3": "fp6", "E2M1": "fp4"}[args.format], "data": "synthetic",
        "config": {"workload": "emulated DGEMM m=n=k=%d, phi = 1, %s channels, FP32 "
                               "accumulation, slabs of 16384" % (n, args.format),
                   "format": args.format, "gemms": head["gemms"]},
        "roofline_whole_call": {"bound": "mfma", "achieved": head["lowp_tflops"], "peak": peak,
                                "unit": "TFLOP/s", "frac": head["lowp_tflops"] / peak},
        "native_fp64": {"ms": native_ms, "value": flops / (native_ms * 1e-3) / 1e12},
        "curve": curve,
    }
    print(json.dumps(out), flush=True)


def blocked_main(args):
    """The blocked call at m = n = 4096 and K = 262144 (twice the INT32
    accumulation cap of 16 INT8 moduli), slabs at the cap, mode W; native
    FP64 on the same operands; exact scaled error on sampled entries."""
    import torch
    import paper_2609_37693_amd as oz
    from workloads import operand_pair
    n, k = args.blocked_mn, args.blocked_k
    A_h, B_h = operand_pair(n, n, k, args.phi, args.seed)
    A = torch.from_numpy(A_h).cuda()
    B = torch.from_numpy(B_h).cuda()
    plan = oz.Plan(num_moduli=args.moduli, scaling=args.scaling)
    cap = plan.k_max()
    if args.k_slab:
        k_slab = args.k_slab
    else:  # equal slabs, whole 64-term K steps, within the cap
        count = -(-k // cap)
        k_slab = min(cap, -(-(-(-k // count)) // 64) * 64)
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ws = torch.empty(oz.blocked_workspace_size(plan, n, n, k, k_slab), dtype=torch.uint8,
                     device="cuda")
    run = lambda: oz.dgemm_blocked(A, B, plan, k_slab, out=C, workspace=ws)
    ms = time_stream(run, args.steps, args.warmup)
    run()
    torch.cuda.synchronize()
    ref = torch.empty_like(C)
    native_ms = time_stream(lambda: torch.matmul(A, B, out=ref), max(3, args.steps // 2), 1)
    rel = float(torch.linalg.norm(C - ref) / torch.linalg.norm(ref))
    rng = np.random.default_rng(5)
    rows = sorted(rng.choice(n, 2, replace=False).tolist())
    cols = sorted(rng.choice(n, 2, replace=False).tolist())
    err = exact_scaled_error(C.cpu().numpy(), A_h, B_h, rows, cols)
    flops = 2.0 * n * n * k
    out = {
        "metric": "emulated DGEMM TFLOP/s, blocked call beyond the INT32 accumulation cap",
        "value": flops / (ms * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "blocked emulated DGEMM m = n = %d, k = %d in slabs of %d, "
                               "phi = %g, %d moduli, mode %s" % (n, k, k_slab, args.phi,
                                                                 args.moduli, args.scaling),
                   "m": n, "n": n, "k": k, "k_slab": k_slab, "kept_bits": list(plan.kept_bits(k))},
        "native_fp64": {"ms": native_ms, "value": flops / (native_ms * 1e-3) / 1e12},
        "speedup_vs_native": native_ms / ms,
        "rel_frobenius_vs_native": rel,
        "scaled_error_sample": err,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if args.workload != "dgemm":
        if not torch.cuda.is_available():
            print("no HIP device", file=sys.stderr)
            sys.exit(1)
        return {"mlp": mlp_main, "grouped": grouped_main, "fp": fp_main,
                "sweep": sweep_main, "blocked": blocked_main}[args.workload](args)
    import paper_2609_37693_amd as oz
    from workloads import operand_pair

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    n = args.size
    A_h, B_h = operand_pair(n, n, n, args.phi, args.seed)
    A = torch.from_numpy(A_h).cuda()
    B = torch.from_numpy(B_h).cuda()
    plan = oz.Plan(num_moduli=args.moduli, scaling=args.scaling)
    moduli = plan.moduli()
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ws = torch.empty(plan.workspace_size(n, n, n), dtype=torch.uint8, device="cuda")

    def step():
        oz.dgemm(A, B, plan, out=C, workspace=ws)

    # whole-call throughput: W warmup calls, then exactly K timed calls
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    flops = 2.0 * n * n * n
    value = flops / (ms * 1e-3) / 1e12

    # dominant kernel: the residue GEMMs, one launch over all moduli
    sa, sb = oz.scale(A, B, plan)
    pa, pb = oz.reduce(A, B, sa, sb, plan)
    z = torch.empty((len(moduli),) + tuple(plan.plane_dims(n, n, n)[:2]), dtype=torch.uint8,
                    device="cuda")
    lib = oz._lib.load()
    import ctypes as C_

    def gemm_only():
        oz._lib.check(lib.ozemu_residue_gemm(plan.handle, oz._stream_ptr(), n, n, n,
                                             C_.c_void_p(pa.data_ptr()),
                                             C_.c_void_p(pb.data_ptr()),
                                             C_.c_void_p(z.data_ptr())))
    gemm_ms = time_stream(gemm_only, max(5, args.steps // 2), 2)
    ops = 2.0 * len(moduli) * n * n * n
    achieved = ops / (gemm_ms * 1e-3) / 1e12

    # per-phase times (synchronized separately, as in a profile)
    phases = {
        "scale": time_stream(lambda: oz.scale(A, B, plan), 5, 1),
        "reduce": time_stream(lambda: oz.reduce(A, B, sa, sb, plan), 5, 1),
        "residue_gemm": gemm_ms,
        "reconstruct": time_stream(lambda: oz.reconstruct(z, sa, sb, n, n, n, plan, out=C), 5, 1),
    }

    # accuracy against native FP64 on the same GPU
    step()
    torch.cuda.synchronize()
    native_ms = None
    ref = A @ B
    if not args.no_native:
        native_ms = time_stream(lambda: torch.matmul(A, B, out=ref), max(5, args.steps // 2), 2)
    rel_fro = float(torch.linalg.norm(C - ref) / torch.linalg.norm(ref))
    absAB = A.abs() @ B.abs()
    scaled_vs_native = float(torch.max((C - ref).abs() / absAB))
    del absAB
    # certified bound on every entry (valid for the shifts of the definition,
    # checked against the library's own)
    certified = None
    shifts_ok = None
    if args.scaling != "G":
        ba, bb = plan.kept_bits(n)
        bound, s_def, t_def = certified_error_bound(A, B, C, ba, bb)
        shifts_ok = bool(torch.equal(s_def, sa.to(torch.int64)) and
                         torch.equal(t_def, sb.to(torch.int64)))
        certified = float(bound.max())
        del bound

    out = {
        "metric": "emulated DGEMM TFLOP/s vs native FP64 MFMA at 8192^3, at <=2^-50 scaled error",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "emulated DGEMM m=n=k=%d, FP64 entries U(-1/2,1/2)*exp(%g*N(0,1)), "
                               "INT8 residue path" % (n, args.phi),
                   "m": n, "n": n, "k": n, "phi": args.phi, "moduli": len(moduli),
                   "scaling_mode": args.scaling, "seed": args.seed},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS,
                     "unit": "TFLOP/s", "frac": achieved / INT8_PEAK_TOPS,
                     "traffic": committed_traffic(n, len(moduli)),
                     "kernel": "residue_gemm_kernel (INT8 MFMA, all moduli, one launch)",
                     "kernel_ms": gemm_ms},
        "phases_ms": phases,
        "native_fp64": {"ms": native_ms,
                        "value": (flops / (native_ms * 1e-3) / 1e12) if native_ms else None,
                        "frac_of_peak": (flops / (native_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS)
                        if native_ms else None},
        "speedup_vs_native": (native_ms / ms) if native_ms else None,
        "rel_frobenius_vs_native": rel_fro,
        "max_scaled_diff_vs_native": scaled_vs_native,
        "certified_max_scaled_error": certified,
        "shifts_match_definition": shifts_ok,
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A_h, B_h, moduli, args.scaling, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
