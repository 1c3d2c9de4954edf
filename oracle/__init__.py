"""CPU oracle for FP64 GEMM emulation through residue (Ozaki II) schemes.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is a plain, slow and obviously correct statement of what the
emulation computes, written from the paper (Mazumder, Calotoiu, Hoefler,
"FP64 Is All You Want, INT8 Is All You Need, FP4/6/8 Is All You Have").
It shares no code, tables or constants with the HIP library. Integers are
exact Python ints or numpy int64 where the bounds stated next to each use
keep them below 2**63; floating point is only used where it is exact
(power-of-two scaling, integer-valued BLAS sums below 2**53) or for the
single final rounding, which CPython performs correctly for int / int.

Modules
-------
``exact``     exact integer matrix products, the exact rational product AB
              and the scaled error metric.
``moduli``    pairwise-coprime modulus sets, CRT window, accumulation caps,
              counting bound (Sec. III-C, III-F, IV-C).
``scheme``    the INT8 residue scheme step by step: exponents, kept bits,
              truncation, balanced residues, residue GEMMs, CRT, rounding
              (Sec. II-A, II-B, V-A).
``alphabets`` the integer alphabets of the low-precision float formats
              (Sec. III-A).
``forms``     limb channels, Toom and schoolbook forms, encoding tables and
              the reduce-then-combine epilogue (Sec. III-A, III-B, III-C).

Parity status of every function is stated in its module header; the pins
that check each function against the paper live in ``tests/test_oracle_*.py``.
"""
