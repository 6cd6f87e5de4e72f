"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only builds inputs (parity-check matrices).  It holds none of the
trapping-set method's arithmetic: no decoding, no girth computation used by
either side, no pattern generation, no canonicalisation.
"""
from .codes import (  # noqa: F401
    Code,
    qc_code,
    csr_code,
    qc_random_shifts,
    qc_greedy_shifts,
    peg_regular,
    tiny_code,
    tiny_code_z8,
    peg1008_code,
    qc2640_code,
    table5_code1,
    batch_codes,
    serving_pool,
)
