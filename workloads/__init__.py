"""Seeded synthetic inputs shaped like the compressed-sensing workloads.

This package only draws random numbers and arranges them into arrays. It holds
none of the operator or solver arithmetic, so both the CPU oracle (through the
tests) and the GPU path (through the tests and the benchmark) can be fed from it
without sharing any computation.

Block layout everywhere: a block of ``ncols`` column vectors of length ``rows``
is an array of shape ``(ncols, rows)``, one column per row of the array.
"""

from .gen import (  # noqa: F401
    cn,
    circulant_1024,
    compressed_sensing_65536,
    kron_hfg,
    toeplitz_batch,
    learn_circulant,
    many_columns,
    power_start,
    ultrasound,
)
