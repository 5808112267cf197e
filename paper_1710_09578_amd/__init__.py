"""Structured linear operators and FISTA on MI355X (gfx950).

The compute path is the HIP library ``libfm.so`` (C ABI in ``include/fm.h``);
``capi`` binds it entry point by entry point, ``operators`` offers the
paper's notation on top (``Circulant(c) @ x``, ``A.H``, ``Product``, ...),
``autograd`` the differentiable applications and unrolled FISTA.
"""

from . import autograd  # noqa: F401
from .capi import FmError, load  # noqa: F401
from .operators import (  # noqa: F401
    Batch,
    BlkDiag,
    Blocks,
    Circulant,
    Dense,
    Diag,
    Fourier,
    Hadamard,
    Kron,
    LFSRCirculant,
    MLToeplitz,
    Operator,
    Partial,
    Product,
    SelectRows,
    Sum,
    Toeplitz,
    calibration_build,
    calibration_load,
    calibration_table,
    compressed_ultrasound,
    fista,
    fista_options,
    omp,
    power_iteration,
)

__version__ = "0.1.0"
