"""Seeded generators for the benchmark and parity workloads.

Every generator returns plain arrays (NumPy, or torch tensors for the two very
large blocks that are drawn directly on a device). Nothing here applies an
operator or runs a solver: measurements ``b = A x + noise`` are formed by the
caller, with the oracle in the tests and with the library in the benchmark.

Random-number conventions (one reading per quantity, applied everywhere):

* standard complex Gaussian CN(0,1): real and imaginary parts each N(0, 1/2);
* sparse amplitudes: real N(0,1) stored as complex;
* Rademacher generator: real +-1 stored as complex;
* dense Kronecker factor: real N(0, 1/32) stored as complex;
* index sets (supports, selected rows): uniform without replacement, sorted
  ascending, stored as int32.

Large workloads derive one independent stream per operator or per column from
``numpy.random.default_rng([seed, k, purpose])`` so that any subset can be
regenerated on its own for a sampled check.
"""

from __future__ import annotations

import math

import numpy as np

C64 = np.complex64


def cn(rng: np.random.Generator, shape) -> np.ndarray:
    """Standard complex Gaussian CN(0,1) rounded to complex64."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return ((re + 1j * im) * math.sqrt(0.5)).astype(C64)


def _sorted_subset(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)


def _sparse_block(rng: np.random.Generator, n: int, k: int, ncols: int) -> np.ndarray:
    """``ncols`` k-sparse vectors of length n with real N(0,1) amplitudes."""
    x = np.zeros((ncols, n), dtype=C64)
    for j in range(ncols):
        supp = _sorted_subset(rng, n, k)
        x[j, supp] = rng.standard_normal(k).astype(np.float32)
    return x


def circulant_1024(ncols: int = 16, n: int = 1024, seed: int = 0):
    """Circulant N=1024 with a CN(0,1) generator and CN(0,1) columns.

    Returns ``(c, X)``: c of shape (n,), X of shape (ncols, n); X is drawn after
    c from the same stream.
    """
    rng = np.random.default_rng(seed)
    c = cn(rng, n)
    x = cn(rng, (ncols, n))
    return c, x


def compressed_sensing_65536(n: int = 65536, m: int = 4096, k: int = 64,
                             sigma: float = 1e-3, ncols: int = 1, seed: int = 1):
    """Row-selected circulant compressed sensing problem.

    Returns a dict with the Rademacher generator ``c`` (n,), the selected rows
    ``rows`` (m,), the sparse ground truth ``x_true`` (ncols, n) and the noise
    ``noise`` (ncols, m) already scaled by sigma.
    """
    rng = np.random.default_rng(seed)
    c = np.where(rng.integers(0, 2, n) == 1, 1.0, -1.0).astype(C64)
    rows = _sorted_subset(rng, n, m)
    x_true = _sparse_block(rng, n, k, ncols)
    noise = (sigma * cn(rng, (ncols, m)).astype(np.complex128)).astype(C64)
    return {"c": c, "rows": rows, "x_true": x_true, "noise": noise, "sigma": sigma}


def kron_hfg(ncols: int = 64, nh: int = 1024, nf: int = 256, ng: int = 32,
             seed: int = 2, device=None):
    """Kron(Hadamard nh, Fourier nf, dense ng x ng) workload.

    Returns ``(G, X)``: the dense factor G (ng, ng) as real N(0, 1/ng) in
    complex64, and the block X of shape (ncols, nh*nf*ng). With ``device`` set
    (a torch device), X is drawn there by torch's seeded generator (the block
    is 4 GiB at full size); otherwise it is drawn on the host, one stream per
    column.
    """
    rng = np.random.default_rng([seed, 0])
    g = (rng.standard_normal((ng, ng)) / math.sqrt(ng)).astype(np.float32).astype(C64)
    rows = nh * nf * ng
    if device is None:
        x = np.empty((ncols, rows), dtype=C64)
        for j in range(ncols):
            x[j] = cn(np.random.default_rng([seed, 1, j]), rows)
        return g, x
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    x = torch.randn((ncols, rows), dtype=torch.complex64, device=device, generator=gen)
    return g, x


def toeplitz_batch(nops: int = 512, nmin: int = 256, nmax: int = 65536,
                   max_cols: int = 32, seed: int = 3, with_fista: bool = False,
                   sigma: float = 1e-3, ops=None):
    """Batch of square Toeplitz operators with log-uniform sizes.

    Sizes N_i = round(exp(U[ln nmin, ln nmax])) and column counts
    n_i ~ U{1..max_cols} come from one stream; each operator then has its own
    stream for its first column ``col``, first row ``row`` (row[0] is not used:
    the first column defines the diagonal), input block ``x`` (n_i, N_i) and,
    with ``with_fista``, sparse truth ``x_true`` (K_i = N_i // 256 nonzeros per
    column) and scaled noise ``noise``.

    ``ops`` restricts the per-operator arrays to a subset of indices (the sizes
    of all operators are always returned).
    """
    rng = np.random.default_rng([seed, 0])
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nops))).astype(np.int64)
    ncols = rng.integers(1, max_cols + 1, nops).astype(np.int64)
    out = {"sizes": sizes, "ncols": ncols, "ops": {}}
    for i in (range(nops) if ops is None else ops):
        r = np.random.default_rng([seed, 1, i])
        n = int(sizes[i])
        d = {"col": cn(r, n), "row": cn(r, n), "x": cn(r, (int(ncols[i]), n))}
        if with_fista:
            d["x_true"] = _sparse_block(r, n, max(n // 256, 1), int(ncols[i]))
            d["noise"] = (sigma * cn(r, (int(ncols[i]), n)).astype(np.complex128)).astype(C64)
        out["ops"][i] = d
    return out


def learn_circulant(n: int = 16384, m: int = 2048, pairs: int = 256, k: int = 32,
                    sigma: float = 1e-3):
    """Learning a circulant generator through unrolled FISTA.

    Returns c_true (seed 41), c_init (seed 42), selected rows (seed 43) and
    ``pairs`` sparse vectors x_p with their scaled noise (seed 44).
    """
    c_true = cn(np.random.default_rng(41), n)
    c_init = cn(np.random.default_rng(42), n)
    rows = _sorted_subset(np.random.default_rng(43), n, m)
    r = np.random.default_rng(44)
    x = _sparse_block(r, n, k, pairs)
    noise = (sigma * cn(r, (pairs, m)).astype(np.complex128)).astype(C64)
    return {"c_true": c_true, "c_init": c_init, "rows": rows, "x": x, "noise": noise}


def many_columns(ncols: int = 65536, n: int = 1024, seed: int = 5, device=None):
    """The 1024-point circulant generator of ``circulant_1024`` with a wide
    block of CN(0,1) columns (drawn by torch's seeded generator on ``device``
    when given)."""
    c, _ = circulant_1024(1, n)
    if device is None:
        return c, cn(np.random.default_rng(seed), (ncols, n))
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return c, torch.randn((ncols, n), dtype=torch.complex64, device=device, generator=gen)


def ultrasound(n1: int = 32, n2: int = 32, n3: int = 512, nf: int = 1, k: int = 32,
               sigma: float = 1e-3, ncols: int = 1, seed: int = 7, blocks=None):
    """Synthetic inputs shaped like the compressed ultrasound model
    b = Psi H x + n: H is an n1 x n1 grid of 2-level Toeplitz blocks (levels
    n2, n3), Psi keeps nf Fourier coefficients of each of the n1 n2 A-scans
    of n3 samples.

    Returns a dict with the block generators ``t`` (n1, n1, 2 n2 - 1, 2 n3 - 1),
    CN(0,1) / sqrt(n1 n2 n3) each from its own stream [seed, 1, i, j] (only the
    blocks in ``blocks``, a list of (i, j), when given; the others stay zero),
    the kept Fourier rows ``psi_rows`` (n1 n2, nf) per A-scan, the sparse
    ground truth ``x_true`` (ncols, n1 n2 n3) with k real N(0,1) amplitudes
    and the noise ``noise`` (ncols, n1 n2 nf) already scaled by sigma.
    """
    rng = np.random.default_rng([seed, 0])
    psi_rows = np.stack([_sorted_subset(rng, n3, nf) for _ in range(n1 * n2)])
    x_true = _sparse_block(rng, n1 * n2 * n3, k, ncols)
    noise = (sigma * cn(rng, (ncols, n1 * n2 * nf)).astype(np.complex128)).astype(C64)
    t = np.zeros((n1, n1, 2 * n2 - 1, 2 * n3 - 1), dtype=C64)
    scale = 1.0 / math.sqrt(n1 * n2 * n3)
    for i, j in (blocks if blocks is not None else [(i, j) for i in range(n1) for j in range(n1)]):
        t[i, j] = (cn(np.random.default_rng([seed, 1, i, j]), (2 * n2 - 1, 2 * n3 - 1)) * scale).astype(C64)
    return {"t": t, "psi_rows": psi_rows, "x_true": x_true, "noise": noise, "sigma": sigma,
            "shape": (n1, n2, n3, nf)}


def power_start(n: int, seed: int = 0) -> np.ndarray:
    """CN(0,1) start vector of length n for a power iteration, rounded to
    complex64 so that it is exactly representable in both precisions."""
    return cn(np.random.default_rng([seed, 99]), n)
