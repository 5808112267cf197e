"""Dense-free FP64 evaluations for sizes whose dense matrix does not fit.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``toeplitz_apply_blocks``: row blocks of the Toeplitz matrix generated from
  the definition and multiplied by BLAS, never storing the whole matrix.
* ``select_circulant_apply``: rows of a row-selected circulant generated from
  the definition, one block at a time.
* ``kron_apply``: the Kronecker product applied by mode products with the
  dense FP64 factor matrices (eq. (7) structure); exact for the columns it is
  given, since columns are independent.
* ``*_fft64``: FFT-based evaluations with numpy.fft in complex128, following
  eq. (5) (cyclic convolution through the frequency domain) and its zero-padded
  non-circular version. Used only where even the block-dense forms are too
  slow; they are pinned against the dense forms in the oracle tests.
"""

from __future__ import annotations

import numpy as np

from . import dense

C128 = np.complex128


def toeplitz_apply_blocks(col, row, x, adjoint_dir: bool = False, block: int = 1024):
    """Toeplitz product with on-the-fly row blocks (x: (ncols, rows))."""
    col = np.asarray(col, dtype=C128)
    row = np.asarray(row, dtype=C128)
    x = np.asarray(x, dtype=C128)
    m, n = col.shape[0], row.shape[0]
    if adjoint_dir:
        # T^H[i, j] = conj(T[j, i]): a Toeplitz matrix with first column
        # conj(row) (diagonal conj(col[0])) and first row conj(col).
        new_col = np.conj(row).copy()
        new_col[0] = np.conj(col[0])
        return toeplitz_apply_blocks(new_col, np.conj(col), x, False, block)
    out = np.empty((x.shape[0], m), dtype=C128)
    for r0 in range(0, m, block):
        r1 = min(m, r0 + block)
        d = np.arange(r0, r1)[:, None] - np.arange(n)[None, :]
        tb = np.where(d >= 0, col[np.clip(d, 0, m - 1)], row[np.clip(-d, 0, n - 1)])
        out[:, r0:r1] = (tb @ x.T).T
    return out


def select_circulant_apply(c, rows, x, adjoint_dir: bool = False, block: int = 512):
    """Product with A = S_rows C(c) from rows built by the circulant
    definition C[i, j] = c[(i - j) mod n], block by block."""
    c = np.asarray(c, dtype=C128)
    rows = np.asarray(rows, dtype=np.int64)
    x = np.asarray(x, dtype=C128)
    n = c.shape[0]
    jj = np.arange(n)[None, :]
    if not adjoint_dir:
        out = np.empty((x.shape[0], rows.shape[0]), dtype=C128)
        for r0 in range(0, rows.shape[0], block):
            rb = rows[r0:r0 + block]
            a = c[(rb[:, None] - jj) % n]
            out[:, r0:r0 + rb.shape[0]] = (a @ x.T).T
        return out
    out = np.zeros((x.shape[0], n), dtype=C128)
    for r0 in range(0, rows.shape[0], block):
        rb = rows[r0:r0 + block]
        a = c[(rb[:, None] - jj) % n]
        out += (a.conj().T @ x[:, r0:r0 + rb.shape[0]].T).T
    return out


def kron_apply(factors, x, adjoint_dir: bool = False):
    """(A_1 (x) ... (x) A_d) x by mode products with dense factors.

    Each column of length prod(n_k) is viewed as a tensor of shape
    (n_1, ..., n_d) (first factor slowest, row-major); factor k multiplies
    along axis k. Adjoint: the Kronecker product of the factor adjoints.
    """
    mats = [np.asarray(f, dtype=C128) for f in factors]
    if adjoint_dir:
        mats = [m.conj().T for m in mats]
    x = np.asarray(x, dtype=C128)
    ncols = x.shape[0]
    dims_in = [m.shape[1] for m in mats]
    out = []
    for j in range(ncols):
        t = x[j].reshape(dims_in)
        for k, m in enumerate(mats):
            t = np.moveaxis(np.tensordot(m, t, axes=([1], [k])), 0, k)
        out.append(t.reshape(-1))
    return np.stack(out)


def kron_apply_int(factors, x, bits: int):
    """Integer Kronecker product by mode products in int64, then wrapped to a
    signed ``bits``-bit result. Exact only while no partial sum leaves int64:
    the caller bounds the inputs (checked here)."""
    mats = [np.asarray(f, dtype=np.int64) for f in factors]
    x = np.asarray(x, dtype=np.int64)
    bound = float(np.max(np.abs(x.astype(np.float64)))) if x.size else 0.0
    for m in mats:
        bound *= float(np.max(np.sum(np.abs(m), axis=1)))
    assert bound < 2.0 ** 62, "int64 partial sums could overflow"
    dims = [m.shape[1] for m in mats]
    out = []
    for j in range(x.shape[0]):
        t = x[j].reshape(dims)
        for k, m in enumerate(mats):
            t = np.moveaxis(np.tensordot(m, t, axes=([1], [k])), 0, k)
        out.append(t.reshape(-1))
    y = np.stack(out)
    if bits == 64:
        return y
    mod, half = 1 << bits, 1 << (bits - 1)
    return (((y + half) % mod) - half).astype(np.int32)


def circulant_apply_fft64(c, x, adjoint_dir: bool = False):
    """Eq. (5) in complex128: y = IFFT(FFT(c) * FFT(x)); adjoint uses conj."""
    c = np.asarray(c, dtype=C128)
    x = np.asarray(x, dtype=C128)
    ch = np.fft.fft(c)
    if adjoint_dir:
        ch = np.conj(ch)
    return np.fft.ifft(np.fft.fft(x, axis=1) * ch[None, :], axis=1)


def toeplitz_apply_fft64(col, row, x, adjoint_dir: bool = False, L: int | None = None):
    """Non-circular convolution by a zero-padded cyclic one of length
    L >= M + N - 1 (the embedding the paper describes for eq. (7))."""
    col = np.asarray(col, dtype=C128)
    row = np.asarray(row, dtype=C128)
    x = np.asarray(x, dtype=C128)
    m, n = col.shape[0], row.shape[0]
    if L is None:
        L = m + n - 1
    assert L >= m + n - 1
    g = np.zeros(L, dtype=C128)
    g[:m] = col
    g[L - n + 1:] = row[1:][::-1]
    gh = np.fft.fft(g)
    if adjoint_dir:
        xp = np.zeros((x.shape[0], L), dtype=C128)
        xp[:, :m] = x
        return np.fft.ifft(np.fft.fft(xp, axis=1) * np.conj(gh)[None, :], axis=1)[:, :n]
    xp = np.zeros((x.shape[0], L), dtype=C128)
    xp[:, :n] = x
    return np.fft.ifft(np.fft.fft(xp, axis=1) * gh[None, :], axis=1)[:, :m]


def toeplitz_fista_fft64(col, row, b, lam, L, iters, momentum=True, stop_tol=0.0, embed: int | None = None,
                         history: bool = False):
    """FISTA of ``fista.fista_op`` with the Toeplitz products done by
    ``toeplitz_apply_fft64``; for batches too large for dense products.
    ``embed``: the cyclic length of the products (any L >= M + N - 1 gives the
    same products; a power of two is faster for numpy.fft)."""
    from .fista import fista_op

    n = np.asarray(row).shape[0]
    return fista_op(lambda v: toeplitz_apply_fft64(col, row, v, L=embed),
                    lambda v: toeplitz_apply_fft64(col, row, v, adjoint_dir=True, L=embed),
                    n, b, lam, L, iters, momentum=momentum, stop_tol=stop_tol, history=history)


def select_circulant_fft64(c, rows):
    """(apply, adjoint) of A = S_rows C(c) through the FFT64 circulant product."""
    rows = np.asarray(rows, dtype=np.int64)
    n = np.asarray(c).shape[0]

    def apply(v):
        return circulant_apply_fft64(c, v)[:, rows]

    def adjoint(u):
        z = np.zeros((u.shape[0], n), dtype=C128)
        z[:, rows] = u
        return circulant_apply_fft64(c, z, adjoint_dir=True)

    return apply, adjoint


def ml_toeplitz_apply_fft64(n_levels, t, x, adjoint_dir: bool = False):
    """Multilevel Toeplitz product by a d-dimensional zero-padded cyclic
    convolution (numpy.fft.fftn in complex128)."""
    n_levels = [int(v) for v in n_levels]
    t = np.asarray(t, dtype=C128)
    x = np.asarray(x, dtype=C128)
    L = [2 * v - 1 for v in n_levels]
    g = np.zeros(L, dtype=C128)
    # offset o (index o + n - 1 in t) sits at position o mod L along each level
    src = np.indices(t.shape).reshape(len(L), -1)
    dst = tuple((src[l] - (n_levels[l] - 1)) % L[l] for l in range(len(L)))
    g[dst] = t.reshape(-1)
    gh = np.fft.fftn(g)
    if adjoint_dir:
        gh = np.conj(gh)
    out = []
    for j in range(x.shape[0]):
        xp = np.zeros(L, dtype=C128)
        xp[tuple(slice(0, v) for v in n_levels)] = x[j].reshape(n_levels)
        yp = np.fft.ifftn(np.fft.fftn(xp) * gh)
        out.append(yp[tuple(slice(0, v) for v in n_levels)].reshape(-1))
    return np.stack(out)


__all__ = [
    "toeplitz_apply_blocks",
    "select_circulant_apply",
    "kron_apply",
    "circulant_apply_fft64",
    "toeplitz_apply_fft64",
    "toeplitz_fista_fft64",
    "ml_toeplitz_apply_fft64",
    "dense",
]
