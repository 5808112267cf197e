"""Dense FP64 operator matrices, built entry by entry from their definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Index conventions are 0-based. A block of column vectors is an array of shape
``(ncols, rows)``; ``apply`` returns the block of results in the same layout.
"""

from __future__ import annotations

import numpy as np

C128 = np.complex128


def fourier(n: int) -> np.ndarray:
    """Unnormalised DFT matrix, F[i,k] = exp(-2 pi j i k / n).

    Eq. (1) (section "Motivation and significance"), read with 0-based indices
    and without normalisation: the exponent is reduced modulo n in integer
    arithmetic before scaling, so each entry is an exactly chosen root of unity.
    """
    i = np.arange(n, dtype=np.int64)
    e = np.outer(i, i) % n
    return np.exp(-2j * np.pi * e / n)


def diag(d) -> np.ndarray:
    """Diagonal matrix with d on its diagonal (Diag(h) in eq. (7))."""
    d = np.asarray(d, dtype=C128)
    return np.diag(d)


def circulant(c) -> np.ndarray:
    """Circulant matrix of the cyclic convolution y = c (*) x of eq. (5).

    The generator c is the first column: C[i,j] = c[(i - j) mod n].
    """
    c = np.asarray(c, dtype=C128)
    n = c.shape[0]
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return c[(i - j) % n]


def toeplitz(col, row) -> np.ndarray:
    """Toeplitz matrix of a non-circular convolution (section "General
    Matrix-free Representations").

    T[i,j] = col[i-j] for i >= j and row[j-i] for i < j, so T is M x N with
    M = len(col), N = len(row). col[0] defines the diagonal; row[0] is unused.
    """
    col = np.asarray(col, dtype=C128)
    row = np.asarray(row, dtype=C128)
    m, n = col.shape[0], row.shape[0]
    d = np.arange(m)[:, None] - np.arange(n)[None, :]          # d = i - j
    below = col[np.clip(d, 0, m - 1)]
    above = row[np.clip(-d, 0, n - 1)]
    return np.where(d >= 0, below, above)


def ml_toeplitz(n_levels, t) -> np.ndarray:
    """Multilevel Toeplitz matrix (block Toeplitz with Toeplitz blocks, the
    2-level structure of the blocks H_ij in eq. (7)).

    ``t`` has shape (2 n_1 - 1, ..., 2 n_d - 1) and holds the generator at
    offsets -(n_l - 1) .. (n_l - 1) along level l (offset o at index o + n_l - 1).
    Rows and columns use row-major multi-indices (last level fastest):
    T[(i_1..i_d), (j_1..j_d)] = t[i_1 - j_1, ..., i_d - j_d].
    """
    n_levels = [int(v) for v in n_levels]
    t = np.asarray(t, dtype=C128)
    assert t.shape == tuple(2 * v - 1 for v in n_levels)
    idx = np.unravel_index(np.arange(int(np.prod(n_levels))), n_levels)
    off = tuple(idx[l][:, None] - idx[l][None, :] + n_levels[l] - 1
                for l in range(len(n_levels)))
    return t[off]


def hadamard(n: int) -> np.ndarray:
    """Walsh-Hadamard matrix in natural (Sylvester) order, entries +-1,
    H[i,j] = (-1)^popcount(i AND j). The paper's text does not define it;
    this is the reading used throughout (n must be a power of two)."""
    assert n > 0 and n & (n - 1) == 0
    a = np.arange(n, dtype=np.int64)[:, None] & np.arange(n, dtype=np.int64)[None, :]
    parity = np.zeros_like(a)
    while a.any():                      # popcount(i AND j) mod 2, bit by bit
        parity ^= a & 1
        a = a >> 1
    return 1 - 2 * parity


def kron(*factors) -> np.ndarray:
    """Kronecker product, first factor slowest (eq. (7)):
    (A (x) B)[i_A m_B + i_B, j_A n_B + j_B] = A[i_A, j_A] B[i_B, j_B]."""
    out = np.asarray(factors[0])
    for f in factors[1:]:
        f = np.asarray(f)
        ma, na = out.shape
        mb, nb = f.shape
        res = np.empty((ma * mb, na * nb), dtype=np.result_type(out, f))
        for ia in range(ma):
            for ja in range(na):
                res[ia * mb:(ia + 1) * mb, ja * nb:(ja + 1) * nb] = out[ia, ja] * f
        out = res
    return out


def select_rows(n_in: int, rows) -> np.ndarray:
    """Row selection S with S[r, rows[r]] = 1 (the Partial operator of the
    compressed model in eq. (9))."""
    rows = np.asarray(rows, dtype=np.int64)
    s = np.zeros((rows.shape[0], n_in), dtype=C128)
    s[np.arange(rows.shape[0]), rows] = 1.0
    return s


def product(*terms) -> np.ndarray:
    """Matrix product t_1 t_2 ... t_k (Product class, applied right to left)."""
    out = np.asarray(terms[0], dtype=C128)
    for t in terms[1:]:
        out = out @ np.asarray(t, dtype=C128)
    return out


def sum_(*terms) -> np.ndarray:
    """Sum of equally shaped matrices."""
    out = np.asarray(terms[0], dtype=C128).copy()
    for t in terms[1:]:
        out = out + np.asarray(t, dtype=C128)
    return out


def blkdiag(*blocks) -> np.ndarray:
    """Block-diagonal arrangement (the BlkDiag of the compressed model)."""
    m = sum(b.shape[0] for b in blocks)
    n = sum(b.shape[1] for b in blocks)
    out = np.zeros((m, n), dtype=C128)
    r = c = 0
    for b in blocks:
        out[r:r + b.shape[0], c:c + b.shape[1]] = b
        r += b.shape[0]
        c += b.shape[1]
    return out


def blocks(grid) -> np.ndarray:
    """Block matrix [A_ij] (the block structure of the ultrasound model's H,
    section "Application to Ultrasonic Nondestructive Testing"): block (i, j)
    occupies rows roff_i .. roff_i + m_i and columns coff_j .. coff_j + n_j,
    with m_i the rows of the blocks of block row i and n_j the columns of the
    blocks of block column j."""
    grid = [[np.asarray(a, dtype=C128) for a in r] for r in grid]
    m_i = [r[0].shape[0] for r in grid]
    n_j = [a.shape[1] for a in grid[0]]
    for r in grid:
        assert [a.shape[1] for a in r] == n_j
        assert all(a.shape[0] == r[0].shape[0] for a in r)
    out = np.zeros((sum(m_i), sum(n_j)), dtype=C128)
    r0 = 0
    for i, r in enumerate(grid):
        c0 = 0
        for j, a in enumerate(r):
            out[r0:r0 + m_i[i], c0:c0 + n_j[j]] = a
            c0 += n_j[j]
        r0 += m_i[i]
    return out


def ml_toeplitz_rows(n_levels, t, rows) -> np.ndarray:
    """Rows ``rows`` of ``ml_toeplitz(n_levels, t)``, built from the same
    definition for those rows only (for operators too large to store)."""
    n_levels = [int(v) for v in n_levels]
    t = np.asarray(t, dtype=C128)
    ri = np.unravel_index(np.asarray(rows, dtype=np.int64), n_levels)
    cj = np.unravel_index(np.arange(int(np.prod(n_levels))), n_levels)
    off = tuple(ri[l][:, None] - cj[l][None, :] + n_levels[l] - 1 for l in range(len(n_levels)))
    return t[off]


def fourier_rows(n: int, rows) -> np.ndarray:
    """Selected rows of the DFT matrix of eq. (1): the blocks Phi of the
    compressed model, eq. (9)."""
    k = np.asarray(rows, dtype=np.int64)[:, None]
    j = np.arange(n)[None, :]
    return np.exp(-2j * np.pi * ((k * j) % n) / n)


def lfsr_sequence(order: int, taps: int, state: int, n: int | None = None) -> np.ndarray:
    """+-1 output of a linear feedback shift register (the generator of the
    LFSR circulant): bit i of the register holds s_{k+i}; each step outputs
    bit 0 (0 -> +1, 1 -> -1) and appends s_{k+order} = XOR of the register
    bits selected by taps. n defaults to 2^order - 1 values."""
    n = (1 << order) - 1 if n is None else n
    reg = [(state >> i) & 1 for i in range(order)]
    tap = [(taps >> i) & 1 for i in range(order)]
    out = np.empty(n, dtype=C128)
    for k in range(n):
        out[k] = -1.0 if reg[0] else 1.0
        new = 0
        for i in range(order):
            new ^= reg[i] & tap[i]
        reg = reg[1:] + [new]
    return out


def adjoint(a) -> np.ndarray:
    """Hermitian transpose, the matrix of the backward transform (eq. 4)."""
    return np.asarray(a).conj().T


def apply(a, x, adjoint_dir: bool = False) -> np.ndarray:
    """Dense product of eq. (2) on a block x of shape (ncols, rows).

    Forward: y = A x (eq. 3). Adjoint: y = A^H x (eq. 4). Complex inputs are
    upcast exactly to complex128.
    """
    a = np.asarray(a, dtype=C128)
    x = np.asarray(x, dtype=C128)
    m = a.conj().T if adjoint_dir else a
    return (m @ x.T).T


def apply_int(h, x, bits: int, adjoint_dir: bool = False) -> np.ndarray:
    """Exact integer product for integer-valued operators, wrapped to a signed
    ``bits``-bit result (arithmetic modulo 2^bits). Uses Python integers, so no
    intermediate overflows; the wrap is applied once at the end."""
    h = np.asarray(h, dtype=object)
    x = np.asarray(x, dtype=object)
    m = h.T if adjoint_dir else h
    y = (m.dot(x.T)).T
    mod = 1 << bits
    half = 1 << (bits - 1)
    f = np.vectorize(lambda v: ((int(v) + half) % mod) - half, otypes=[object])
    return f(y).astype(np.int64 if bits == 64 else np.int32)
